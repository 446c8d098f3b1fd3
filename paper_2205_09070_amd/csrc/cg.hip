// Block conjugate gradients on [y, z_1..z_P] (Section 2.5) for gfx950.
//
// Vector-block layout ("slab layout"): column 0 (y, or the first dense
// column) is a plain vector of ny = round_up(n, 32) doubles; columns
// 1..R-1 are packed in slabs of 32 columns, slab s being a row-major
// [n][32] array at offset ny + s*n*32.  Slab columns past R-1 are padding
// and stay zero.  A slab row is 256 bytes, i.e. two whole cache lines.
//
// SpMM (the hot loop): a 16-lane group handles one matrix row, lane j
// holding slab columns 2j and 2j+1 (one 16-byte load per gathered
// neighbour row), so a wavefront carries four rows at once.  The row's
// (column, value) pairs are loaded 16 at a time, one per lane, and
// broadcast inside each group of 16 lanes with a DPP row broadcast.
// Column 0 is gathered lane-parallel: each lane multiplies its own entry's
// value by y[col] and the 16 partial sums are reduced at the row's end.
// Rows are visited in a Morton order of the cell grid, each XCD taking a
// contiguous eighth of that order (workgroups are dealt to the 8 XCDs
// round-robin), which keeps the gathered rows in the XCD's own L2.
//
// Reductions are deterministic: every block writes one partial per column
// into part[column][block]; a small kernel sums each column's partials in
// a fixed order.  No atomics take part in any sum.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <climits>
#include <cmath>
#include <utility>
#include <vector>

#include "kernel_math.hpp"
#include "sdgp_internal.hpp"

namespace sdgp {

namespace {

constexpr int kT = 256;          // threads per block
constexpr int kTile = 16;        // rows per block tile (4 waves x 4 groups of 16 lanes)
constexpr int kSlab = 32;        // columns per slab
constexpr int kSC = kSlab + 1;   // LDS stride of per-column values (slab columns + column 0)
constexpr int kMaxNbs = 32768;   // SpMM blocks
constexpr int kMaxNbu = 8192;    // upper bound on the update kernels' grid (default: one resident round)
constexpr int kGS = 2;           // row-steps whose loads the update passes issue together
constexpr int64_t kUnionMinRows = 65536;  // union-list SpMM by default from this many rows

struct CgState {
  double* rz;       // [2][R] parity buffers of r.z (r.r unpreconditioned)
  double* rz0;      // [R] b^T M^{-1} b (b^T b unpreconditioned): SLQ weight
  int32_t* act;     // [2][R] active flags
  int32_t* failed;  // [R] p^T A p <= 0 met
  double* bnorm2;   // [R]
  double* rr_last;  // [R] |r|^2 at each column's last iteration
  int32_t* iters;   // [R]
  int32_t* done;    // [1] executed iterations once every column stopped
  int32_t* not_spd; // [1]
  int32_t* it;      // [1] iteration counter (advanced by k_cg_check)
  double* hist_a;   // [max_iter][R]
  double* hist_b;   // [max_iter][R]
};

struct CgArgs {
  int64_t n, ny;
  int R, ns;                  // columns, slabs
  const int64_t* row_ptr;
  const int32_t* col;
  const double* val;
  double *X, *Rr, *P, *Q, *V; // slab layout (V: M^{-1} b, may be null)
  const int32_t* sched;       // SpMM row order (may be null)
  const double* F;            // [n][n1] sorted bump values
  const double* Sinv;         // [n1][n1] (c I + F^T F)^{-1}
  int n1;
  int use_pc;                 // z = M^{-1} r, M = c I + F F^T
  int lowrank_op;             // operator K_core + F F^T (F F^T applied on the fly)
  double inv_c, sqrt_c;
  int nbs, nbu;               // blocks of the SpMM / update kernels
  int max_iter;
  double rtol2;               // column 0 (y, or every column of caller right-hand sides)
  double prtol2;              // probe columns 1 .. R-1
  double* s_part;             // [R][nbs] p.(A p) partials of the SpMM
  double* s_red;              // [R]
  double* u_part;             // [(1+n1) R][nbu]: r.r, then F^T r (row R + i R + c)
  double* u_red;              // [(1+n1) R]
  double* w_red;              // [(n1+1) R]: u = S^{-1} g (row i R + c), then g.u (row n1 R + c)
  double* p_part;             // [n1 R][nbu] F^T p (row i R + c)
  double* p_red;              // [n1 R]
  // 4-row union lists of the shared-gather SpMM: group q = schedule rows
  // 4q .. 4q+3; entries urp[q] .. urp[q+1]-1 hold the group's distinct
  // columns (ascending, ucol) and their 4 values (uval[4e + r] for row 4q+r,
  // 0 where that row lacks the column)
  const int64_t* urp;
  const int32_t* ucol;
  const double* uval;
  CgState st;
};

__device__ __forceinline__ bool stopped(const CgArgs& A) { return *A.st.done || *A.st.it >= A.max_iter; }

// The CG kernels read their arrays through pointers held in device memory
// (one argument block per member), which the compiler cannot prove to be
// global; these casts let it emit global (not flat) memory instructions.
#define GL __attribute__((address_space(1)))
typedef double dv2 __attribute__((ext_vector_type(2)));

// Slab vectors streamed through a pass (the SpMM output, the update passes'
// vectors): every element is touched once per pass and not again until the
// next pass, so these loads and stores carry the non-temporal hint.
__device__ __forceinline__ dv2 ld_s(const GL double* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const GL dv2*>(p));
}
__device__ __forceinline__ void st_s(GL double* p, dv2 v) {
  __builtin_nontemporal_store(v, reinterpret_cast<GL dv2*>(p));
}
struct Gv {
  const GL int64_t* row_ptr;
  const GL int32_t* col;
  const GL double* val;
  GL double *X, *Rr, *P, *Q, *V;
  const GL int32_t* sched;
  const GL double* F;
  GL double *s_part, *u_part, *p_part;
};
__device__ __forceinline__ Gv gview(const CgArgs& A) {
  Gv g;
  g.row_ptr = (const GL int64_t*)A.row_ptr;
  g.col = (const GL int32_t*)A.col;
  g.val = (const GL double*)A.val;
  g.X = (GL double*)A.X;
  g.Rr = (GL double*)A.Rr;
  g.P = (GL double*)A.P;
  g.Q = (GL double*)A.Q;
  g.V = (GL double*)A.V;
  g.sched = (const GL int32_t*)A.sched;
  g.F = (const GL double*)A.F;
  g.s_part = (GL double*)A.s_part;
  g.u_part = (GL double*)A.u_part;
  g.p_part = (GL double*)A.p_part;
  return g;
}

// ------------------------------------------------------------ SpMM core
template <int u>
__device__ __forceinline__ int bcast16_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x150 + u, 0xF, 0xF, false);  // row_newbcast:u
}
template <int u>
__device__ __forceinline__ double bcast16_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = bcast16_i<u>((int)(b & 0xffffffffll));
  const int hi = bcast16_i<u>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// 16 gathers of the calling lane's two slab columns, all issued before any
// product is summed; acc[0..7]: four accumulator pairs (entry u feeds pair
// u % 4).
template <int... us>
__device__ __forceinline__ void gather16(int cj, double vj, const GL double* __restrict__ Xs, int64_t ld,
                                         double* acc, std::integer_sequence<int, us...>) {
  double vv[16];
  dv2 xv[16];
  ((vv[us] = bcast16_d<us>(vj),
    xv[us] = *reinterpret_cast<const GL dv2*>(Xs + (int64_t)(uint32_t)bcast16_i<us>(cj) * ld)), ...);
#pragma unroll
  for (int u = 0; u < 16; u += 4) {
    acc[0] += vv[u] * xv[u].x;
    acc[1] += vv[u] * xv[u].y;
    acc[2] += vv[u + 1] * xv[u + 1].x;
    acc[3] += vv[u + 1] * xv[u + 1].y;
    acc[4] += vv[u + 2] * xv[u + 2].x;
    acc[5] += vv[u + 2] * xv[u + 2].y;
    acc[6] += vv[u + 3] * xv[u + 3].x;
    acc[7] += vv[u + 3] * xv[u + 3].y;
  }
}

// Row dot products of one matrix row (entries k0..k1) with the two slab
// columns of the calling lane: q = sum_k val[k] * Xs[col[k] * ld + {0, 1}],
// Xs pointing at the lane's first column.  With kY, yacc also receives the
// lane's share of sum_k val[k] * ycol[col[k]] (entries kb + j).  The next
// 16 (column, value) pairs are loaded while the current 16 gathers are in
// flight.  Every lane of the wavefront must call this together (DPP
// broadcasts); ``self`` is a valid row index used for the padding entries.
template <bool kY, bool kSlabs = true>
__device__ __forceinline__ void slab_row(int64_t k0, int64_t k1, int32_t self, const GL int32_t* __restrict__ col,
                                         const GL double* __restrict__ val, const GL double* __restrict__ Xs,
                                         int64_t ld, const GL double* __restrict__ ycol, dv2& q, double& yacc) {
  const int j = lane_id() & 15;
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int64_t kb = k0;
  bool in = kb + j < k1;
  int cj = in ? col[kb + j] : self;
  double vj = in ? val[kb + j] : 0.0;
  while (__any(kb < k1)) {
    const int64_t kn = kb + 16 + j;
    const bool inn = kn < k1;
    const int cn = inn ? col[kn] : self;
    const double vn = inn ? val[kn] : 0.0;
    if constexpr (kY) yacc += vj * ycol[cj];
    if constexpr (kSlabs) gather16(cj, vj, Xs, ld, acc, std::make_integer_sequence<int, 16>{});
    cj = cn;
    vj = vn;
    kb += 16;
  }
  q.x = (acc[0] + acc[2]) + (acc[4] + acc[6]);
  q.y = (acc[1] + acc[3]) + (acc[5] + acc[7]);
}

// Sum over the 16 lanes of a DPP row; lane 0 of the row holds the sum.
__device__ __forceinline__ double row16_sum(double v) {
  v += __shfl_xor(v, 8, 16);
  v += __shfl_xor(v, 4, 16);
  v += __shfl_xor(v, 2, 16);
  v += __shfl_xor(v, 1, 16);
  return v;
}

// Block sums of per-thread (2-column) values over the 16 row slots of a
// tile: red[(w*4+g)*32 + col] in LDS, thread t < 32 adds in fixed order.
__device__ __forceinline__ double tile_colsum(double* red, double v0, double v1) {
  const int lane = lane_id(), g = lane >> 4, j = lane & 15, w = threadIdx.x >> 6;
  __syncthreads();
  red[(w * 4 + g) * kSlab + 2 * j] = v0;
  red[(w * 4 + g) * kSlab + 2 * j + 1] = v1;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x < kSlab)
    for (int q = 0; q < kTile; ++q) s += red[q * kSlab + threadIdx.x];
  return s;
}

// Block sum of one value per thread (fixed order); valid in thread 0.
__device__ __forceinline__ double block_sum(double* red, double v) {
  __syncthreads();
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  return red[0];
}

// Q = A P, per-block partials of p.q.  kMode 1: slab 0 and column 0
// together (grid y = 1); kMode 2: slabs 1.. (grid y = ns - 1); kMode 0:
// column 0 only (no slabs).  With the factored operator A = K_core + F F^T
// this computes K_core P; the F F^T part is added by the update kernel.
template <int kMode>
__global__ __launch_bounds__(kT) void k_cg_spmm(const CgArgs* __restrict__ AA) {
  const CgArgs& A = AA[blockIdx.z];
  const Gv G = gview(A);
  if (stopped(A)) return;
  constexpr bool kY = kMode != 2;
  constexpr bool kSlabs = kMode != 0;
  __shared__ double red[kTile * kSlab];
  __shared__ double redy[kTile];
  const int lane = lane_id(), g = lane >> 4, j = lane & 15, w = threadIdx.x >> 6;
  const int s = kMode == 2 ? (int)blockIdx.y + 1 : 0;
  const int64_t n = A.n;
  const int64_t so = A.ny + (int64_t)s * n * kSlab + 2 * j;
  const GL double* Ps = G.P + so;
  GL double* Qs = G.Q + so;
  const int xcd = blockIdx.x & 7;
  const int64_t bi = blockIdx.x >> 3, nbx = gridDim.x >> 3;
  const int64_t nx = (n + 7) >> 3, lo = xcd * nx, hi = min(n, lo + nx);
  double pq0 = 0.0, pq1 = 0.0, pqy = 0.0;
  for (int64_t pb = lo + bi * kTile + w * 4; pb < hi; pb += nbx * kTile) {
    const int64_t p = pb + g;
    const bool live = p < hi;
    const int64_t a = live ? (G.sched ? (int64_t)G.sched[p] : p) : 0;
    const int64_t k0 = live ? G.row_ptr[a] : 0, k1 = live ? G.row_ptr[a + 1] : 0;
    dv2 q;
    double yacc = 0.0;
    slab_row<kY, kSlabs>(k0, k1, (int32_t)a, G.col, G.val, Ps, kSlab, G.P, q, yacc);
    if (kY) yacc = row16_sum(yacc);
    if (live) {
      if (kSlabs) {
        st_s(Qs + a * kSlab, q);
        const dv2 pv = *reinterpret_cast<const GL dv2*>(Ps + a * kSlab);
        pq0 += pv.x * q.x;
        pq1 += pv.y * q.y;
      }
      if (kY && j == 0) {
        G.Q[a] = yacc;
        pqy += G.P[a] * yacc;
      }
    }
  }
  if (kSlabs) {
    const double t = tile_colsum(red, pq0, pq1);
    if (threadIdx.x < kSlab) {
      const int rc = 1 + s * kSlab + threadIdx.x;
      if (rc < A.R) G.s_part[(int64_t)rc * A.nbs + blockIdx.x] = t;
    }
  }
  if (kY) {
    __syncthreads();
    if (j == 0) redy[w * 4 + g] = pqy;
    __syncthreads();
    if (threadIdx.x == 0) {
      double ty = 0.0;
      for (int q = 0; q < kTile; ++q) ty += redy[q];
      G.s_part[blockIdx.x] = ty;
    }
  }
}

// ------------------------------------------------------- union-list SpMM
// Lists of the shared-gather SpMM, built once per solve.  A group is four
// consecutive rows of the row schedule (the four rows one wavefront of the
// SpMM owns); its list is the merge of the four rows' ascending column lists.
// One thread per group; k_union_count writes the list lengths, k_union_fill
// (after a scan into urp) the columns and values.
__device__ __forceinline__ void union_head(int64_t n, int64_t p, const int64_t* __restrict__ rp,
                                           const int32_t* __restrict__ sched, int64_t& k, int64_t& e) {
  k = e = 0;
  if (p < n) {
    const int64_t a = sched ? (int64_t)sched[p] : p;
    k = rp[a];
    e = rp[a + 1];
  }
}
__device__ __forceinline__ int32_t head_col(int64_t k, int64_t e, const int32_t* __restrict__ col) {
  return k < e ? col[k] : INT32_MAX;
}
__global__ __launch_bounds__(256) void k_union_count(int64_t n, int64_t ng, const int64_t* __restrict__ rp,
                                                     const int32_t* __restrict__ col,
                                                     const int32_t* __restrict__ sched, int32_t* __restrict__ cnt) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= ng) return;
  int64_t k0, e0, k1, e1, k2, e2, k3, e3;
  union_head(n, 4 * q, rp, sched, k0, e0);
  union_head(n, 4 * q + 1, rp, sched, k1, e1);
  union_head(n, 4 * q + 2, rp, sched, k2, e2);
  union_head(n, 4 * q + 3, rp, sched, k3, e3);
  int32_t c = 0;
  for (;;) {
    const int32_t h0 = head_col(k0, e0, col), h1 = head_col(k1, e1, col);
    const int32_t h2 = head_col(k2, e2, col), h3 = head_col(k3, e3, col);
    const int32_t m = min(min(h0, h1), min(h2, h3));
    if (m == INT32_MAX) break;
    k0 += h0 == m;
    k1 += h1 == m;
    k2 += h2 == m;
    k3 += h3 == m;
    ++c;
  }
  cnt[q] = c;
}
__global__ __launch_bounds__(256) void k_union_fill(int64_t n, int64_t ng, const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ col, const double* __restrict__ val,
                                                    const int32_t* __restrict__ sched, const int64_t* __restrict__ urp,
                                                    int32_t* __restrict__ ucol, double* __restrict__ uval) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= ng) return;
  int64_t k0, e0, k1, e1, k2, e2, k3, e3;
  union_head(n, 4 * q, rp, sched, k0, e0);
  union_head(n, 4 * q + 1, rp, sched, k1, e1);
  union_head(n, 4 * q + 2, rp, sched, k2, e2);
  union_head(n, 4 * q + 3, rp, sched, k3, e3);
  const int64_t u0 = urp[q], u1 = urp[q + 1];
  for (int64_t u = u0; u < u1; ++u) {   // the merge yields exactly u1 - u0 entries (k_union_count)
    const int32_t h0 = head_col(k0, e0, col), h1 = head_col(k1, e1, col);
    const int32_t h2 = head_col(k2, e2, col), h3 = head_col(k3, e3, col);
    const int32_t m = min(min(h0, h1), min(h2, h3));
    if (m == INT32_MAX) break;
    ucol[u] = m;
    uval[4 * u + 0] = h0 == m ? val[k0++] : 0.0;
    uval[4 * u + 1] = h1 == m ? val[k1++] : 0.0;
    uval[4 * u + 2] = h2 == m ? val[k2++] : 0.0;
    uval[4 * u + 3] = h3 == m ? val[k3++] : 0.0;
  }
}

// One union entry for all four rows: the entry's gathered slab row (lane j:
// columns 2j, 2j+1), times each row's value (row-broadcast from the lane
// holding the entry), is added into the four rows' accumulators.
template <int u>
__device__ __forceinline__ void union_fma(const dv2& x, const double* vr, double (*acc)[2]) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double v = bcast16_d<u>(vr[r]);
    acc[r][0] += v * x.x;
    acc[r][1] += v * x.y;
  }
}
template <int... us>
__device__ __forceinline__ void union_batch(int cj, const double* vr, const GL double* __restrict__ Xs,
                                            double (*acc)[2], std::integer_sequence<int, us...>) {
  // all 16 gathers in flight before the arithmetic
  dv2 xv[16];
  ((xv[us] = *reinterpret_cast<const GL dv2*>(Xs + (int64_t)(uint32_t)bcast16_i<us>(cj) * kSlab)), ...);
  ((union_fma<us>(xv[us], vr, acc)), ...);
}

// Q = A P over the union lists, per-block partials of p.q as in k_cg_spmm.
// A wavefront owns the four rows of one group and walks the group's list 64
// entries at a time (one entry per lane); each 16-lane group takes 16 of
// them (row-broadcast of the entry's column and four values), so every
// listed neighbour row is gathered once for the four rows.  The four groups'
// partial sums are then added across the wavefront.  kMode 1: slab 0 and
// column 0 (grid y = 1); kMode 2: slabs 1.. (grid y = ns - 1).  Groups are
// dealt to the XCDs in contiguous runs (the XCD share rounded to whole
// groups); each wavefront loads the list bounds of its next group while it
// works on the current one.
template <int kMode>
__global__ __launch_bounds__(kT) void k_cg_spmm_u(const CgArgs* __restrict__ AA) {
  const CgArgs& A = AA[blockIdx.z];
  const Gv G = gview(A);
  if (stopped(A)) return;
  constexpr bool kY = kMode == 1;
  __shared__ double red[kTile * kSlab];
  __shared__ double redy[kTile];
  const GL int64_t* urp = (const GL int64_t*)A.urp;
  const GL int32_t* ucol = (const GL int32_t*)A.ucol;
  const GL dv2* uval = (const GL dv2*)A.uval;
  const int lane = lane_id(), g = lane >> 4, j = lane & 15, w = threadIdx.x >> 6;
  const int s = kMode == 2 ? (int)blockIdx.y + 1 : 0;
  const int64_t n = A.n;
  const int64_t so = A.ny + (int64_t)s * n * kSlab + 2 * j;
  const GL double* Ps = G.P + so;
  GL double* Qs = G.Q + so;
  const int xcd = blockIdx.x & 7;
  const int64_t bi = blockIdx.x >> 3, nbx = gridDim.x >> 3;
  const int64_t nx = (((n + 7) >> 3) + 3) & ~(int64_t)3, lo = xcd * nx, hi = min(n, lo + nx);
  double pq0 = 0.0, pq1 = 0.0, pqy = 0.0;
  const int64_t stride = nbx * kTile;
  int64_t pb = lo + bi * kTile + w * 4;
  // list bounds of the current group, those of the next one loaded a group ahead
  int64_t k0 = 0, k1 = 0;
  if (pb < hi) {
    k0 = urp[pb >> 2];
    k1 = urp[(pb >> 2) + 1];
  }
  for (; pb < hi; pb += stride) {
    const int64_t pn = pb + stride;
    int64_t k0n = 0, k1n = 0;
    if (pn < hi) {
      k0n = urp[pn >> 2];
      k1n = urp[(pn >> 2) + 1];
    }
    const int64_t p = pb + g;
    const bool live = p < hi;
    const int64_t a = live ? (G.sched ? (int64_t)G.sched[p] : p) : 0;
    const int32_t a0 = G.sched ? G.sched[pb] : (int32_t)pb;
    double acc[4][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    double ya[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t kb = k0; kb < k1; kb += 64) {     // uniform over the wavefront
      const int64_t k = kb + lane;
      const bool in = k < k1;
      const int cj = in ? ucol[k] : a0;
      double vr[4] = {0.0, 0.0, 0.0, 0.0};
      if (in) {
        const dv2 v01 = uval[2 * k], v23 = uval[2 * k + 1];
        vr[0] = v01.x;
        vr[1] = v01.y;
        vr[2] = v23.x;
        vr[3] = v23.y;
      }
      if (kY) {
        const double yv = G.P[cj];
#pragma unroll
        for (int r = 0; r < 4; ++r) ya[r] += vr[r] * yv;
      }
      union_batch(cj, vr, Ps, acc, std::make_integer_sequence<int, 16>{});
    }
    // the four 16-lane groups' partial sums (lanes j, j+16, j+32, j+48)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      acc[r][0] += __shfl_xor(acc[r][0], 16);
      acc[r][1] += __shfl_xor(acc[r][1], 16);
      acc[r][0] += __shfl_xor(acc[r][0], 32);
      acc[r][1] += __shfl_xor(acc[r][1], 32);
      if (kY)
        for (int o = 32; o > 0; o >>= 1) ya[r] += __shfl_xor(ya[r], o);
    }
    dv2 qv = {acc[0][0], acc[0][1]};
    double yacc = ya[0];
    if (g == 1) { qv = dv2{acc[1][0], acc[1][1]}; yacc = ya[1]; }
    if (g == 2) { qv = dv2{acc[2][0], acc[2][1]}; yacc = ya[2]; }
    if (g == 3) { qv = dv2{acc[3][0], acc[3][1]}; yacc = ya[3]; }
    if (live) {
      st_s(Qs + a * kSlab, qv);
      const dv2 pv = *reinterpret_cast<const GL dv2*>(Ps + a * kSlab);
      pq0 += pv.x * qv.x;
      pq1 += pv.y * qv.y;
      if (kY && j == 0) {
        G.Q[a] = yacc;
        pqy += G.P[a] * yacc;
      }
    }
    k0 = k0n;
    k1 = k1n;
  }
  const double t = tile_colsum(red, pq0, pq1);
  if (threadIdx.x < kSlab) {
    const int rc = 1 + s * kSlab + threadIdx.x;
    if (rc < A.R) G.s_part[(int64_t)rc * A.nbs + blockIdx.x] = t;
  }
  if (kY) {
    __syncthreads();
    if (j == 0) redy[w * 4 + g] = pqy;
    __syncthreads();
    if (threadIdx.x == 0) {
      double ty = 0.0;
      for (int q = 0; q < kTile; ++q) ty += redy[q];
      G.s_part[blockIdx.x] = ty;
    }
  }
}

// out[c] = sum_b part[c][b] in a fixed order (one 1024-thread block per
// column).  which: 0 SpMM partials, 1 update partials (r.r and F^T r),
// 2 F^T p partials.
constexpr int kSumT = 1024;
__global__ __launch_bounds__(kSumT) void k_cg_colsum(const CgArgs* __restrict__ AA, int which) {
  const CgArgs& A = AA[blockIdx.z];
  if (stopped(A)) return;
  const Gv G = gview(A);
  __shared__ double red[kSumT];
  const GL double* part;
  double* out;
  int nparts, ncols;
  if (which == 0) { part = G.s_part; out = A.s_red; nparts = A.nbs; ncols = A.R; }
  else if (which == 1) { part = G.u_part; out = A.u_red; nparts = A.nbu; ncols = (1 + (A.use_pc ? A.n1 : 0)) * A.R; }
  else { part = G.p_part; out = A.p_red; nparts = A.nbu; ncols = A.n1 * A.R; }
  const int c = blockIdx.x;
  if (c >= ncols) return;
  const GL double* pc = part + (int64_t)c * nparts;
  double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
  int b = threadIdx.x;
  for (; b + 3 * kSumT < nparts; b += 4 * kSumT) {
    v0 += pc[b];
    v1 += pc[b + kSumT];
    v2 += pc[b + 2 * kSumT];
    v3 += pc[b + 3 * kSumT];
  }
  for (; b < nparts; b += kSumT) v0 += pc[b];
  red[threadIdx.x] = (v0 + v1) + (v2 + v3);
  __syncthreads();
  for (int o = kSumT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

// Preconditioner coefficients per column (one 64-thread block per column):
// u = S^{-1} g with g = F^T r from u_red, and g.u, each sum in a fixed order.
__global__ __launch_bounds__(64) void k_cg_small_solve(const CgArgs* __restrict__ AA) {
  const CgArgs& A = AA[blockIdx.z];
  if (stopped(A)) return;
  const int rc = blockIdx.x;
  if (rc >= A.R) return;
  __shared__ double gs[64];
  __shared__ double gu[64];
  const int i = threadIdx.x;
  const int n1 = A.n1;
  gs[i] = i < n1 ? A.u_red[(int64_t)A.R + (int64_t)i * A.R + rc] : 0.0;
  __syncthreads();
  double u = 0.0;
  if (i < n1)
    for (int k = 0; k < n1; ++k) u += A.Sinv[i * n1 + k] * gs[k];
  if (i < n1) A.w_red[(int64_t)i * A.R + rc] = u;
  gu[i] = i < n1 ? gs[i] * u : 0.0;
  __syncthreads();
  if (i == 0) {
    double t = 0.0;
    for (int k = 0; k < n1; ++k) t += gu[k];
    A.w_red[(int64_t)n1 * A.R + rc] = t;
  }
}

// ------------------------------------------------------------ updates
// Per-thread column handling of the streaming kernels.  Slab blocks
// (blockIdx.y < ns): rows a = 16 t + 4 w + g of tiles t = blockIdx.x +
// k nbu, lane j holding slab columns 2j, 2j+1.  Column-0 blocks
// (blockIdx.y == ns): one row per thread, a = 256 t + threadIdx.x.

// ------------------------------------------------------------ F^T v
// Slab blocks accumulate F^T v (v = r, p or z: the n1 x 32 block of the
// slab's columns) on the FP64 matrix cores: per step the wavefront's four
// rows are the K = 4 dimension of v_mfma_f64_16x16x4f64 with
//   A[i][k] = F[a_k][16 mt + i]   (lane 16 k + i),
//   B[k][c] = v[a_k][2 c + par]   (lane 16 k + c; par = even / odd column),
// so lane (g, j) supplies exactly its own row's F value and its own two
// columns.  The 16 x 16 result keeps D[4 q + g][j] in lane (g, j),
// register q (checked on gfx950).  Column-0 blocks (one row per thread)
// accumulate in scalars.
typedef double d4 __attribute__((ext_vector_type(4)));

template <int NT>
__device__ __forceinline__ void ft_step(const double* f, double v0, double v1, d4 (*acc)[2]) {
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) {
    acc[mt][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[mt], v0, acc[mt][0], 0, 0, 0);
    acc[mt][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[mt], v1, acc[mt][1], 0, 0, 0);
  }
}

// F values of the calling lane for row a (a < 0: zeros): f[mt] = F[a][16 mt + j].
template <int NT>
__device__ __forceinline__ void load_f(const CgArgs& A, int64_t a, double* f) {
  const GL double* F = (const GL double*)A.F;
  const int j = lane_id() & 15;
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) {
    const int i = 16 * mt + j;
    f[mt] = (a >= 0 && i < A.n1) ? F[a * (int64_t)A.n1 + i] : 0.0;
  }
}

// sum_i F[a][i] w[i][cl] with the row's F values spread over the 16 lanes
// of the group (f from load_f) and w in LDS (stride kSlab).  Every lane of
// the wavefront must call this together (DPP broadcasts).
template <int H, int... us>
__device__ __forceinline__ double fdot16(double f, int n1i, const double* w, int cl,
                                         std::integer_sequence<int, us...>) {
  double s = 0.0;
  ((s += (H + us < n1i) ? bcast16_d<us>(f) * w[(H + us) * kSC + cl] : 0.0), ...);
  return s;
}
template <int NT>
__device__ __forceinline__ double frow_bc(const double* f, int n1, const double* w, int cl) {
  double s = 0.0;
  for (int mt = 0; mt < NT && 16 * mt < n1; ++mt) {
    if (mt == 0) s += fdot16<0>(f[0], n1, w, cl, std::make_integer_sequence<int, 16>{});
    else if (mt == 1) s += fdot16<16>(f[1], n1, w, cl, std::make_integer_sequence<int, 16>{});
    else if (mt == 2) s += fdot16<32>(f[2], n1, w, cl, std::make_integer_sequence<int, 16>{});
    else s += fdot16<48>(f[3], n1, w, cl, std::make_integer_sequence<int, 16>{});
  }
  return s;
}

// Block sums of the wavefronts' F^T v tiles into part rows base + i R + rc
// (slab blocks).  red: at least 4 * 512 doubles of LDS.
template <int NT>
__device__ void put_ft_partials(const CgArgs& A, double* red, d4 (*acc)[2], GL double* part, int64_t base) {
  const int lane = lane_id(), g = lane >> 4, j = lane & 15, w = threadIdx.x >> 6;
  const int s = blockIdx.y;
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) {
    if (16 * mt >= A.n1) continue;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      red[w * 512 + (4 * q + g) * kSlab + 2 * j] = acc[mt][0][q];
      red[w * 512 + (4 * q + g) * kSlab + 2 * j + 1] = acc[mt][1][q];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 512; e += kT) {
      const int i = 16 * mt + (e >> 5);
      const int rc = 1 + s * kSlab + (e & 31);
      const double t = red[e] + red[512 + e] + red[1024 + e] + red[1536 + e];
      if (i < A.n1 && rc < A.R) part[(base + (int64_t)i * A.R + rc) * A.nbu + blockIdx.x] = t;
    }
  }
}

// Column-0 block sums: v0 (when has0) into part row row0, and the scalar
// F^T v accumulators gy[i] into part rows base + i R (when hasg); wavefront
// sums by DPP butterflies, then the four wavefronts in LDS (fixed order).
template <int NI>
__device__ void put_y_partials(const CgArgs& A, double* red, bool has0, double v0, int64_t row0, bool hasg,
                               const double* gy, GL double* part, int64_t base) {
  constexpr int NV = (NI > 0 ? NI : 1) + 1;
  const int w = threadIdx.x >> 6, lane = lane_id();
  __syncthreads();
  if (has0) {
    const double t = wave_sum(v0);
    if (lane == 0) red[w * NV] = t;
  }
  if (hasg) {
#pragma unroll
    for (int i = 0; i < (NI > 0 ? NI : 1); ++i) {
      if (i >= A.n1) continue;
      const double t = wave_sum(gy[i]);
      if (lane == 0) red[w * NV + 1 + i] = t;
    }
  }
  __syncthreads();
  const int nv = hasg ? 1 + A.n1 : 1;
  for (int v = threadIdx.x; v < nv; v += kT) {
    if (v == 0 && !has0) continue;
    const double t = (red[v] + red[NV + v]) + (red[2 * NV + v] + red[3 * NV + v]);
    const int64_t row = v == 0 ? row0 : base + (int64_t)(v - 1) * A.R;
    part[row * A.nbu + blockIdx.x] = t;
  }
}

// F w for the wavefront's 16-row tile on the matrix cores (used with many
// bump functions, where the per-row broadcast products cost more): with
// rows base .. base+15 and K = 4 bump indices per instruction,
//   A[m][k] = F[base + m][4 s + k]   (lane 16 k + m),
//   B[k][c] = w[4 s + k][2 c + par]  (lane 16 k + c; w in LDS, stride kSlab),
// so D[4 q + g][j] (lane (g, j), register q) is the product for the row the
// lane owns at step q, even column (de) / odd column (dd).
template <int NS>
__device__ __forceinline__ void fw_tile(const GL double* __restrict__ F, int n1, int64_t n, int64_t base,
                                        const double* w, d4& de, d4& dd) {
  const int g = lane_id() >> 4, j = lane_id() & 15;
  const int64_t row = base + j;
  de = d4{0.0, 0.0, 0.0, 0.0};
  dd = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = 4 * s + g;
    const bool ok = i < n1;
    const double fa = (row < n && ok) ? F[row * n1 + i] : 0.0;
    const double b0 = ok ? w[i * kSC + 2 * j] : 0.0;
    const double b1 = ok ? w[i * kSC + 2 * j + 1] : 0.0;
    de = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, b0, de, 0, 0, 0);
    dd = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, b1, dd, 0, 0, 0);
  }
}
// fw_tile plus, when yfold, the column-0 product in lanes j == 0:
// dy[q] of lane (g, 0) = sum_i F[base + 4q + g][i] w[i][kSlab].
template <int NS>
__device__ __forceinline__ void fw_tile_y(const GL double* __restrict__ F, int n1, int64_t n, int64_t base,
                                          const double* w, bool yfold, d4& de, d4& dd, d4& dy) {
  const int g = lane_id() >> 4, j = lane_id() & 15;
  const int64_t row = base + j;
  de = d4{0.0, 0.0, 0.0, 0.0};
  dd = d4{0.0, 0.0, 0.0, 0.0};
  dy = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int i = 4 * s + g;
    const bool ok = i < n1;
    const double fa = (row < n && ok) ? F[row * n1 + i] : 0.0;
    const double b0 = ok ? w[i * kSC + 2 * j] : 0.0;
    const double b1 = ok ? w[i * kSC + 2 * j + 1] : 0.0;
    de = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, b0, de, 0, 0, 0);
    dd = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, b1, dd, 0, 0, 0);
    if (yfold) {
      const double by = (ok && j == 0) ? w[i * kSC + kSlab] : 0.0;
      dy = __builtin_amdgcn_mfma_f64_16x16x4f64(fa, by, dy, 0, 0, 0);
    }
  }
}
// Column-0 partials of a yfold block: v (nonzero in lanes j == 0 only) into
// part row row0, and the column-0 F^T tile accumulators acc_y (D[i][0] in
// lanes j == 0) into part rows base + i R.
template <int NT>
__device__ void put_yfold_partials(const CgArgs& A, double* red, bool has0, double v, int64_t row0, bool hasg,
                                   const d4* acc_y, GL double* part, int64_t base) {
  const int lane = lane_id(), g = lane >> 4, j = lane & 15, w = threadIdx.x >> 6;
  __syncthreads();
  if (j == 0) {
    red[w * 4 + g] = v;
    if (hasg) {
#pragma unroll
      for (int mt = 0; mt < NT; ++mt)
#pragma unroll
        for (int q = 0; q < 4; ++q) red[64 + w * 64 + 16 * mt + 4 * q + g] = acc_y[mt][q];
    }
  }
  __syncthreads();
  if (has0 && threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < 16; ++k) t += red[k];
    part[row0 * A.nbu + blockIdx.x] = t;
  }
  if (hasg)
    for (int i = threadIdx.x; i < A.n1; i += kT) {
      const double t = (red[64 + i] + red[128 + i]) + (red[192 + i] + red[256 + i]);
      part[(base + (int64_t)i * A.R) * A.nbu + blockIdx.x] = t;
    }
}

__device__ __forceinline__ double pick4(const d4& v, int q) {
  return q == 0 ? v[0] : (q == 1 ? v[1] : (q == 2 ? v[2] : v[3]));
}
// Slab blocks with 16-row wavefront tiles: block steps and the wavefront's
// first row at step k.
constexpr int kWaveRows = 16;
constexpr int kBlockRows = 4 * kWaveRows;
__device__ __forceinline__ int64_t tile_steps(const CgArgs& A) {
  const int64_t tiles = (A.n + kBlockRows - 1) / kBlockRows;
  return tiles > (int64_t)blockIdx.x ? (tiles - blockIdx.x + A.nbu - 1) / A.nbu : 0;
}
__device__ __forceinline__ int64_t wave_base(const CgArgs& A, int64_t k) {
  return (blockIdx.x + k * (int64_t)A.nbu) * kBlockRows + (threadIdx.x >> 6) * kWaveRows;
}

// Per-column scalars are computed once per block into LDS by the column's
// owner thread (slab blocks: thread cl < 32 for column 1 + 32 s + cl;
// column-0 blocks: thread 0); each thread then reads those of its own
// columns (cl = 2j, 2j+1, or cl = 0).
__device__ __forceinline__ bool is_ycol(const CgArgs& A) { return (int)blockIdx.y == A.ns; }
__device__ __forceinline__ int col_of(const CgArgs& A, bool ycol, int cl) {
  return (ycol || cl == kSlab) ? 0 : 1 + (int)blockIdx.y * kSlab + cl;   // cl == kSlab: column 0
}
__device__ __forceinline__ int my_cl(bool ycol) { return ycol ? 0 : 2 * (lane_id() & 15); }

// Row visited by step k of the calling thread (or -1 past the end).
__device__ __forceinline__ int64_t thread_row(const CgArgs& A, bool ycol, int64_t k) {
  if (ycol) {
    const int64_t a = (blockIdx.x + k * (int64_t)A.nbu) * kT + threadIdx.x;
    return a < A.n ? a : -1;
  }
  const int64_t t = blockIdx.x + k * (int64_t)A.nbu;
  const int64_t a = t * kTile + (threadIdx.x >> 6) * 4 + (lane_id() >> 4);
  return a < A.n ? a : -1;
}
// Steps of the calling block (uniform over the block).
__device__ __forceinline__ int64_t thread_steps(const CgArgs& A, bool ycol) {
  const int64_t per = ycol ? kT : kTile;
  const int64_t tiles = (A.n + per - 1) / per;
  return tiles > (int64_t)blockIdx.x ? (tiles - blockIdx.x + A.nbu - 1) / A.nbu : 0;
}
// Offset of the thread's (first) element in row a.
__device__ __forceinline__ int64_t elem(const CgArgs& A, bool ycol, int64_t a) {
  return ycol ? a : A.ny + (int64_t)blockIdx.y * A.n * kSlab + a * kSlab + 2 * (lane_id() & 15);
}

// u = S^{-1} g of column rc (from k_cg_small_solve) into us[i * kSC]
// (stride kSlab); returns g.u.
template <int NI>
__device__ __forceinline__ double coef_u(const CgArgs& A, int rc, double* us) {
  for (int i = 0; i < A.n1; ++i) us[i * kSC] = A.w_red[(int64_t)i * A.R + rc];
  return A.w_red[(int64_t)A.n1 * A.R + rc];
}

// sum_i F[a][i] w[i][0] for a column-0 thread's own row.
template <int NI>
__device__ __forceinline__ double frow_dot(const GL double* __restrict__ Fa, int n1, const double* w) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < (NI > 0 ? NI : 1); ++i)
    if (i < n1) s += Fa[i] * w[i * kSC];
  return s;
}

// A row's F values into registers: 16-byte loads when the row holds
// exactly NI (even) values, so its 16-byte alignment follows from F's.
template <int NI>
__device__ __forceinline__ void load_frow(const GL double* __restrict__ Fa, int n1, double* f) {
  if (NI > 0 && n1 == NI) {
#pragma unroll
    for (int i = 0; i < (NI > 0 ? NI : 2); i += 2) {
      const dv2 v = *reinterpret_cast<const GL dv2*>(Fa + i);
      f[i] = v.x;
      f[i + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int i = 0; i < (NI > 0 ? NI : 1); ++i) f[i] = i < n1 ? Fa[i] : 0.0;
  }
}
// sum_i f[i] w[i][.] (w in LDS, stride kSC); the order of frow_dot.
template <int NI>
__device__ __forceinline__ double freg_dot(const double* f, int n1, const double* w) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < (NI > 0 ? NI : 1); ++i)
    if (i < n1) s += f[i] * w[i * kSC];
  return s;
}

constexpr int kRed = 4 * 512;   // LDS doubles for the block reductions

// alpha = r.z / p.A p (p.A p = p.K_core p + |F^T p|^2 with the factored
// operator); r -= alpha A p; partials of r.r and F^T r.  The solution
// update x += alpha p is left to the p-update pass, which reads p anyway.
template <int NI, int FW>
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(NI <= 32 ? 3 : 1))) void k_cg_update_xr(const CgArgs* __restrict__ AA) {
  constexpr int NT = (NI + 15) / 16;
  const CgArgs& A = AA[blockIdx.z];
  const Gv G = gview(A);
  if (stopped(A)) return;
  __shared__ double red[kRed];
  __shared__ double s_alpha[kSC];
  __shared__ int s_act[kSC];
  __shared__ double s_gp[(NI > 0 ? NI : 1) * kSC];
  const int it = *A.st.it;
  const int par = it & 1;
  const bool ycol = FW == 0 && is_ycol(A);   // matrix-core launches have no column-0 blocks
  const bool lr = NI > 0 && A.lowrank_op;
  const bool pc = NI > 0 && A.use_pc;
  // matrix-core launches have no column-0 blocks: slab 0 also owns column 0
  const bool yfold = FW == 1 && !ycol && blockIdx.y == 0;
  if ((int)threadIdx.x < (ycol ? 1 : (yfold ? kSC : kSlab))) {
    const int cl = threadIdx.x;
    const int rc = col_of(A, ycol, cl);
    double alpha = 0.0;
    int act = 0;
    if (rc < A.R) {
      const bool was = A.st.act[par * A.R + rc] != 0;
      double d = A.s_red[rc];
      if (lr)
        for (int i = 0; i < A.n1; ++i) {
          const double gi = A.p_red[(int64_t)i * A.R + rc];
          s_gp[i * kSC + cl] = gi;
          d += gi * gi;
        }
      if (was) {
        if (d > 0.0 && isfinite(d)) {
          alpha = A.st.rz[par * A.R + rc] / d;
          act = 1;
        }
        if (blockIdx.x == 0) {
          A.st.hist_a[(int64_t)it * A.R + rc] = alpha;
          if (!act) {
            A.st.failed[rc] = 1;
            *A.st.not_spd = 1;
          }
        }
      }
    } else if (lr) {
      for (int i = 0; i < A.n1; ++i) s_gp[i * kSC + cl] = 0.0;
    }
    s_alpha[cl] = alpha;
    s_act[cl] = act;
  }
  __syncthreads();
  const int64_t steps = thread_steps(A, ycol);
  if (ycol) {
    const double al = s_alpha[0];
    double rr = 0.0;
    double gy[NI > 0 ? NI : 1];
#pragma unroll
    for (int i = 0; i < (NI > 0 ? NI : 1); ++i) gy[i] = 0.0;
    if (s_act[0])
      for (int64_t k = 0; k < steps; ++k) {
        const int64_t a = thread_row(A, true, k);
        if (a < 0) continue;
        double f[NI > 0 ? NI : 2];
        if (lr || pc) load_frow<NI>(G.F + a * (int64_t)A.n1, A.n1, f);
        double q = G.Q[a];
        if (lr) q += freg_dot<NI>(f, A.n1, s_gp);
        const double r = G.Rr[a] - al * q;
        G.Rr[a] = r;
        rr += r * r;
        if (pc) {
#pragma unroll
          for (int i = 0; i < (NI > 0 ? NI : 1); ++i)
            if (i < A.n1) gy[i] += f[i] * r;
        }
      }
    put_y_partials<NI>(A, red, true, rr, 0, pc, gy, G.u_part, A.R);
    return;
  }
  const int cl = my_cl(false);
  const double al0 = s_alpha[cl], al1 = s_alpha[cl + 1];
  const int jl = lane_id() & 15;
  const double aly = yfold ? s_alpha[kSlab] : 0.0;
  const bool acty = yfold && s_act[kSlab] != 0;
  const bool mine = s_act[cl] || s_act[cl + 1] || (acty && jl == 0);
  double rry = 0.0;
  d4 acc_y[NT > 0 ? NT : 1];
#pragma unroll
  for (int mt = 0; mt < (NT > 0 ? NT : 1); ++mt) acc_y[mt] = d4{0.0, 0.0, 0.0, 0.0};
  double rr0 = 0.0, rr1 = 0.0;
  d4 acc[NT > 0 ? NT : 1][2];
#pragma unroll
  for (int mt = 0; mt < (NT > 0 ? NT : 1); ++mt) acc[mt][0] = acc[mt][1] = d4{0.0, 0.0, 0.0, 0.0};
  if (FW == 1 && __any(mine)) {
    // F (F^T p) per 16-row wavefront tile on the matrix cores
    constexpr int NS = (NI + 3) / 4;
    const int g = lane_id() >> 4;
    const int64_t nst = tile_steps(A);
    for (int64_t k = 0; k < nst; ++k) {
      const int64_t base = wave_base(A, k);
      if (base >= A.n) break;                       // uniform over the wavefront
      d4 ce = {0.0, 0.0, 0.0, 0.0}, cd = {0.0, 0.0, 0.0, 0.0}, cy = {0.0, 0.0, 0.0, 0.0};
      if (NS > 0 && lr) fw_tile_y<NS>(G.F, A.n1, A.n, base, s_gp, yfold, ce, cd, cy);
      // row-steps in pairs: both steps' loads before either step's stores,
      // then the arithmetic in row-step order (as in the p-update pass)
#pragma unroll
      for (int h = 0; h < 4 / kGS; ++h) {
        int64_t ar[kGS];
        bool in[kGS], iny[kGS];
        dv2 qv[kGS], rv[kGS];
        double qyv[kGS], ryv[kGS];
        double f[kGS][NT > 0 ? NT : 1];
#pragma unroll
        for (int e = 0; e < kGS; ++e) {
          const int64_t a = base + 4 * (kGS * h + e) + g;
          ar[e] = a;
          in[e] = a < A.n;
          iny[e] = acty && jl == 0 && in[e];        // column 0 of row a
          qyv[e] = iny[e] ? G.Q[a] : 0.0;
          ryv[e] = iny[e] ? G.Rr[a] : 0.0;
          qv[e] = rv[e] = dv2{0.0, 0.0};
          if (in[e]) {
            const int64_t o = elem(A, false, a);
            qv[e] = ld_s(G.Q + o);
            rv[e] = ld_s(G.Rr + o);
          }
          if (NT > 0 && pc) load_f<NT>(A, in[e] ? a : -1, f[e]);
        }
#pragma unroll
        for (int e = 0; e < kGS; ++e) {
          const int st = kGS * h + e;
          const int64_t a = ar[e];
          double ry = 0.0;
          if (iny[e]) {
            const double qy = qyv[e] + pick4(cy, st);
            ry = ryv[e] - aly * qy;
            G.Rr[a] = ry;
            rry += ry * ry;
          }
          dv2 r = {0.0, 0.0};
          if (in[e]) {
            const int64_t o = elem(A, false, a);
            dv2 q = qv[e];
            r = rv[e];
            q.x += pick4(ce, st);
            q.y += pick4(cd, st);
            r.x -= al0 * q.x;
            r.y -= al1 * q.y;
            st_s(G.Rr + o, r);
            rr0 += r.x * r.x;
            rr1 += r.y * r.y;
          }
          if (NT > 0 && pc) {
            ft_step<NT>(f[e], r.x, r.y, acc);
            if (yfold) {
#pragma unroll
              for (int mt = 0; mt < NT; ++mt)
                acc_y[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[e][mt], ry, acc_y[mt], 0, 0, 0);
            }
          }
        }
      }
    }
  } else if (FW == 0 && __any(mine)) {
    for (int64_t k = 0; k < steps; ++k) {
      const int64_t a = thread_row(A, false, k);
      double f[NT > 0 ? NT : 1];
      if (NT > 0) load_f<NT>(A, a, f);
      double c0 = 0.0, c1 = 0.0;
      if (lr) {
        c0 = frow_bc<NT>(f, A.n1, s_gp, cl);
        c1 = frow_bc<NT>(f, A.n1, s_gp, cl + 1);
      }
      dv2 r = {0.0, 0.0};
      if (a >= 0) {
        const int64_t o = elem(A, false, a);
        dv2 q = ld_s(G.Q + o);
        r = ld_s(G.Rr + o);
        q.x += c0;
        q.y += c1;
        r.x -= al0 * q.x;
        r.y -= al1 * q.y;
        st_s(G.Rr + o, r);
        rr0 += r.x * r.x;
        rr1 += r.y * r.y;
      }
      if (NT > 0 && pc) ft_step<NT>(f, r.x, r.y, acc);
    }
  }
  const double t = tile_colsum(red, rr0, rr1);
  if (threadIdx.x < kSlab) {
    const int rc = 1 + (int)blockIdx.y * kSlab + (int)threadIdx.x;
    if (rc < A.R) G.u_part[(int64_t)rc * A.nbu + blockIdx.x] = t;
  }
  if (NT > 0 && pc) put_ft_partials<NT>(A, red, acc, G.u_part, A.R);
  if (yfold) put_yfold_partials<(NT > 0 ? NT : 1)>(A, red, true, rry, 0, NT > 0 && pc, acc_y, G.u_part, A.R);
}

// x += alpha p (with this iteration's p, before it is replaced);
// beta = r.z_new / r.z; convergence on |r|; p = z + beta p with
// z = M^{-1} r = (r - F u) / c formed on the fly (r.z_new = (r.r - g.u)/c,
// g = F^T r, u = (cI + F^T F)^{-1} g).  With the factored operator also
// the partials of F^T p for the next iteration.
template <int NI, int FW>
__global__ __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(NI <= 32 ? 3 : 1))) void k_cg_update_p(const CgArgs* __restrict__ AA) {
  constexpr int NT = (NI + 15) / 16;
  const CgArgs& A = AA[blockIdx.z];
  const Gv G = gview(A);
  if (stopped(A)) return;
  __shared__ double red[kRed];
  __shared__ double s_beta[kSC];
  __shared__ int s_cont[kSC];
  __shared__ double s_alpha[kSC];
  __shared__ int s_xa[kSC];
  __shared__ double s_u[(NI > 0 ? NI : 1) * kSC];
  const int it = *A.st.it;
  const int par = it & 1, nxt = par ^ 1;
  const bool ycol = FW == 0 && is_ycol(A);   // matrix-core launches have no column-0 blocks
  const bool lr = NI > 0 && A.lowrank_op;
  const bool pc = NI > 0 && A.use_pc;
  // matrix-core launches have no column-0 blocks: slab 0 also owns column 0
  const bool yfold = FW == 1 && !ycol && blockIdx.y == 0;
  if ((int)threadIdx.x < (ycol ? 1 : (yfold ? kSC : kSlab))) {
    const int cl = threadIdx.x;
    const int rc = col_of(A, ycol, cl);
    double beta = 0.0, alpha = 0.0;
    int cont = 0, xa = 0;
    if (rc < A.R) {
      const double rr_new = A.u_red[rc];
      const double rz_new = pc ? (rr_new - coef_u<NI>(A, rc, s_u + cl)) * A.inv_c : rr_new;
      const bool act = A.st.act[par * A.R + rc] != 0 && A.st.failed[rc] == 0;
      const double rz_old = A.st.rz[par * A.R + rc];
      if (act) {
        alpha = A.st.hist_a[(int64_t)it * A.R + rc];
        xa = 1;
        beta = rz_new / rz_old;
        cont = !(rr_new <= (rc == 0 ? A.rtol2 : A.prtol2) * A.st.bnorm2[rc]) ? 1 : 0;
      }
      if (blockIdx.x == 0) {
        A.st.rz[nxt * A.R + rc] = act ? rz_new : rz_old;
        A.st.act[nxt * A.R + rc] = cont;
        if (act) {
          A.st.hist_b[(int64_t)it * A.R + rc] = beta;
          A.st.iters[rc] += 1;
          A.st.rr_last[rc] = rr_new;
        }
      }
    } else if (pc) {
      for (int i = 0; i < A.n1; ++i) s_u[i * kSC + cl] = 0.0;
    }
    s_beta[cl] = beta;
    s_cont[cl] = cont;
    s_alpha[cl] = alpha;
    s_xa[cl] = xa;
  }
  __syncthreads();
  const int64_t steps = thread_steps(A, ycol);
  if (ycol) {
    const double be = s_beta[0];
    double gy[NI > 0 ? NI : 1];
#pragma unroll
    for (int i = 0; i < (NI > 0 ? NI : 1); ++i) gy[i] = 0.0;
    const bool cont = s_cont[0] != 0;
    const double al = s_alpha[0];
    if (s_xa[0])
      for (int64_t k = 0; k < steps; ++k) {
        const int64_t a = thread_row(A, true, k);
        if (a < 0) continue;
        const double p_old = G.P[a];
        G.X[a] += al * p_old;
        if (!cont) continue;
        double f[NI > 0 ? NI : 2];
        if (lr || pc) load_frow<NI>(G.F + a * (int64_t)A.n1, A.n1, f);
        const double r = G.Rr[a];
        const double z = pc ? (r - freg_dot<NI>(f, A.n1, s_u)) * A.inv_c : r;
        const double p = z + be * p_old;
        G.P[a] = p;
        if (lr) {
#pragma unroll
          for (int i = 0; i < (NI > 0 ? NI : 1); ++i)
            if (i < A.n1) gy[i] += f[i] * p;
        }
      }
    if (lr) put_y_partials<NI>(A, red, false, 0.0, 0, true, gy, G.p_part, 0);
    return;
  }
  const int cl = my_cl(false);
  const double be0 = s_beta[cl], be1 = s_beta[cl + 1];
  const bool c0 = s_cont[cl] != 0, c1 = s_cont[cl + 1] != 0;
  const double al0 = s_alpha[cl], al1 = s_alpha[cl + 1];
  const bool xa = s_xa[cl] || s_xa[cl + 1];
  const int jl = lane_id() & 15;
  const double bey = yfold ? s_beta[kSlab] : 0.0;
  const bool cy = yfold && s_cont[kSlab] != 0;
  const double aly = yfold ? s_alpha[kSlab] : 0.0;
  const bool xay = yfold && s_xa[kSlab] != 0;
  d4 acc_y[NT > 0 ? NT : 1];
#pragma unroll
  for (int mt = 0; mt < (NT > 0 ? NT : 1); ++mt) acc_y[mt] = d4{0.0, 0.0, 0.0, 0.0};
  d4 acc[NT > 0 ? NT : 1][2];
#pragma unroll
  for (int mt = 0; mt < (NT > 0 ? NT : 1); ++mt) acc[mt][0] = acc[mt][1] = d4{0.0, 0.0, 0.0, 0.0};
  if (FW == 1 && __any(xa || (xay && jl == 0))) {
    // F u per 16-row wavefront tile on the matrix cores
    constexpr int NS = (NI + 3) / 4;
    const int g = lane_id() >> 4;
    const int64_t nst = tile_steps(A);
    for (int64_t k = 0; k < nst; ++k) {
      const int64_t base = wave_base(A, k);
      if (base >= A.n) break;                       // uniform over the wavefront
      d4 ue = {0.0, 0.0, 0.0, 0.0}, ud = {0.0, 0.0, 0.0, 0.0}, uy = {0.0, 0.0, 0.0, 0.0};
      if (NS > 0 && pc) fw_tile_y<NS>(G.F, A.n1, A.n, base, s_u, yfold, ue, ud, uy);
      // row-steps in pairs: both steps' loads are issued before either
      // step's stores (the compiler cannot reorder them itself, not knowing
      // that the rows differ), then the arithmetic in row-step order
#pragma unroll
      for (int h = 0; h < 4 / kGS; ++h) {
        int64_t ar[kGS];
        bool in[kGS], iny[kGS];
        dv2 rv[kGS], pv[kGS], xv[kGS];
        double pyv[kGS], xyv[kGS], ryv[kGS];
        double f[kGS][NT > 0 ? NT : 1];
#pragma unroll
        for (int e = 0; e < kGS; ++e) {
          const int64_t a = base + 4 * (kGS * h + e) + g;
          ar[e] = a;
          in[e] = a < A.n;
          iny[e] = yfold && jl == 0 && in[e];       // column 0 of row a
          pyv[e] = iny[e] ? G.P[a] : 0.0;
          xyv[e] = (iny[e] && xay) ? G.X[a] : 0.0;
          ryv[e] = (iny[e] && cy) ? G.Rr[a] : 0.0;
          rv[e] = pv[e] = xv[e] = dv2{0.0, 0.0};
          if (in[e]) {
            const int64_t o = elem(A, false, a);
            rv[e] = ld_s(G.Rr + o);
            pv[e] = ld_s(G.P + o);
            if (xa) xv[e] = ld_s(G.X + o);
          }
          if (NT > 0 && lr) load_f<NT>(A, in[e] ? a : -1, f[e]);
        }
#pragma unroll
        for (int e = 0; e < kGS; ++e) {
          const int st = kGS * h + e;
          const int64_t a = ar[e];
          double py = 0.0;
          if (iny[e]) {
            py = pyv[e];
            if (xay) G.X[a] = xyv[e] + aly * py;
            if (cy) {
              const double zy = pc ? (ryv[e] - pick4(uy, st)) * A.inv_c : ryv[e];
              py = zy + bey * py;
              G.P[a] = py;
            }
          }
          dv2 p = {0.0, 0.0};
          if (in[e]) {
            const int64_t o = elem(A, false, a);
            const dv2 r = rv[e];
            p = pv[e];
            if (xa) {
              dv2 x = xv[e];
              x.x += al0 * p.x;
              x.y += al1 * p.y;
              st_s(G.X + o, x);
            }
            const double z0 = pc ? (r.x - pick4(ue, st)) * A.inv_c : r.x;
            const double z1 = pc ? (r.y - pick4(ud, st)) * A.inv_c : r.y;
            if (c0) p.x = z0 + be0 * p.x;
            if (c1) p.y = z1 + be1 * p.y;
            st_s(G.P + o, p);
          }
          if (NT > 0 && lr) {
            ft_step<NT>(f[e], p.x, p.y, acc);
            if (yfold) {
#pragma unroll
              for (int mt = 0; mt < NT; ++mt)
                acc_y[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[e][mt], py, acc_y[mt], 0, 0, 0);
            }
          }
        }
      }
    }
  } else if (FW == 0 && __any(xa)) {
    for (int64_t k = 0; k < steps; ++k) {
      const int64_t a = thread_row(A, false, k);
      double f[NT > 0 ? NT : 1];
      if (NT > 0) load_f<NT>(A, a, f);
      double u0 = 0.0, u1 = 0.0;
      if (pc) {
        u0 = frow_bc<NT>(f, A.n1, s_u, cl);
        u1 = frow_bc<NT>(f, A.n1, s_u, cl + 1);
      }
      dv2 p = {0.0, 0.0};
      if (a >= 0) {
        const int64_t o = elem(A, false, a);
        const dv2 r = ld_s(G.Rr + o);
        p = ld_s(G.P + o);
        if (xa) {
          dv2 x = ld_s(G.X + o);
          x.x += al0 * p.x;
          x.y += al1 * p.y;
          st_s(G.X + o, x);
        }
        const double z0 = pc ? (r.x - u0) * A.inv_c : r.x;
        const double z1 = pc ? (r.y - u1) * A.inv_c : r.y;
        if (c0) p.x = z0 + be0 * p.x;
        if (c1) p.y = z1 + be1 * p.y;
        st_s(G.P + o, p);
      }
      if (NT > 0 && lr) ft_step<NT>(f, p.x, p.y, acc);
    }
  }
  if (NT > 0 && lr) put_ft_partials<NT>(A, red, acc, G.p_part, 0);
  if (yfold && NT > 0 && lr) put_yfold_partials<(NT > 0 ? NT : 1)>(A, red, false, 0.0, 0, true, acc_y, G.p_part, 0);
}

// Records the executed iteration count in done when no column is active
// and advances the iteration counter (one block per member).
__global__ void k_cg_check(const CgArgs* __restrict__ AA) {
  const CgArgs& A = AA[blockIdx.z];
  const Gv G = gview(A);
  if (stopped(A)) return;
  const int it = *A.st.it;
  const int nxt = (it & 1) ^ 1;
  __shared__ int left;
  if (threadIdx.x == 0) left = 0;
  __syncthreads();
  int mine = 0;
  for (int r = threadIdx.x; r < A.R; r += blockDim.x) mine |= A.st.act[nxt * A.R + r];
  if (mine) atomicOr(&left, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (!left) *A.st.done = it + 1;
    *A.st.it = it + 1;
  }
}

// ------------------------------------------------------------ start
// x = 0, r = b, p = 0 over the whole slab layout (padding included).
// Column 0 is y (or the first dense column); probe p (column 1+p) is the
// Rademacher vector w_p of caller row perm[a], or with the preconditioner
// sqrt(c) w_p + F v_p (v_p: n1 Rademacher signs), whose covariance is M.
__global__ void k_cg_start(const CgArgs* __restrict__ AA, const double* __restrict__ ys,
                           const int32_t* __restrict__ perm, int kind, uint64_t seed,
                           const double* __restrict__ dense) {
  const CgArgs& A = AA[blockIdx.z];
  const Gv G = gview(A);
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t n = A.n;
  const int64_t tot = A.ny + (int64_t)A.ns * n * kSlab;
  if (idx >= tot) return;
  int64_t a;
  int rc;
  if (idx < A.ny) {
    a = idx;
    rc = 0;
  } else {
    const int64_t t = idx - A.ny;
    const int64_t s = t / (n * kSlab);
    const int64_t rem = t - s * n * kSlab;
    a = rem >> 5;
    rc = 1 + (int)(s * kSlab) + (int)(rem & 31);
  }
  double b = 0.0;
  if (a < n && rc < A.R) {
    if (kind == PK_DENSE) {
      b = dense[a * A.R + rc];
    } else if (rc == 0) {
      b = ys[a];
    } else if (kind == PK_IDENTITY) {
      b = (perm[a] == rc - 1) ? 1.0 : 0.0;
    } else {
      const uint64_t pbase = (uint64_t)(rc - 1) << 32;
      b = (splitmix64_at(seed, pbase + (uint64_t)perm[a] + 1ull) >> 63) ? -1.0 : 1.0;
      if (A.use_pc) {
        double fv = 0.0;
        const GL double* Fa = G.F + a * (int64_t)A.n1;
        for (int i = 0; i < A.n1; ++i) {
          const double v = (splitmix64_at(seed, pbase + 0xFFFFFFFFull - (uint64_t)i) >> 63) ? -1.0 : 1.0;
          fv += Fa[i] * v;
        }
        b = A.sqrt_c * b + fv;
      }
    }
  }
  G.X[idx] = 0.0;
  G.Rr[idx] = b;
  G.P[idx] = 0.0;
}

// Partials of b.b and F^T b.
template <int NI>
__global__ __launch_bounds__(kT) void k_cg_norm(const CgArgs* __restrict__ AA) {
  constexpr int NT = (NI + 15) / 16;
  const CgArgs& A = AA[blockIdx.z];
  const Gv G = gview(A);
  __shared__ double red[kRed];
  const bool ycol = is_ycol(A);
  const bool pc = NI > 0 && A.use_pc;
  const int64_t steps = thread_steps(A, ycol);
  if (ycol) {
    double rr = 0.0;
    double gy[NI > 0 ? NI : 1];
#pragma unroll
    for (int i = 0; i < (NI > 0 ? NI : 1); ++i) gy[i] = 0.0;
    for (int64_t k = 0; k < steps; ++k) {
      const int64_t a = thread_row(A, true, k);
      if (a < 0) continue;
      const double r = G.Rr[a];
      rr += r * r;
      if (pc) {
        const GL double* Fa = G.F + a * (int64_t)A.n1;
#pragma unroll
        for (int i = 0; i < (NI > 0 ? NI : 1); ++i)
          if (i < A.n1) gy[i] += Fa[i] * r;
      }
    }
    put_y_partials<NI>(A, red, true, rr, 0, pc, gy, G.u_part, A.R);
    return;
  }
  double rr0 = 0.0, rr1 = 0.0;
  d4 acc[NT > 0 ? NT : 1][2];
#pragma unroll
  for (int mt = 0; mt < (NT > 0 ? NT : 1); ++mt) acc[mt][0] = acc[mt][1] = d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t k = 0; k < steps; ++k) {
    const int64_t a = thread_row(A, false, k);
    dv2 r = {0.0, 0.0};
    if (a >= 0) {
      r = *reinterpret_cast<const GL dv2*>(G.Rr + elem(A, false, a));
      rr0 += r.x * r.x;
      rr1 += r.y * r.y;
    }
    if (NT > 0 && pc) {
      double f[NT > 0 ? NT : 1];
      load_f<NT>(A, a, f);
      ft_step<NT>(f, r.x, r.y, acc);
    }
  }
  const double t = tile_colsum(red, rr0, rr1);
  if (threadIdx.x < kSlab) {
    const int rc = 1 + (int)blockIdx.y * kSlab + (int)threadIdx.x;
    if (rc < A.R) G.u_part[(int64_t)rc * A.nbu + blockIdx.x] = t;
  }
  if (NT > 0 && pc) put_ft_partials<NT>(A, red, acc, G.u_part, A.R);
}

// Initial state: p = z0 = M^{-1} b (b when unpreconditioned), V = z0,
// rz0 = b.z0, bnorm2 = b.b; with the factored operator the partials of
// F^T p.
template <int NI>
__global__ __launch_bounds__(kT) void k_cg_init_fin(const CgArgs* __restrict__ AA) {
  constexpr int NT = (NI + 15) / 16;
  const CgArgs& A = AA[blockIdx.z];
  const Gv G = gview(A);
  __shared__ double red[kRed];
  __shared__ double s_u[(NI > 0 ? NI : 1) * kSC];
  const bool ycol = is_ycol(A);
  const bool lr = NI > 0 && A.lowrank_op;
  const bool pc = NI > 0 && A.use_pc;
  if ((int)threadIdx.x < (ycol ? 1 : kSlab)) {
    const int cl = threadIdx.x;
    const int rc = col_of(A, ycol, cl);
    if (rc < A.R) {
      const double bb = A.u_red[rc];
      const double rz0 = pc ? (bb - coef_u<NI>(A, rc, s_u + cl)) * A.inv_c : bb;
      if (blockIdx.x == 0) {
        A.st.bnorm2[rc] = bb;
        A.st.rr_last[rc] = bb;
        A.st.rz[rc] = rz0;
        A.st.rz[A.R + rc] = rz0;
        A.st.rz0[rc] = rz0;
        A.st.act[rc] = bb > 0.0 ? 1 : 0;
        A.st.act[A.R + rc] = 0;
        A.st.failed[rc] = 0;
        A.st.iters[rc] = 0;
      }
    } else if (pc) {
      for (int i = 0; i < A.n1; ++i) s_u[i * kSC + cl] = 0.0;
    }
  }
  __syncthreads();
  const int64_t steps = thread_steps(A, ycol);
  if (ycol) {
    double gy[NI > 0 ? NI : 1];
#pragma unroll
    for (int i = 0; i < (NI > 0 ? NI : 1); ++i) gy[i] = 0.0;
    for (int64_t k = 0; k < steps; ++k) {
      const int64_t a = thread_row(A, true, k);
      if (a < 0) continue;
      const GL double* Fa = G.F + a * (int64_t)A.n1;
      const double r = G.Rr[a];
      const double z = pc ? (r - frow_dot<NI>(Fa, A.n1, s_u)) * A.inv_c : r;
      G.P[a] = z;
      if (G.V) G.V[a] = z;
      if (lr) {
#pragma unroll
        for (int i = 0; i < (NI > 0 ? NI : 1); ++i)
          if (i < A.n1) gy[i] += Fa[i] * z;
      }
    }
    if (lr) put_y_partials<NI>(A, red, false, 0.0, 0, true, gy, G.p_part, 0);
    return;
  }
  const int cl = my_cl(false);
  d4 acc[NT > 0 ? NT : 1][2];
#pragma unroll
  for (int mt = 0; mt < (NT > 0 ? NT : 1); ++mt) acc[mt][0] = acc[mt][1] = d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t k = 0; k < steps; ++k) {
    const int64_t a = thread_row(A, false, k);
    double f[NT > 0 ? NT : 1];
    if (NT > 0) load_f<NT>(A, a, f);
    double u0 = 0.0, u1 = 0.0;
    if (pc) {
      u0 = frow_bc<NT>(f, A.n1, s_u, cl);
      u1 = frow_bc<NT>(f, A.n1, s_u, cl + 1);
    }
    dv2 z = {0.0, 0.0};
    if (a >= 0) {
      const int64_t o = elem(A, false, a);
      const dv2 r = *reinterpret_cast<const GL dv2*>(G.Rr + o);
      z.x = pc ? (r.x - u0) * A.inv_c : r.x;
      z.y = pc ? (r.y - u1) * A.inv_c : r.y;
      *reinterpret_cast<GL dv2*>(G.P + o) = z;
      if (G.V) *reinterpret_cast<GL dv2*>(G.V + o) = z;
    }
    if (NT > 0 && lr) ft_step<NT>(f, z.x, z.y, acc);
  }
  if (NT > 0 && lr) put_ft_partials<NT>(A, red, acc, G.p_part, 0);
}

// dst[a][rc] = src(a, rc): slab layout to row-major [n][R].
__global__ void k_cg_unpack(const CgArgs* __restrict__ AA, int which) {
  const CgArgs& A = AA[blockIdx.z];
  const Gv G = gview(A);
  const GL double* src = which == 0 ? G.X : G.V;
  GL double* dst = which == 0 ? G.P : G.Q;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= A.n * (int64_t)A.R) return;
  const int64_t a = idx / A.R;
  const int rc = (int)(idx - a * A.R);
  dst[idx] = rc == 0 ? src[a] : src[A.ny + (int64_t)((rc - 1) >> 5) * A.n * kSlab + a * kSlab + ((rc - 1) & 31)];
}

// ------------------------------------------------------------ launches
struct Launch {
  int nbs, nbu, ns, R, n1;
  bool use_pc, lowrank;
  int B;
  bool uni;     // SpMM over the 4-row union lists
  bool fw;      // F w products of the update kernels on the matrix cores
};

template <int NI>
void launch_iteration(hipStream_t st, const CgArgs* dA, const Launch& L, Ctx* c) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c != nullptr && c->timing) {
    e0 = c->event();
    SDGP_HIP(hipEventRecord(e0, st));
  }
  if (L.ns == 0) {
    k_cg_spmm<0><<<dim3(L.nbs, 1, L.B), kT, 0, st>>>(dA);
  } else if (L.uni) {
    k_cg_spmm_u<1><<<dim3(L.nbs, 1, L.B), kT, 0, st>>>(dA);
    if (L.ns > 1) {
      SDGP_CHECK_LAUNCH();
      k_cg_spmm_u<2><<<dim3(L.nbs, L.ns - 1, L.B), kT, 0, st>>>(dA);
    }
  } else {
    k_cg_spmm<1><<<dim3(L.nbs, 1, L.B), kT, 0, st>>>(dA);
    if (L.ns > 1) {
      SDGP_CHECK_LAUNCH();
      k_cg_spmm<2><<<dim3(L.nbs, L.ns - 1, L.B), kT, 0, st>>>(dA);
    }
  }
  SDGP_CHECK_LAUNCH();
  if (c != nullptr && c->timing) {
    e1 = c->event();
    SDGP_HIP(hipEventRecord(e1, st));
    c->spmm_events.push_back({e0, e1});
  }
  k_cg_colsum<<<dim3(L.R, 1, L.B), kSumT, 0, st>>>(dA, 0);
  SDGP_CHECK_LAUNCH();
  if (L.fw) k_cg_update_xr<NI, 1><<<dim3(L.nbu, L.ns, L.B), kT, 0, st>>>(dA);
  else k_cg_update_xr<NI, 0><<<dim3(L.nbu, L.ns + 1, L.B), kT, 0, st>>>(dA);
  SDGP_CHECK_LAUNCH();
  k_cg_colsum<<<dim3((1 + (L.use_pc ? L.n1 : 0)) * L.R, 1, L.B), kSumT, 0, st>>>(dA, 1);
  SDGP_CHECK_LAUNCH();
  if (L.use_pc) {
    k_cg_small_solve<<<dim3(L.R, 1, L.B), 64, 0, st>>>(dA);
    SDGP_CHECK_LAUNCH();
  }
  if (L.fw) k_cg_update_p<NI, 1><<<dim3(L.nbu, L.ns, L.B), kT, 0, st>>>(dA);
  else k_cg_update_p<NI, 0><<<dim3(L.nbu, L.ns + 1, L.B), kT, 0, st>>>(dA);
  SDGP_CHECK_LAUNCH();
  if (L.lowrank) {
    k_cg_colsum<<<dim3(L.n1 * L.R, 1, L.B), kSumT, 0, st>>>(dA, 2);
    SDGP_CHECK_LAUNCH();
  }
  k_cg_check<<<dim3(1, 1, L.B), 256, 0, st>>>(dA);
  SDGP_CHECK_LAUNCH();
}

template <int NI>
void launch_start(hipStream_t st, const CgArgs* dA, const Launch& L) {
  k_cg_norm<NI><<<dim3(L.nbu, L.ns + 1, L.B), kT, 0, st>>>(dA);
  SDGP_CHECK_LAUNCH();
  k_cg_colsum<<<dim3((1 + (L.use_pc ? L.n1 : 0)) * L.R, 1, L.B), kSumT, 0, st>>>(dA, 1);
  SDGP_CHECK_LAUNCH();
  if (L.use_pc) {
    k_cg_small_solve<<<dim3(L.R, 1, L.B), 64, 0, st>>>(dA);
    SDGP_CHECK_LAUNCH();
  }
  k_cg_init_fin<NI><<<dim3(L.nbu, L.ns + 1, L.B), kT, 0, st>>>(dA);
  SDGP_CHECK_LAUNCH();
  if (L.lowrank) {
    k_cg_colsum<<<dim3(L.n1 * L.R, 1, L.B), kSumT, 0, st>>>(dA, 2);
    SDGP_CHECK_LAUNCH();
  }
}

void cg_iteration(int NI, hipStream_t st, const CgArgs* dA, const Launch& L, Ctx* c) {
  switch (NI) {
    case 0: launch_iteration<0>(st, dA, L, c); break;
    case 8: launch_iteration<8>(st, dA, L, c); break;
    case 16: launch_iteration<16>(st, dA, L, c); break;
    case 32: launch_iteration<32>(st, dA, L, c); break;
    default: launch_iteration<64>(st, dA, L, c); break;
  }
}

void cg_start(int NI, hipStream_t st, const CgArgs* dA, const Launch& L) {
  switch (NI) {
    case 0: launch_start<0>(st, dA, L); break;
    case 8: launch_start<8>(st, dA, L); break;
    case 16: launch_start<16>(st, dA, L); break;
    case 32: launch_start<32>(st, dA, L); break;
    default: launch_start<64>(st, dA, L); break;
  }
}

int64_t round8(int64_t v) { return (v + 7) / 8 * 8; }

// Blocks of the update kernels resident per CU (the p-update needs at least
// as many registers as the x/r-update); the default grid is one round of
// them over the whole GPU.
template <int NI>
int update_blocks_per_cu(bool fw) {
  int nb = 0;
  const hipError_t e = fw ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cg_update_p<NI, 1>, kT, 0)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cg_update_p<NI, 0>, kT, 0);
  return (e == hipSuccess && nb > 0) ? nb : 2;
}
int update_blocks_per_cu(int NI, bool fw) {
  switch (NI) {
    case 0: return update_blocks_per_cu<0>(fw);
    case 8: return update_blocks_per_cu<8>(fw);
    case 16: return update_blocks_per_cu<16>(fw);
    case 32: return update_blocks_per_cu<32>(fw);
    default: return update_blocks_per_cu<64>(fw);
  }
}

// ------------------------------------------------------------ autotuner
// The first solve of a problem class (architecture, bump-function class,
// right-hand-side slabs, population or single, log2 of the rows, entries
// per row in half-octaves for single solves, operator form, preconditioner)
// times candidate
// launch shapes on the caller's own problem: short trial solves of
// kTrialIters CG iterations each, timed with HIP events over the
// iterations after the first kTrialSkip.  Stage 1 sweeps the SpMM form
// (union lists or CSR rows) and its grid; stage 2 sweeps the update
// kernels' grid (one, two or three resident rounds) and the F w product
// form.  A candidate replaces the incumbent only when it is at least 1%
// faster.  The winner goes to the persistent store and is used from then
// on; the shapes change only the order of floating-point sums.
constexpr int kTrialIters = 24;
constexpr int kTrialSkip = 8;
constexpr int64_t kTuneMinRows = 65536;

struct ShapeGuard {   // leaves trial mode on every exit path
  Ctx* c;
  ~ShapeGuard() { c->in_trial = false; }
};

// A population's members differ in their entries per row, so its class
// leaves that out (one tuned shape serves every population of the class).
std::string tune_key(const Ctx* c, int NI, int ns, int B, int64_t n, int64_t nnz, bool lr, bool pc) {
  const double per_row = std::max(1.0, (double)nnz / (double)std::max<int64_t>(n, 1));
  int lgn = 0;
  while (((int64_t)2 << lgn) <= n) ++lgn;
  const int rb = B > 1 ? -1 : (int)std::lround(2.0 * std::log2(per_row));
  char buf[160];
  std::snprintf(buf, sizeof(buf), "%s|ni%d|ns%d|b%d|n%d|r%d|lr%d|pc%d", c->arch.c_str(), NI, ns, B > 1 ? 2 : 1,
                lgn, rb, lr ? 1 : 0, pc ? 1 : 0);
  return buf;
}

}  // namespace

// Trial solves of the tuner (see above); returns the fastest shape, with
// ms_per_iter < 0 when the solve is too short to time.
static TuneChoice run_tuner(Ctx* c, const std::vector<CgMember>& mem, const Sorted& s, const double* ys, int kind,
                            int P, uint64_t seed, double rtol, const double* dense_rhs, int dense_R, int NI,
                            int ns, int64_t n, int n1) {
  ShapeGuard guard{c};
  const int64_t tiles = (n + kTile - 1) / kTile;
  auto trial = [&](const TuneChoice& t) -> double {
    c->in_trial = true;
    c->trial = t;
    c->trial_ms = -1.0;
    block_cg_multi(c, mem, s, ys, kind, P, seed, rtol, kTrialIters, dense_rhs, dense_R, false, false);
    c->in_trial = false;
    return c->trial_ms;
  };
  TuneChoice best;   // the defaults, made explicit
  best.spmm_blocks = (int)std::min<int64_t>(kMaxNbs, round8(tiles));
  best.union_spmm = (ns > 0 && n >= kUnionMinRows) ? 1 : 0;
  best.fw_mfma = (ns > 0 && n1 > 0) ? 1 : 0;
  const int round1 = update_blocks_per_cu(NI, best.fw_mfma != 0) * c->cu_count;
  best.update_blocks = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)kMaxNbu, (int64_t)round1, round8(tiles)}));
  double t_best = trial(best);
  best.default_ms_per_iter = t_best;
  best.ms_per_iter = t_best;
  if (t_best <= 0.0) return best;
  auto consider = [&](const TuneChoice& cand) {
    const double t = trial(cand);
    if (t > 0.0 && t < 0.99 * t_best) {
      const double d = best.default_ms_per_iter;
      best = cand;
      best.default_ms_per_iter = d;
      best.ms_per_iter = t;
      t_best = t;
    }
  };
  // stage 1: SpMM form and grid
  {
    const TuneChoice base = best;
    std::vector<int> grids;
    for (int g : {8192, 16384, 32768, 65528}) {
      const int v = (int)std::min<int64_t>(g, round8(tiles));
      if (std::find(grids.begin(), grids.end(), v) == grids.end()) grids.push_back(v);
    }
    std::vector<int> forms = {base.union_spmm};
    if (ns > 0) forms.push_back(1 - base.union_spmm);
    for (int u : forms)
      for (int g : grids) {
        if (u == base.union_spmm && g == base.spmm_blocks) continue;
        TuneChoice cand = base;
        cand.union_spmm = u;
        cand.spmm_blocks = g;
        consider(cand);
      }
  }
  // stage 2: update grid and F w product form
  {
    const TuneChoice base = best;
    std::vector<int> fws = {base.fw_mfma};
    if (ns > 0 && n1 > 0) fws.push_back(1 - base.fw_mfma);
    for (int f : fws) {
      const int r1 = update_blocks_per_cu(NI, f != 0) * c->cu_count;
      for (int k = 1; k <= 3; ++k) {
        const int ub = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)k * r1, (int64_t)65535, round8(tiles)}));
        if (f == base.fw_mfma && ub == base.update_blocks) continue;
        TuneChoice cand = base;
        cand.fw_mfma = f;
        cand.update_blocks = ub;
        consider(cand);
      }
    }
  }
  return best;
}

std::vector<CgResult> block_cg_multi(Ctx* c, const std::vector<CgMember>& mem, const Sorted& s, const double* ys,
                                     int kind, int P, uint64_t seed, double rtol, int max_iter,
                                     const double* dense_rhs, int dense_R, bool keep_v, bool use_graph,
                                     double probe_rtol) {
  const int B = (int)mem.size();
  require(B >= 1 && B <= 65535, "1..65535 members");
  const int64_t n = s.n;
  require(n >= 1, "no points");
  int R;
  if (kind == PK_DENSE) R = dense_R;
  else if (kind == PK_IDENTITY) R = (int)(1 + n);
  else if (kind == PK_NONE) R = 1;
  else R = 1 + P;
  require(R >= 1, "no right-hand sides");
  require(max_iter >= 1, "cg_max_iter must be >= 1");
  require(rtol > 0.0 && std::isfinite(rtol), "cg_rtol must be > 0");
  require(probe_rtol >= 0.0 && std::isfinite(probe_rtol), "probe_rtol must be >= 0");
  // probe columns (after y) converge at their own tolerance when one is given
  const bool probe_cols = kind == PK_RADEMACHER || kind == PK_IDENTITY;
  const double prt = (probe_cols && probe_rtol > 0.0) ? probe_rtol : rtol;
  require(kind != PK_DENSE || B == 1, "dense right-hand sides take one member");
  require(n <= 0x7fffffffLL, "n must fit a 32-bit column index");
  const Precond* pc0 = mem[0].pc;
  const bool use_pc = pc0 != nullptr && pc0->n1 > 0 && pc0->apply;
  const bool use_lr = pc0 != nullptr && pc0->n1 > 0 && pc0->lowrank_op;
  const int n1 = (use_pc || use_lr) ? pc0->n1 : 0;
  for (int m = 0; m < B; ++m) {
    const Precond* p = mem[m].pc;
    const bool up = p != nullptr && p->n1 > 0 && p->apply;
    const bool ul = p != nullptr && p->n1 > 0 && p->lowrank_op;
    require(up == use_pc && ul == use_lr && (!(up || ul) || p->n1 == n1), "members must share the solver form");
    require(mem[m].A.n == n, "members must share the point set");
  }
  require(n1 <= 64, "at most 64 bump functions");
  require((R - 1 + kSlab - 1) / kSlab + 1 <= 65535, "too many right-hand sides");
  const int NI = n1 == 0 ? 0 : (n1 <= 8 ? 8 : (n1 <= 16 ? 16 : (n1 <= 32 ? 32 : 64)));
  const int ns = (R - 1 + kSlab - 1) / kSlab;
  const int64_t ny = (n + kSlab - 1) / kSlab * kSlab;
  const size_t NV = (size_t)ny + (size_t)ns * n * kSlab;   // doubles per vector block
  require(NV >= (size_t)n * R, "layout");
  const int64_t tiles = (n + kTile - 1) / kTile;
  // Launch shape: a tuner trial's candidate; else the context options when
  // any is set; else the tuned shape of this problem class (tuned now when
  // the store has none); else the defaults.
  TuneChoice sh;
  int tuned = 0;
  const bool user_shape = c->spmm_blocks > 0 || c->update_blocks > 0 || c->union_spmm >= 0 || c->fw_mfma >= 0;
  if (c->in_trial) {
    sh = c->trial;
  } else if (user_shape) {
    sh.spmm_blocks = c->spmm_blocks;
    sh.update_blocks = c->update_blocks;
    sh.union_spmm = c->union_spmm;
    sh.fw_mfma = c->fw_mfma;
  } else if (c->autotune == 2 || (c->autotune == 1 && n >= kTuneMinRows)) {
    int64_t nnz = 0;
    for (const auto& mm : mem) nnz = std::max<int64_t>(nnz, mm.A.nnz);
    const std::string key = tune_key(c, NI, ns, B, n, nnz, use_lr, use_pc);
    const std::string path = tune_cache_path();
    TuneChoice t;
    if (tune_cache_get(path, key, &t)) {
      sh = t;
      tuned = 1;
    } else if (!c->arena) {   // trials need events; the static-workspace call only reads the store
      t = run_tuner(c, mem, s, ys, kind, P, seed, rtol, dense_rhs, dense_R, NI, ns, n, n1);
      if (t.ms_per_iter > 0.0) {
        tune_cache_put(path, key, t);
        sh = t;
        tuned = 2;
      }
    }
  }
  const int64_t nbs_cap = sh.spmm_blocks > 0 ? sh.spmm_blocks : kMaxNbs;
  const int nbs = (int)std::min<int64_t>(nbs_cap, round8(tiles));
  // F w products of the update kernels on the matrix cores (measured faster at
  // 16 and at 32 bump functions); 0 per-row broadcasts
  const bool fw = ns > 0 && n1 > 0 && sh.fw_mfma != 0;
  const int64_t nbu_cap = sh.update_blocks > 0
                              ? sh.update_blocks
                              : std::min<int64_t>(kMaxNbu, (int64_t)update_blocks_per_cu(NI, fw) * c->cu_count);
  const int nbu = (int)std::max<int64_t>(1, std::min<int64_t>(nbu_cap, round8(tiles)));
  const int nu = 1 + (use_pc ? n1 : 0);
  double* X = c->get<double>(S_CG_X, NV * B);
  double* Rr = c->get<double>(S_CG_R, NV * B);
  double* Pp = c->get<double>(S_CG_P, NV * B);
  double* Q = c->get<double>(S_CG_Q, NV * B);
  double* V = (use_pc && keep_v) ? c->get<double>(S_CG_V, NV * B) : nullptr;
  double* s_part = c->get<double>(S_CG_PART, (size_t)R * nbs * B);
  double* s_red = c->get<double>(S_CG_SRED, (size_t)R * B);
  double* u_part = c->get<double>(S_CG_PART2, (size_t)nu * R * nbu * B);
  double* u_red = c->get<double>(S_CG_G, (size_t)nu * R * B);
  double* w_red = use_pc ? c->get<double>(S_CG_WRED, (size_t)(n1 + 1) * R * B) : nullptr;
  double* p_part = use_lr ? c->get<double>(S_CG_PARTG, (size_t)n1 * R * nbu * B) : nullptr;
  double* p_red = use_lr ? c->get<double>(S_CG_GP, (size_t)n1 * R * B) : nullptr;
  // 4-row union lists of the shared-gather SpMM (per member): lengths,
  // exclusive scan on the host (once per solve), columns and values
  // (automatic from kUnionMinRows rows: below that, building the lists costs
  // more than the solve saves)
  bool uni = ns > 0 && (sh.union_spmm > 0 || (sh.union_spmm < 0 && n >= kUnionMinRows));
  const int64_t ng = (n + 3) / 4;
  int64_t* urp = nullptr;
  int32_t* ucol = nullptr;
  double* uval = nullptr;
  std::vector<int64_t> uoff(B + 1, 0);
  std::vector<int64_t> hp;
  const unsigned ugb = (unsigned)((ng + 255) / 256);
  if (uni) {
    int32_t* ucnt = c->get<int32_t>(S_CG_UCNT, (size_t)ng * B);
    for (int m = 0; m < B; ++m) {
      k_union_count<<<ugb, 256, 0, c->stream>>>(n, ng, mem[m].A.row_ptr, mem[m].A.col, s.sched,
                                                ucnt + (size_t)m * ng);
      SDGP_CHECK_LAUNCH();
    }
    std::vector<int32_t> hc((size_t)ng * B);
    SDGP_HIP(hipMemcpyAsync(hc.data(), ucnt, hc.size() * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    SDGP_HIP(hipStreamSynchronize(c->stream));
    hp.resize((size_t)(ng + 1) * B);
    for (int m = 0; m < B; ++m) {
      int64_t acc = 0;
      for (int64_t q = 0; q < ng; ++q) {
        hp[(size_t)m * (ng + 1) + q] = acc;
        acc += hc[(size_t)m * ng + q];
      }
      hp[(size_t)m * (ng + 1) + ng] = acc;
      require(acc <= mem[m].A.nnz || mem[m].A.nnz < 0, "union lists longer than the matrix");
      uoff[m + 1] = uoff[m] + acc;
    }
    // the lists take 36 B per entry on top of the CSR; in automatic mode the
    // CSR SpMM is used instead when they would take more than half of the
    // free device memory (large populations)
    size_t free_b = 0, total_b = 0;
    const bool fits = hipMemGetInfo(&free_b, &total_b) != hipSuccess ||
                      (double)uoff[B] * 36.0 + (double)hp.size() * 8.0 <= 0.5 * (double)free_b;
    if (!fits && c->union_spmm <= 0) uni = false;   // unless the caller asked for the lists
  }
  if (uni) {
    urp = c->get<int64_t>(S_CG_UPTR, hp.size());
    SDGP_HIP(hipMemcpyAsync(urp, hp.data(), hp.size() * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
    ucol = c->get<int32_t>(S_CG_UCOL, (size_t)std::max<int64_t>(uoff[B], 1));
    uval = c->get<double>(S_CG_UVAL, (size_t)std::max<int64_t>(uoff[B], 1) * 4);
    for (int m = 0; m < B; ++m) {
      k_union_fill<<<ugb, 256, 0, c->stream>>>(n, ng, mem[m].A.row_ptr, mem[m].A.col, mem[m].A.val, s.sched,
                                               urp + (size_t)m * (ng + 1), ucol + uoff[m], uval + 4 * uoff[m]);
      SDGP_CHECK_LAUNCH();
    }
    SDGP_HIP(hipStreamSynchronize(c->stream));   // hp is read by the copy above
  }
  double* ha = c->get<double>(S_CG_HIST_A, (size_t)max_iter * R * B);
  double* hb = c->get<double>(S_CG_HIST_B, (size_t)max_iter * R * B);
  // per-member state block: doubles rz[2R], rz0[R], bnorm2[R], rr_last[R];
  // ints act[2R], failed[R], iters[R], done, not_spd, it
  const size_t sbytes = ((5 * (size_t)R) * 8 + (4 * (size_t)R + 3) * 4 + 255) / 256 * 256;
  char* sb = c->get<char>(S_CG_STATE, sbytes * B);
  SDGP_HIP(hipMemsetAsync(sb, 0, sbytes * B, c->stream));
  std::vector<CgArgs> hA(B);
  for (int m = 0; m < B; ++m) {
    CgArgs& A = hA[m];
    const Csr& Am = mem[m].A;
    const Precond* p = mem[m].pc;
    A.n = n;
    A.ny = ny;
    A.R = R;
    A.ns = ns;
    A.row_ptr = Am.row_ptr;
    A.col = Am.col;
    A.val = Am.val;
    A.X = X + m * NV;
    A.Rr = Rr + m * NV;
    A.P = Pp + m * NV;
    A.Q = Q + m * NV;
    A.V = V ? V + m * NV : nullptr;
    A.sched = s.sched;
    A.F = n1 > 0 ? p->F : nullptr;
    A.Sinv = use_pc ? p->Sinv : nullptr;
    A.n1 = n1;
    A.use_pc = use_pc ? 1 : 0;
    A.lowrank_op = use_lr ? 1 : 0;
    A.inv_c = use_pc ? 1.0 / p->c : 1.0;
    A.sqrt_c = use_pc ? std::sqrt(p->c) : 1.0;
    A.nbs = nbs;
    A.nbu = nbu;
    A.max_iter = max_iter;
    A.rtol2 = rtol * rtol;
    A.prtol2 = prt * prt;
    A.s_part = s_part + (size_t)m * R * nbs;
    A.s_red = s_red + (size_t)m * R;
    A.u_part = u_part + (size_t)m * nu * R * nbu;
    A.u_red = u_red + (size_t)m * nu * R;
    A.w_red = w_red ? w_red + (size_t)m * (n1 + 1) * R : nullptr;
    A.p_part = p_part ? p_part + (size_t)m * n1 * R * nbu : nullptr;
    A.p_red = p_red ? p_red + (size_t)m * n1 * R : nullptr;
    A.urp = uni ? urp + (size_t)m * (ng + 1) : nullptr;
    A.ucol = uni ? ucol + uoff[m] : nullptr;
    A.uval = uni ? uval + 4 * uoff[m] : nullptr;
    char* mb = sb + sbytes * m;
    A.st.rz = reinterpret_cast<double*>(mb);
    A.st.rz0 = A.st.rz + 2 * (size_t)R;
    A.st.bnorm2 = A.st.rz0 + R;
    A.st.rr_last = A.st.bnorm2 + R;
    int32_t* ib = reinterpret_cast<int32_t*>(A.st.rr_last + R);
    A.st.act = ib;
    A.st.failed = ib + 2 * (size_t)R;
    A.st.iters = A.st.failed + R;
    A.st.done = A.st.iters + R;
    A.st.not_spd = A.st.done + 1;
    A.st.it = A.st.not_spd + 1;
    A.st.hist_a = ha + (size_t)m * max_iter * R;
    A.st.hist_b = hb + (size_t)m * max_iter * R;
  }
  CgArgs* dA = c->get<CgArgs>(S_CG_ARGS, B);
  SDGP_HIP(hipMemcpyAsync(dA, hA.data(), B * sizeof(CgArgs), hipMemcpyHostToDevice, c->stream));
  Launch L{nbs, nbu, ns, R, n1, use_pc, use_lr, B, uni, fw};
  if (!c->in_trial) {
    c->last_shape.spmm_blocks = nbs;
    c->last_shape.update_blocks = nbu;
    c->last_shape.union_spmm = uni ? 1 : 0;
    c->last_shape.fw_mfma = fw ? 1 : 0;
    c->last_shape.ms_per_iter = sh.ms_per_iter;
    c->last_shape.default_ms_per_iter = sh.default_ms_per_iter;
    c->last_tuned = tuned;
  }
  {
    const int64_t gx = ((int64_t)NV + 255) / 256;
    require(gx < 0x7fffffff, "n*R too large");
    k_cg_start<<<dim3((unsigned)gx, 1, B), 256, 0, c->stream>>>(dA, ys, s.perm, kind, seed, dense_rhs);
    SDGP_CHECK_LAUNCH();
  }
  cg_start(NI, c->stream, dA, L);
  // iterate; poll the per-member flags now and then.  Members that have
  // stopped leave the launch grid (grid z covers the active members only).
  std::vector<int32_t> flags((size_t)3 * B);
  std::vector<int> active(B);
  for (int m = 0; m < B; ++m) active[m] = m;
  std::vector<CgArgs> hAct;
  auto poll = [&](hipStream_t st) -> bool {  // true when the active set shrank
    for (int m : active)
      SDGP_HIP(hipMemcpyAsync(&flags[3 * m], hA[m].st.done, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SDGP_HIP(hipStreamSynchronize(st));
    std::vector<int> still;
    for (int m : active)
      if (flags[3 * m] == 0 && flags[3 * m + 2] < max_iter) still.push_back(m);
    if (still.size() == active.size()) return false;
    active.swap(still);
    if (!active.empty()) {
      hAct.clear();
      for (int m : active) hAct.push_back(hA[m]);
      SDGP_HIP(hipMemcpyAsync(dA, hAct.data(), hAct.size() * sizeof(CgArgs), hipMemcpyHostToDevice, st));
      SDGP_HIP(hipStreamSynchronize(st));
      L.B = (int)active.size();
    }
    return true;
  };
  // y alone: once every probe column of a single evaluation has stopped
  // (they stop first when their tolerance is looser than y's), the rest of
  // y's solve runs the column-0 kernels only -- the CSR SpMM of column 0
  // and the column-0 blocks of the update kernels -- with the device
  // arguments' slab count set to 0 (restored for the unpack).
  const bool tail_ok = B == 1 && ns > 0 && probe_cols && prt > rtol && !c->in_trial;
  bool tail = false;
  int tail_from = 0;                              // iterations executed when y went alone
  std::vector<int32_t> act_h((size_t)2 * R);
  auto try_tail = [&](hipStream_t st) -> bool {   // true when switched
    if (!tail_ok || tail || active.empty()) return false;
    const int E = flags[2];                       // iterations executed (from the last poll)
    SDGP_HIP(hipMemcpyAsync(act_h.data(), hA[0].st.act, 2 * R * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SDGP_HIP(hipStreamSynchronize(st));
    const int32_t* a = act_h.data() + (size_t)(E & 1) * R;   // state for iteration E
    if (!a[0]) return false;
    for (int r = 1; r < R; ++r)
      if (a[r]) return false;
    tail = true;
    tail_from = E;
    L.ns = 0;
    L.uni = false;
    L.fw = false;
    hA[0].ns = 0;
    SDGP_HIP(hipMemcpyAsync(dA, hA.data(), sizeof(CgArgs), hipMemcpyHostToDevice, st));
    SDGP_HIP(hipStreamSynchronize(st));
    hA[0].ns = ns;
    return true;
  };
  c->spmm_events.clear();
  int launched = 0;
  if (use_graph) {
    // capture k iterations and replay them: the iteration counters live on
    // the device, so every replay advances the solve; kernels of members
    // that are done, or past max_iter, return at once.  The graph is
    // captured again whenever the active set shrinks.
    const int k = 8;
    hipStream_t gs = c->graph_stream();
    hipEvent_t ready = c->event();
    SDGP_HIP(hipEventRecord(ready, c->stream));
    SDGP_HIP(hipStreamWaitEvent(gs, ready, 0));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    auto capture = [&]() {
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      exec = nullptr;
      graph = nullptr;
      SDGP_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
      for (int q = 0; q < k; ++q) cg_iteration(NI, gs, dA, L, nullptr);
      SDGP_HIP(hipStreamEndCapture(gs, &graph));
      hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (ie != hipSuccess) {
        (void)hipGraphDestroy(graph);
        graph = nullptr;
        throw Error(SDGP_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
      }
    };
    capture();
    int every = 1;
    while (!active.empty() && launched < max_iter) {
      for (int q = 0; q < every && launched < max_iter; ++q) {
        SDGP_HIP(hipGraphLaunch(exec, gs));
        launched += k;
      }
      if (poll(gs) && !active.empty()) capture();
      else if (try_tail(gs)) capture();
      every = std::min(every * 2, 8);
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    hipEvent_t back = c->event();
    SDGP_HIP(hipEventRecord(back, gs));
    SDGP_HIP(hipStreamWaitEvent(c->stream, back, 0));
  } else {
    int check = 8;
    hipEvent_t t0 = nullptr;
    while (!active.empty() && launched < max_iter) {
      const int upto = std::min(max_iter, launched + check);
      for (; launched < upto; ++launched) cg_iteration(NI, c->stream, dA, L, c);
      if (c->in_trial && launched == kTrialSkip) {
        t0 = c->event();
        SDGP_HIP(hipEventRecord(t0, c->stream));
      }
      poll(c->stream);
      try_tail(c->stream);
      check = std::min(check * 2, 64);
    }
    // trial: timed only when no member converged before the end (the
    // iterations after convergence would be empty launches)
    bool full = true;
    for (int m = 0; m < B; ++m)
      if (flags[3 * m] != 0) full = false;
    if (c->in_trial && t0 && full && launched > kTrialSkip) {
      hipEvent_t t1 = c->event();
      SDGP_HIP(hipEventRecord(t1, c->stream));
      SDGP_HIP(hipEventSynchronize(t1));
      float ms = 0.0f;
      SDGP_HIP(hipEventElapsedTime(&ms, t0, t1));
      c->trial_ms = (double)ms / (double)(launched - kTrialSkip);
    }
  }
  // every member's arguments again, for the unpack
  if (L.B != B || tail) {
    SDGP_HIP(hipMemcpyAsync(dA, hA.data(), B * sizeof(CgArgs), hipMemcpyHostToDevice, c->stream));
    L.B = B;
  }
  // solutions (and M^{-1} b) back to row-major [n][R], into the P and Q
  // storage that the iteration no longer needs
  {
    const int64_t gx = ((int64_t)n * R + 255) / 256;
    require(gx < 0x7fffffff, "n*R too large");
    k_cg_unpack<<<dim3((unsigned)gx, 1, B), 256, 0, c->stream>>>(dA, 0);
    SDGP_CHECK_LAUNCH();
    if (V) {
      k_cg_unpack<<<dim3((unsigned)gx, 1, B), 256, 0, c->stream>>>(dA, 1);
      SDGP_CHECK_LAUNCH();
    }
  }
  // results
  std::vector<CgResult> out(B);
  std::vector<int32_t> its((size_t)R * B), actv((size_t)2 * R * B);
  std::vector<double> bn((size_t)R * B), rl((size_t)R * B);
  for (int m = 0; m < B; ++m) {
    SDGP_HIP(hipMemcpyAsync(&its[(size_t)m * R], hA[m].st.iters, R * sizeof(int32_t), hipMemcpyDeviceToHost,
                            c->stream));
    SDGP_HIP(hipMemcpyAsync(&actv[(size_t)2 * m * R], hA[m].st.act, 2 * R * sizeof(int32_t),
                            hipMemcpyDeviceToHost, c->stream));
    SDGP_HIP(hipMemcpyAsync(&bn[(size_t)m * R], hA[m].st.bnorm2, R * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
    SDGP_HIP(hipMemcpyAsync(&rl[(size_t)m * R], hA[m].st.rr_last, R * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
    SDGP_HIP(hipMemcpyAsync(&flags[3 * m], hA[m].st.done, 3 * sizeof(int32_t), hipMemcpyDeviceToHost,
                            c->stream));
  }
  SDGP_HIP(hipStreamSynchronize(c->stream));
  for (int m = 0; m < B; ++m) {
    CgResult& res = out[m];
    const CgArgs& A = hA[m];
    res.R = R;
    res.X = A.P;
    res.V = A.V ? A.Q : nullptr;
    res.rz0 = A.st.rz0;
    res.hist_a = A.st.hist_a;
    res.hist_b = A.st.hist_b;
    res.col_iters = A.st.iters;
    res.not_spd = flags[3 * m + 1] != 0;
    res.logdetM = use_pc ? mem[m].pc->logdetM : 0.0;
    const int executed = flags[3 * m] > 0 ? flags[3 * m] : flags[3 * m + 2];
    const int lastpar = executed & 1;  // parity holding the latest state
    bool conv = true;
    for (int r = 0; r < R; ++r)
      if (actv[(size_t)2 * m * R + lastpar * R + r]) conv = false;
    res.iters = executed;
    res.iters_y = its[(size_t)m * R];
    res.relres_max = 0.0;
    for (int r = 0; r < R; ++r) {
      const double b2 = bn[(size_t)m * R + r];
      if (b2 > 0.0) res.relres_max = std::max(res.relres_max, std::sqrt(rl[(size_t)m * R + r] / b2));
    }
    res.converged = conv && !res.not_spd;
  }
  if (!c->in_trial) c->last_y_tail = tail ? std::max(0, out[0].iters - tail_from) : 0;
  return out;
}

CgResult block_cg(Ctx* c, const Csr& Am, const Sorted& s, const double* ys, int kind, int P, uint64_t seed,
                  double rtol, int max_iter, const double* dense_rhs, int dense_R, const Precond* pc,
                  bool keep_v, PhaseTimer* t, double probe_rtol) {
  (void)t;
  std::vector<CgMember> mem(1);
  mem[0].A = Am;
  mem[0].pc = pc;
  return block_cg_multi(c, mem, s, ys, kind, P, seed, rtol, max_iter, dense_rhs, dense_R, keep_v,
                        c->use_graph, probe_rtol)[0];
}

// Plain SpMM Y = A X for row-major X, Y [n][R] with R even (16-byte rows
// of pairs): slabs of 32 columns over grid y, 16 lanes per row.
namespace {
__global__ __launch_bounds__(kT) void k_spmm_slab(int64_t n, const int64_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col, const double* __restrict__ val,
                                                  const double* __restrict__ X, int R, double* __restrict__ Y) {
  const int lane = lane_id(), g = lane >> 4, j = lane & 15, w = threadIdx.x >> 6;
  const int c0 = (int)blockIdx.y * kSlab + 2 * j;
  const int cc = c0 + 1 < R ? c0 : R - 2;   // lanes past the last column read a valid pair
  const int xcd = blockIdx.x & 7;
  const int64_t bi = blockIdx.x >> 3, nbx = gridDim.x >> 3;
  const int64_t nx = (n + 7) >> 3, lo = xcd * nx, hi = min(n, lo + nx);
  for (int64_t pb = lo + bi * kTile + w * 4; pb < hi; pb += nbx * kTile) {
    const int64_t a = pb + g;
    const bool live = a < hi;
    const int64_t k0 = live ? row_ptr[a] : 0, k1 = live ? row_ptr[a + 1] : 0;
    dv2 q;
    double unused = 0.0;
    slab_row<false>(k0, k1, live ? (int32_t)a : 0, (const GL int32_t*)col, (const GL double*)val,
                    (const GL double*)(X + cc), R, nullptr, q, unused);
    if (live && c0 + 1 < R) *reinterpret_cast<dv2*>(Y + a * R + c0) = q;
  }
}
}  // namespace

void spmm_slab(Ctx* c, const Csr& A, const double* X, int R, double* Y) {
  require(R >= 2 && R % 2 == 0, "slab SpMM needs an even column count");
  require(A.n <= 0x7fffffffLL, "n must fit a 32-bit column index");
  const int64_t tiles = (A.n + kTile - 1) / kTile;
  const int nb = (int)std::min<int64_t>(kMaxNbs, round8(tiles));
  const int ns = (R + kSlab - 1) / kSlab;
  k_spmm_slab<<<dim3(nb, ns), kT, 0, c->stream>>>(A.n, A.row_ptr, A.col, A.val, X, R, Y);
  SDGP_CHECK_LAUNCH();
}

}  // namespace sdgp
