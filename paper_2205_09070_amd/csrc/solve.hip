// Iterative solves on the sparse covariance (Section 2.5): SpMM, block
// conjugate gradients on [y, z_1..z_P], and stochastic Lanczos quadrature of
// ln det A from the CG coefficients, for gfx950.
//
// Layout: every vector block is row-major [n][R] so one wavefront handles one
// row and its 64 lanes hold 64 consecutive right-hand sides: a gathered
// neighbour row X[b, :] is one coalesced load.  CSR entries of a row are
// fetched 64 at a time by the lanes and broadcast with readlane.
//
// Reductions are deterministic: each block writes per-column partial sums;
// the consumer kernel of the next phase re-reduces all partials of its
// column chunk in a fixed order inside every block (so every block obtains
// bit-identical scalars without atomics or grid-wide barriers).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>
#include <vector>

#include "kernel_math.hpp"
#include "sdgp_internal.hpp"

namespace sdgp {

namespace {

constexpr int kCgBlock = 1024;             // 16 wavefronts
constexpr int kCgWaves = kCgBlock / kWave;

// y = sum_k val[k] X[col[k], rc] over one CSR row (the calling wave's row).
// The row's entries are loaded 64 at a time by the lanes and broadcast with
// readlane; 16 gathers are issued before their products are summed so that
// enough loads are in flight to cover the cache latency.
__device__ __forceinline__ double row_dot(const int64_t k0, const int64_t k1, const int32_t* __restrict__ col,
                                          const double* __restrict__ val, const double* __restrict__ Xc,
                                          const int64_t R) {
  const int lane = lane_id();
  double acc = 0.0;
  for (int64_t kb = k0; kb < k1; kb += kWave) {
    const int64_t k = kb + lane;
    int cj = 0;
    double vj = 0.0;
    if (k < k1) { cj = col[k]; vj = val[k]; }
    const int cnt = (int)min((int64_t)kWave, k1 - kb);
    int j = 0;
    for (; j + 16 <= cnt; j += 16) {
      double xv[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) xv[u] = Xc[(int64_t)readlane_i32(cj, j + u) * R];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc += readlane_f64(vj, j + u) * xv[u];
    }
    for (; j + 4 <= cnt; j += 4) {
      double xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) xv[u] = Xc[(int64_t)readlane_i32(cj, j + u) * R];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc += readlane_f64(vj, j + u) * xv[u];
    }
    for (; j < cnt; ++j) acc += readlane_f64(vj, j) * Xc[(int64_t)readlane_i32(cj, j) * R];
  }
  return acc;
}

// Rows handled by the calling wave under an XCD-aware mapping: the grid's
// blocks are dealt round-robin to the 8 XCDs, so XCD x (blocks with
// blockIdx.x % 8 == x) takes the x-th eighth of the rows and all its waves
// sweep that range together, keeping the gathered neighbour rows in the
// XCD's own L2.  gridDim.x must be a multiple of 8.
struct RowSweep {
  int64_t a, hi, step;
  __device__ RowSweep(int64_t n, int waves_per_block) {
    const int xcd = blockIdx.x & 7;
    const int64_t bi = blockIdx.x >> 3;
    const int64_t nbx = gridDim.x >> 3;
    const int64_t nx = (n + 7) >> 3;
    const int64_t lo = xcd * nx;
    hi = min(n, lo + nx);
    step = nbx * waves_per_block;
    a = lo + bi * waves_per_block + (threadIdx.x >> 6);
  }
};

// Plain SpMM: Y = A X (one wave per row, lanes over a 64-column chunk).
__global__ __launch_bounds__(256) void k_spmm(int64_t n, const int64_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col, const double* __restrict__ val,
                                              const double* __restrict__ X, int R, double* __restrict__ Y) {
  const int rc = blockIdx.y * kWave + lane_id();
  const int rcc = rc < R ? rc : R - 1;
  for (RowSweep w(n, 4); w.a < w.hi; w.a += w.step) {
    const int64_t a = w.a;
    const double v = row_dot(row_ptr[a], row_ptr[a + 1], col, val, X + rcc, R);
    if (rc < R) Y[a * (int64_t)R + rc] = v;
  }
}

// SpMV (one right-hand side): 16 lanes per row, 4 rows per wave; each lane
// first loads up to 8 of its row's (column, value) pairs, then issues the 8
// gathers together (two round trips per 128 entries instead of sixteen).
__global__ __launch_bounds__(256) void k_spmv(int64_t n, const int64_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col, const double* __restrict__ val,
                                              const double* __restrict__ x, double* __restrict__ y) {
  const int sub = threadIdx.x & 15;
  const int xcd = blockIdx.x & 7;
  const int64_t bi = blockIdx.x >> 3, nbx = gridDim.x >> 3;
  const int64_t nx = (n + 7) >> 3, lo = xcd * nx, hi = min(n, lo + nx);
  const int64_t groups = blockDim.x >> 4;
  for (int64_t a = lo + bi * groups + (threadIdx.x >> 4); a - (threadIdx.x >> 4) < hi; a += nbx * groups) {
    double acc = 0.0;
    if (a < hi) {
      const int64_t k1 = row_ptr[a + 1];
      for (int64_t k0 = row_ptr[a] + sub; k0 < k1; k0 += 16 * 8) {
        int cj[8];
        double vj[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int64_t k = k0 + 16 * u;
          cj[u] = k < k1 ? col[k] : 0;
          vj[u] = k < k1 ? val[k] : 0.0;
        }
        double xv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) xv[u] = x[cj[u]];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += vj[u] * xv[u];
      }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 16);
    if (a < hi && sub == 0) y[a] = acc;
  }
}

struct CgState {
  double* rz;       // [2][R] parity buffers of the CG scalar r.z (r.r unpreconditioned)
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

// Fixed-order reduction of per-block partials part[b*stride + rc] (b < nb)
// for the 64-column chunk of this block into sh[0..63].  All blocks obtain
// bit-identical values.
__device__ void chunk_reduce(const double* __restrict__ part, int nb, int64_t stride, int R, double* sh,
                             double* scratch) {
  const int t = threadIdx.x;
  const int l = t & 63, w = t >> 6;
  const int rc = blockIdx.y * kWave + l;
  double s = 0.0;
  if (rc < R)
    for (int b = w; b < nb; b += kCgWaves) s += part[(int64_t)b * stride + rc];
  scratch[w * kWave + l] = s;
  __syncthreads();
  if (t < kWave) {
    double tot = 0.0;
    for (int q = 0; q < kCgWaves; ++q) tot += scratch[q * kWave + t];
    sh[t] = tot;
  }
  __syncthreads();
}

// Block partial of per-lane values over the block's waves into
// part[blockIdx.x*stride + rc].
__device__ void block_partial(double v, double* scratch, double* part, int64_t stride, int R) {
  const int t = threadIdx.x;
  const int l = t & 63, w = t >> 6;
  __syncthreads();
  scratch[w * kWave + l] = v;
  __syncthreads();
  if (t < kWave) {
    double tot = 0.0;
    for (int q = 0; q < kCgWaves; ++q) tot += scratch[q * kWave + t];
    const int rc = blockIdx.y * kWave + t;
    if (rc < R) part[(int64_t)blockIdx.x * stride + rc] = tot;
  }
}

struct CgArgs {
  int64_t n;
  int R;
  const int64_t* row_ptr;
  const int32_t* col;
  const double* val;
  double *X, *Rr, *P, *Q;
  double* part;        // [nb][R] p.Ap partials (written by the SpMM, read by update_xr)
  double* part2;       // [nb][R] r.r partials (written by update_xr / norm_part, read after)
  double* partg;       // [nb][n1][R]  F^T p / F^T r partials (each reduced by its own launch)
  double* g;           // [n1][R]
  double* V;           // [n][R] M^{-1} b (preconditioned, may be null)
  const int32_t* sched;  // row processing order for the SpMM (may be null)
  const double* F;     // [n][n1] sorted bump values
  const double* Sinv;  // [n1][n1] (c I + F^T F)^{-1}
  int n1;
  int use_pc;          // preconditioned: g = F^T r, z = M^{-1} r on the fly
  int lowrank_op;      // operator K_core P + F (F^T P) (SUM combine)
  double* gp;          // [n1][R] F^T p (lowrank_op)
  double inv_c, sqrt_c;
  int nb;
  int max_iter;
  CgState st;
  double rtol2;
};

// Per-block partials of F^T v (v: this lane's column of the block's rows)
// given per-lane accumulators acc[NI]: reduced 4 at a time through LDS.
template <int NI>
__device__ void block_partial_g(const double* acc, double* gs, const CgArgs& A, double* out) {
  const int t = threadIdx.x;
  const int l = t & 63, w = t >> 6;
  const int rc = blockIdx.y * kWave + l;
#pragma unroll
  for (int i0 = 0; i0 < NI; i0 += 4) {
    if (i0 >= A.n1) break;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) gs[(q * kCgWaves + w) * kWave + l] = acc[i0 + q];
    __syncthreads();
    if (t < 4 * kWave) {
      const int q = t >> 6;
      const int i = i0 + q;
      double tot = 0.0;
      for (int ww = 0; ww < kCgWaves; ++ww) tot += gs[(q * kCgWaves + ww) * kWave + l];
      if (i < A.n1 && rc < A.R) out[((int64_t)blockIdx.x * A.n1 + i) * A.R + rc] = tot;
    }
  }
}

// u = Sinv g for the block's 64 columns into us[i][l] (gs, us in LDS), then
// gu[l] = g.u per column.  g is read from A.g.
template <int NI>
__device__ void solve_small(const CgArgs& A, double* gs, double* us, double* gu) {
  const int t = threadIdx.x;
  const int l = t & 63;
  const int rc = blockIdx.y * kWave + l;
  for (int idx = t; idx < A.n1 * kWave; idx += blockDim.x) {
    const int i = idx >> 6, ll = idx & 63;
    const int r = blockIdx.y * kWave + ll;
    gs[i * kWave + ll] = r < A.R ? A.g[(int64_t)i * A.R + r] : 0.0;
  }
  __syncthreads();
  for (int idx = t; idx < A.n1 * kWave; idx += blockDim.x) {
    const int i = idx >> 6, ll = idx & 63;
    double u = 0.0;
    for (int j = 0; j < A.n1; ++j) u += A.Sinv[i * A.n1 + j] * gs[j * kWave + ll];
    us[i * kWave + ll] = u;
  }
  __syncthreads();
  if (t < kWave) {
    double d = 0.0;
    for (int i = 0; i < A.n1; ++i) d += gs[i * kWave + t] * us[i * kWave + t];
    gu[t] = d;
  }
  __syncthreads();
  (void)rc;
}

// z_a = M^{-1} r at row a, column lane: (r - F_a . u) / c.
template <int NI>
__device__ __forceinline__ double apply_prec(const CgArgs& A, int64_t a, double r, const double* us) {
  if (NI == 0) return r;
  const int lane = lane_id();
  const double* Fa = A.F + a * (int64_t)A.n1;
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NI; ++i)
    if (i < A.n1) s += Fa[i] * us[i * kWave + lane];
  return (r - s) * A.inv_c;
}

// Q = A P (with the factored operator: Q = K_core P, and F^T P partials),
// partial p.q per column.
template <int NI>
__global__ __launch_bounds__(kCgBlock) void k_cg_spmm(const CgArgs* __restrict__ AA) {
  const CgArgs& A = AA[blockIdx.z];
  if (*A.st.done || *A.st.it >= A.max_iter) return;
  __shared__ double scratch[kCgBlock];
  __shared__ double gsh[NI > 0 ? 4 * kCgBlock : 1];
  const int lane = lane_id();
  const int rc = blockIdx.y * kWave + lane;
  const int rcc = rc < A.R ? rc : A.R - 1;
  const int64_t R = A.R;
  double pq = 0.0;
  double gacc[NI > 0 ? NI : 1];
#pragma unroll
  for (int i = 0; i < (NI > 0 ? NI : 1); ++i) gacc[i] = 0.0;
  const bool lr = NI > 0 && A.lowrank_op;
  for (RowSweep w(A.n, kCgWaves); w.a < w.hi; w.a += w.step) {
    const int64_t a = A.sched ? (int64_t)A.sched[w.a] : w.a;
    const double q = row_dot(A.row_ptr[a], A.row_ptr[a + 1], A.col, A.val, A.P + rcc, R);
    if (rc < A.R) {
      A.Q[a * R + rc] = q;
      const double pa = A.P[a * R + rc];
      pq += pa * q;
      if (lr) {
        const double* Fa = A.F + a * (int64_t)A.n1;
#pragma unroll
        for (int i = 0; i < (NI > 0 ? NI : 1); ++i)
          if (i < A.n1) gacc[i] += Fa[i] * pa;
      }
    }
  }
  block_partial(pq, scratch, A.part, A.R, A.R);
  if (lr) block_partial_g<NI>(gacc, gsh, A, A.partg);
}

// out[i][r] = sum_b partg[b][i][r] (fixed order); grid (n1, chunks).
__global__ __launch_bounds__(kCgBlock) void k_cg_reduce_g(const CgArgs* __restrict__ AA, int which) {
  const CgArgs& A = AA[blockIdx.z];
  if (*A.st.done || *A.st.it >= A.max_iter) return;
  double* __restrict__ out = which == 0 ? A.gp : A.g;
  __shared__ double scratch[kCgBlock];
  const int i = blockIdx.x;
  const int t = threadIdx.x;
  const int l = t & 63, w = t >> 6;
  const int rc = blockIdx.y * kWave + l;
  double s = 0.0;
  if (rc < A.R)
    for (int b = w; b < A.nb; b += kCgWaves) s += A.partg[((int64_t)b * A.n1 + i) * A.R + rc];
  scratch[w * kWave + l] = s;
  __syncthreads();
  if (t < kWave && rc < A.R) {
    double tot = 0.0;
    for (int q = 0; q < kCgWaves; ++q) tot += scratch[q * kWave + t];
    out[(int64_t)i * A.R + rc] = tot;
  }
}

// One row of the x/r update (lane = column): returns the new residual.
template <int NI>
__device__ __forceinline__ void xr_row(const CgArgs& A, int64_t a, int rc, double alpha, const double* gpl,
                                       double& rr, double* gacc) {
  const int64_t o = a * (int64_t)A.R + rc;
  double q = A.Q[o];
  const double* Fa = A.F + a * (int64_t)A.n1;
  if (NI > 0 && A.lowrank_op) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < (NI > 0 ? NI : 1); ++i)
      if (i < A.n1) s += Fa[i] * gpl[i * kWave + (rc & 63)];
    q += s;
  }
  A.X[o] += alpha * A.P[o];
  const double r = A.Rr[o] - alpha * q;
  A.Rr[o] = r;
  rr += r * r;
  if (NI > 0 && A.use_pc) {
#pragma unroll
    for (int i = 0; i < (NI > 0 ? NI : 1); ++i)
      if (i < A.n1) gacc[i] += Fa[i] * r;
  }
}

// alpha = r.z / p.A p; x += alpha p; r -= alpha A p; partials r.r and F^T r.
// With the factored operator p.A p = p.(K_core p) + |F^T p|^2 and
// A p = K_core p + F (F^T p) is completed here on the fly.
template <int NI>
__global__ __launch_bounds__(kCgBlock) void k_cg_update_xr(const CgArgs* __restrict__ AA) {
  const CgArgs& A = AA[blockIdx.z];
  if (*A.st.done) return;
  const int it = *A.st.it;
  if (it >= A.max_iter) return;
  __shared__ double scratch[kCgBlock];
  __shared__ double pAp[kWave];
  __shared__ double gsh[NI > 0 ? 4 * kCgBlock : 1];
  __shared__ double gpl[NI > 0 ? NI * kWave : 1];
  chunk_reduce(A.part, A.nb, A.R, A.R, pAp, scratch);
  const int lane = lane_id();
  const int rc = blockIdx.y * kWave + lane;
  if (NI > 0 && A.lowrank_op) {
    for (int idx = threadIdx.x; idx < A.n1 * kWave; idx += blockDim.x) {
      const int i = idx >> 6, ll = idx & 63;
      const int r = blockIdx.y * kWave + ll;
      gpl[i * kWave + ll] = r < A.R ? A.gp[(int64_t)i * A.R + r] : 0.0;
    }
    __syncthreads();
    if (threadIdx.x < kWave) {
      double gg = 0.0;
      for (int i = 0; i < A.n1; ++i) gg += gpl[i * kWave + threadIdx.x] * gpl[i * kWave + threadIdx.x];
      pAp[threadIdx.x] += gg;
    }
    __syncthreads();
  }
  const int par = it & 1;
  double alpha = 0.0;
  bool act = false;
  if (rc < A.R) {
    act = A.st.act[par * A.R + rc] != 0;
    if (act) {
      const double d = pAp[lane];
      if (d > 0.0 && isfinite(d)) alpha = A.st.rz[par * A.R + rc] / d;
      else act = false;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < kWave && rc < A.R) {
    const bool was = A.st.act[par * A.R + rc] != 0;
    if (was) A.st.hist_a[(int64_t)it * A.R + rc] = alpha;
    if (was && !act) { A.st.failed[rc] = 1; *A.st.not_spd = 1; }
  }
  const int64_t W = (int64_t)gridDim.x * kCgWaves;
  double rr = 0.0;
  double gacc[NI > 0 ? NI : 1];
#pragma unroll
  for (int i = 0; i < (NI > 0 ? NI : 1); ++i) gacc[i] = 0.0;
  if (act) {
    // two rows in flight per wave
    int64_t a = blockIdx.x * (int64_t)kCgWaves + (threadIdx.x >> 6);
    for (; a + W < A.n; a += 2 * W) {
      xr_row<NI>(A, a, rc, alpha, gpl, rr, gacc);
      xr_row<NI>(A, a + W, rc, alpha, gpl, rr, gacc);
    }
    if (a < A.n) xr_row<NI>(A, a, rc, alpha, gpl, rr, gacc);
  }
  block_partial(rr, scratch, A.part2, A.R, A.R);
  if (NI > 0 && A.use_pc) block_partial_g<NI>(gacc, gsh, A, A.partg);
}

// beta = r.z_new / r.z; convergence on |r|; p = z + beta p with
// z = M^{-1} r formed on the fly (r.z_new = (r.r - g.u)/c, g = F^T r,
// u = (cI + F^T F)^{-1} g, so no extra pass is needed).
template <int NI>
__global__ __launch_bounds__(kCgBlock) void k_cg_update_p(const CgArgs* __restrict__ AA) {
  const CgArgs& A = AA[blockIdx.z];
  if (*A.st.done) return;
  const int it = *A.st.it;
  if (it >= A.max_iter) return;
  __shared__ double scratch[kCgBlock];
  __shared__ double rrn[kWave];
  __shared__ double gu[kWave];
  __shared__ double gs[NI > 0 ? NI * kWave : 1];
  __shared__ double us[NI > 0 ? NI * kWave : 1];
  chunk_reduce(A.part2, A.nb, A.R, A.R, rrn, scratch);
  const bool pc = NI > 0 && A.use_pc;
  if (pc) solve_small<NI>(A, gs, us, gu);
  const int lane = lane_id();
  const int rc = blockIdx.y * kWave + lane;
  const int par = it & 1, nxt = par ^ 1;
  double beta = 0.0;
  bool cont = false;
  bool act = false;
  double rz_new = 0.0, rz_old = 0.0;
  if (rc < A.R) {
    act = A.st.act[par * A.R + rc] != 0 && A.st.failed[rc] == 0;
    rz_old = A.st.rz[par * A.R + rc];
    const double rr_new = rrn[lane];
    rz_new = pc ? (rr_new - gu[lane]) * A.inv_c : rr_new;
    if (act) {
      beta = rz_new / rz_old;
      cont = !(rr_new <= A.rtol2 * A.st.bnorm2[rc]);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < kWave && rc < A.R) {
    A.st.rz[nxt * A.R + rc] = act ? rz_new : rz_old;
    A.st.act[nxt * A.R + rc] = cont ? 1 : 0;
    if (act) {
      A.st.hist_b[(int64_t)it * A.R + rc] = beta;
      A.st.iters[rc] += 1;
      A.st.rr_last[rc] = rrn[lane];
    }
  }
  const int64_t R = A.R;
  const int64_t W = (int64_t)gridDim.x * kCgWaves;
  if (cont) {
    int64_t a = blockIdx.x * (int64_t)kCgWaves + (threadIdx.x >> 6);
    for (; a + W < A.n; a += 2 * W) {
      const int64_t o0 = a * R + rc, o1 = (a + W) * R + rc;
      const double r0 = A.Rr[o0], r1 = A.Rr[o1];
      const double p0 = A.P[o0], p1 = A.P[o1];
      const double z0 = pc ? apply_prec<NI>(A, a, r0, us) : r0;
      const double z1 = pc ? apply_prec<NI>(A, a + W, r1, us) : r1;
      A.P[o0] = z0 + beta * p0;
      A.P[o1] = z1 + beta * p1;
    }
    if (a < A.n) {
      const int64_t o = a * R + rc;
      A.P[o] = (pc ? apply_prec<NI>(A, a, A.Rr[o], us) : A.Rr[o]) + beta * A.P[o];
    }
  }
}

// Records the executed iteration count in done when no column is active
// (one block, after update_p).
__global__ void k_cg_check(const CgArgs* __restrict__ AA) {
  const CgArgs& A = AA[blockIdx.z];
  if (*A.st.done) return;
  const int it = *A.st.it;
  if (it >= A.max_iter) return;
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

// Right-hand sides and x = 0, r = b.  Probe p (column 1+p) is the Rademacher
// vector w_p of caller row perm[a], or with the preconditioner
// sqrt(c) w_p + F v_p (v_p: n1 Rademacher signs), whose covariance is M.
__global__ void k_cg_init(const CgArgs* __restrict__ AA, const double* __restrict__ ys,
                          const int32_t* __restrict__ perm, int kind, uint64_t seed,
                          const double* __restrict__ dense) {
  const CgArgs& A = AA[blockIdx.z];
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t tot = A.n * (int64_t)A.R;
  if (idx >= tot) return;
  const int64_t a = idx / A.R;
  const int r = (int)(idx % A.R);
  double b;
  if (kind == PK_DENSE) {
    b = dense[idx];
  } else if (r == 0) {
    b = ys[a];
  } else if (kind == PK_IDENTITY) {
    b = (perm[a] == r - 1) ? 1.0 : 0.0;
  } else {
    const uint64_t pbase = (uint64_t)(r - 1) << 32;
    b = (splitmix64_at(seed, pbase + (uint64_t)perm[a] + 1ull) >> 63) ? -1.0 : 1.0;
    if (A.use_pc) {
      double fv = 0.0;
      const double* Fa = A.F + a * (int64_t)A.n1;
      for (int i = 0; i < A.n1; ++i) {
        const double v = (splitmix64_at(seed, pbase + 0xFFFFFFFFull - (uint64_t)i) >> 63) ? -1.0 : 1.0;
        fv += Fa[i] * v;
      }
      b = A.sqrt_c * b + fv;
    }
  }
  A.X[idx] = 0.0;
  A.Rr[idx] = b;
}

// Partials of b.b and F^T b.
template <int NI>
__global__ __launch_bounds__(kCgBlock) void k_cg_norm_part(const CgArgs* __restrict__ AA) {
  const CgArgs& A = AA[blockIdx.z];
  __shared__ double scratch[kCgBlock];
  __shared__ double gsh[NI > 0 ? 4 * kCgBlock : 1];
  const int rc = blockIdx.y * kWave + lane_id();
  const int64_t R = A.R;
  const int64_t W = (int64_t)gridDim.x * kCgWaves;
  double s = 0.0;
  double gacc[NI > 0 ? NI : 1];
#pragma unroll
  for (int i = 0; i < (NI > 0 ? NI : 1); ++i) gacc[i] = 0.0;
  if (rc < A.R)
    for (int64_t a = blockIdx.x * (int64_t)kCgWaves + (threadIdx.x >> 6); a < A.n; a += W) {
      const double v = A.Rr[a * R + rc];
      s += v * v;
      if (NI > 0 && A.use_pc) {
        const double* Fa = A.F + a * (int64_t)A.n1;
#pragma unroll
        for (int i = 0; i < NI; ++i)
          if (i < A.n1) gacc[i] += Fa[i] * v;
      }
    }
  block_partial(s, scratch, A.part2, A.R, A.R);
  if (NI > 0 && A.use_pc) block_partial_g<NI>(gacc, gsh, A, A.partg);
}

// Initial state: p = z0 = M^{-1} b (b when unpreconditioned), V = z0,
// rz0 = b.z0, bnorm2 = b.b.
template <int NI>
__global__ __launch_bounds__(kCgBlock) void k_cg_init_fin(const CgArgs* __restrict__ AA) {
  const CgArgs& A = AA[blockIdx.z];
  __shared__ double scratch[kCgBlock];
  __shared__ double nrm[kWave];
  __shared__ double gu[kWave];
  __shared__ double gs[NI > 0 ? NI * kWave : 1];
  __shared__ double us[NI > 0 ? NI * kWave : 1];
  chunk_reduce(A.part2, A.nb, A.R, A.R, nrm, scratch);
  const bool pc = NI > 0 && A.use_pc;
  if (pc) solve_small<NI>(A, gs, us, gu);
  const int lane = lane_id();
  const int rc = blockIdx.y * kWave + lane;
  if (blockIdx.x == 0 && threadIdx.x < kWave && rc < A.R) {
    const double bb = nrm[lane];
    const double rz0 = pc ? (bb - gu[lane]) * A.inv_c : bb;
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
  const int64_t R = A.R;
  const int64_t W = (int64_t)gridDim.x * kCgWaves;
  if (rc < A.R)
    for (int64_t a = blockIdx.x * (int64_t)kCgWaves + (threadIdx.x >> 6); a < A.n; a += W) {
      const int64_t o = a * R + rc;
      const double z = pc ? apply_prec<NI>(A, a, A.Rr[o], us) : A.Rr[o];
      A.P[o] = z;
      if (A.V) A.V[o] = z;
    }
}

// ------------------------------------------------------------ utilities
__global__ void k_dot_part(const double* __restrict__ a, int64_t sa, const double* __restrict__ b,
                           int64_t sb, int64_t n, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    s += a[i * sa] * b[i * sb];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_probe_bits(const int32_t* __restrict__ perm, int64_t n, int P, uint64_t seed,
                             uint64_t* __restrict__ bits) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  uint64_t m = 0;
  for (int p = 0; p < P; ++p) {
    const uint64_t k = ((uint64_t)p << 32) + (uint64_t)perm[s] + 1ull;
    if (splitmix64_at(seed, k) >> 63) m |= 1ull << p;
  }
  bits[s] = m;
}

// Dense right-hand sides B[b][j] = kappa[t0 + j, b] for a chunk of test rows
// (B zeroed beforehand; every (b, j) is written at most once).
__global__ void k_scatter_chunk(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                const double* __restrict__ val, int64_t t0, int Rc, int64_t nq,
                                double* __restrict__ B) {
  const int64_t j = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  if (j >= Rc || t0 + j >= nq) return;
  const int64_t t = t0 + j;
  for (int64_t k = rp[t] + lane_id(); k < rp[t + 1]; k += kWave) B[(int64_t)col[k] * Rc + j] = val[k];
}

// var[t] = kxx[t] - sum_b kappa[t, b] V[b][j] for the chunk's test rows.
__global__ void k_rowdot_chunk(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                               const double* __restrict__ val, int64_t t0, int Rc, int64_t nq,
                               const double* __restrict__ V, const double* __restrict__ kxx,
                               double* __restrict__ var) {
  const int64_t j = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  if (j >= Rc || t0 + j >= nq) return;
  const int64_t t = t0 + j;
  double s = 0.0;
  for (int64_t k = rp[t] + lane_id(); k < rp[t + 1]; k += kWave) s += val[k] * V[(int64_t)col[k] * Rc + j];
  s = wave_sum(s);
  if (lane_id() == 0) var[t] = kxx[t] - s;
}

// Blocks per column chunk for the CG kernels: about two 1024-thread blocks
// per CU, a multiple of 8 (the XCD-aware row sweep needs it).
// Gershgorin bound: per-block partial maxima of sum_b |A_ab| over rows.
__global__ void k_rowabs_max(const int64_t* __restrict__ rp, const double* __restrict__ val, int64_t n,
                             double* __restrict__ part) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < n; a += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t k = rp[a]; k < rp[a + 1]; ++k) s += fabs(val[k]);
    m = fmax(m, s);
  }
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Rademacher probe block Z[n][P] (caller row perm[a]) and V = Z.
__global__ void k_taylor_init(const int32_t* __restrict__ perm, int64_t n, int P, uint64_t seed,
                              double* __restrict__ Z, double* __restrict__ V) {
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n * P) return;
  const int64_t a = idx / P;
  const int p = (int)(idx % P);
  const uint64_t k = ((uint64_t)p << 32) + (uint64_t)perm[a] + 1ull;
  const double z = (splitmix64_at(seed, k) >> 63) ? -1.0 : 1.0;
  Z[idx] = z;
  V[idx] = z;
}

// V <- V - W / alpha (= C V) and partial sums of Z . V.
__global__ void k_taylor_step(int64_t len, const double* __restrict__ Z, const double* __restrict__ W,
                              double* __restrict__ V, double inv_alpha, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = V[i] - W[i] * inv_alpha;
    V[i] = v;
    s += Z[i] * v;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

inline int cg_nb(int64_t n, int R) {
  const int chunks = (R + kWave - 1) / kWave;
  int64_t nb = std::max<int64_t>(1, 512 / chunks);
  nb = std::min<int64_t>(nb, (n + kCgWaves - 1) / kCgWaves);
  nb = (nb + 7) / 8 * 8;
  return (int)nb;
}

}  // namespace

void posterior_variance(Ctx* c, const Csr& A, const Sorted& s, const Csr& K0, const double* kxx, double rtol,
                        int max_iter, const Precond* pc, double* var, bool* converged) {
  const int64_t n = A.n, n0 = K0.n;
  *converged = true;
  for (int64_t t0 = 0; t0 < n0; t0 += kWave) {
    const int Rc = (int)std::min<int64_t>(kWave, n0 - t0);
    double* B = c->get<double>(S_POST, (size_t)n * Rc);
    SDGP_HIP(hipMemsetAsync(B, 0, (size_t)n * Rc * sizeof(double), c->stream));
    const unsigned g = (unsigned)((Rc + 3) / 4);
    k_scatter_chunk<<<g, 256, 0, c->stream>>>(K0.row_ptr, K0.col, K0.val, t0, Rc, n0, B);
    SDGP_CHECK_LAUNCH();
    CgResult cg = block_cg(c, A, s, nullptr, PK_DENSE, 0, 0, rtol, max_iter, B, Rc, pc, false, nullptr);
    if (cg.not_spd) throw Error(SDGP_ERR_NOT_SPD, "CG met p^T A p <= 0: the covariance is not positive definite");
    if (!cg.converged) *converged = false;
    k_rowdot_chunk<<<g, 256, 0, c->stream>>>(K0.row_ptr, K0.col, K0.val, t0, Rc, n0, cg.X, kxx, var);
    SDGP_CHECK_LAUNCH();
  }
}

double logdet_taylor(Ctx* c, const Csr& A, const Sorted& s, int P, int terms, uint64_t seed, double* alpha_out) {
  require(P >= 1 && P <= 4096, "probes must be 1..4096");
  require(terms >= 1, "terms must be >= 1");
  const int64_t n = A.n;
  const int nbm = (int)std::min<int64_t>(1024, (n + 255) / 256);
  double* pm = c->get<double>(S_RED_PART, std::max(nbm, 1024));
  k_rowabs_max<<<nbm, 256, 0, c->stream>>>(A.row_ptr, A.val, n, pm);
  SDGP_CHECK_LAUNCH();
  std::vector<double> hm(nbm);
  SDGP_HIP(hipMemcpyAsync(hm.data(), pm, nbm * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  double alpha = 0.0;
  for (double v : hm) alpha = std::max(alpha, v);
  require(alpha > 0.0 && std::isfinite(alpha), "matrix has no positive row sums");
  const size_t len = (size_t)n * P;
  double* Z = c->get<double>(S_CG_X, len);
  double* V = c->get<double>(S_CG_R, len);
  double* W = c->get<double>(S_CG_Q, len);
  k_taylor_init<<<(unsigned)((len + 255) / 256), 256, 0, c->stream>>>(s.perm, n, P, seed, Z, V);
  SDGP_CHECK_LAUNCH();
  const int nb = (int)std::min<int64_t>(1024, ((int64_t)len + 255) / 256);
  std::vector<double> hp((size_t)nb * terms);
  double* part = c->get<double>(S_RED_OUT, (size_t)nb * terms);
  for (int k = 1; k <= terms; ++k) {
    spmm(c, A, V, P, W);
    k_taylor_step<<<nb, 256, 0, c->stream>>>((int64_t)len, Z, W, V, 1.0 / alpha, part + (size_t)(k - 1) * nb);
    SDGP_CHECK_LAUNCH();
  }
  SDGP_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  double acc = 0.0;
  for (int k = 1; k <= terms; ++k) {
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += hp[(size_t)(k - 1) * nb + b];
    acc += t / P / k;
  }
  *alpha_out = alpha;
  return (double)n * std::log(alpha) - acc;
}

void spmm(Ctx* c, const Csr& A, const double* X, int R, double* Y) {
  require(R >= 1 && R <= (1 << 20), "R must be in 1..2^20");
  const int64_t cu = std::max(8, c->cu_count);
  if (R == 1) {
    // 16 rows per 256-thread block; about 8 blocks per CU in flight
    int64_t blocks = std::min<int64_t>((A.n + 15) / 16, cu * 8);
    blocks = std::max<int64_t>(8, (blocks + 7) / 8 * 8);
    k_spmv<<<(unsigned)blocks, 256, 0, c->stream>>>(A.n, A.row_ptr, A.col, A.val, X, Y);
    SDGP_CHECK_LAUNCH();
    return;
  }
  const int chunks = (R + kWave - 1) / kWave;
  int64_t blocks = std::min<int64_t>((A.n + 3) / 4, std::max<int64_t>(8, cu * 8 / chunks));
  blocks = std::max<int64_t>(8, (blocks + 7) / 8 * 8);
  dim3 grid((unsigned)blocks, (unsigned)chunks);
  k_spmm<<<grid, 256, 0, c->stream>>>(A.n, A.row_ptr, A.col, A.val, X, R, Y);
  SDGP_CHECK_LAUNCH();
}

double dot_device(Ctx* c, const double* a, int64_t sa, const double* b, int64_t sb, int64_t n) {
  const int nb = (int)std::min<int64_t>(256, (n + 255) / 256);
  double* part = c->get<double>(S_RED_PART, nb);
  k_dot_part<<<nb, 256, 0, c->stream>>>(a, sa, b, sb, n, part);
  SDGP_CHECK_LAUNCH();
  std::vector<double> hp(nb);
  SDGP_HIP(hipMemcpyAsync(hp.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  double s = 0.0;
  for (int i = 0; i < nb; ++i) s += hp[i];
  return s;
}

void probe_bits(Ctx* c, const Sorted& s, int P, uint64_t seed, uint64_t* zbits) {
  k_probe_bits<<<(unsigned)((s.n + 255) / 256), 256, 0, c->stream>>>(s.perm, s.n, P, seed, zbits);
  SDGP_CHECK_LAUNCH();
}

namespace {

// Gram matrix F^T F: block b accumulates rows [b*slab, (b+1)*slab) staged
// 64 at a time in LDS; thread t owns the pairs idx = t, t+256, ...
__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ F, int64_t n, int n1, int64_t slab,
                                              double* __restrict__ part) {
  __shared__ double rows[64 * kMaxN1];
  const int np = n1 * n1;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  const int64_t lo = blockIdx.x * slab, hi = min(n, lo + slab);
  for (int64_t a0 = lo; a0 < hi; a0 += 64) {
    const int cnt = (int)min((int64_t)64, hi - a0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < cnt * n1; idx += blockDim.x) rows[idx] = F[a0 * n1 + idx];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int idx = threadIdx.x + q * 256;
      if (idx < np) {
        const int i = idx / n1, j = idx % n1;
        double s = 0.0;
        for (int k = 0; k < cnt; ++k) s += rows[k * n1 + i] * rows[k * n1 + j];
        acc[q] += s;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = threadIdx.x + q * 256;
    if (idx < np) part[(int64_t)blockIdx.x * np + idx] = acc[q];
  }
}

// One CG iteration for every member (grid z = member).
template <int NI>
void launch_cg_iteration(hipStream_t st, const CgArgs* dA, const CgArgs& h0, dim3 grid, int chunks, int B,
                         Ctx* c) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c != nullptr && c->timing) { e0 = c->event(); SDGP_HIP(hipEventRecord(e0, st)); }
  k_cg_spmm<NI><<<grid, kCgBlock, 0, st>>>(dA);
  SDGP_CHECK_LAUNCH();
  if (c != nullptr && c->timing) {
    e1 = c->event();
    SDGP_HIP(hipEventRecord(e1, st));
    c->spmm_events.push_back({e0, e1});
  }
  if (NI > 0 && h0.lowrank_op) {
    k_cg_reduce_g<<<dim3(h0.n1, chunks, B), kCgBlock, 0, st>>>(dA, 0);
    SDGP_CHECK_LAUNCH();
  }
  k_cg_update_xr<NI><<<grid, kCgBlock, 0, st>>>(dA);
  SDGP_CHECK_LAUNCH();
  if (NI > 0 && h0.use_pc) {
    k_cg_reduce_g<<<dim3(h0.n1, chunks, B), kCgBlock, 0, st>>>(dA, 1);
    SDGP_CHECK_LAUNCH();
  }
  k_cg_update_p<NI><<<grid, kCgBlock, 0, st>>>(dA);
  SDGP_CHECK_LAUNCH();
  k_cg_check<<<dim3(1, 1, B), 256, 0, st>>>(dA);
  SDGP_CHECK_LAUNCH();
}

template <int NI>
void launch_cg_init(hipStream_t st, const CgArgs* dA, const CgArgs& h0, dim3 grid, int chunks, int B) {
  k_cg_norm_part<NI><<<grid, kCgBlock, 0, st>>>(dA);
  SDGP_CHECK_LAUNCH();
  if (NI > 0 && h0.use_pc) {
    k_cg_reduce_g<<<dim3(h0.n1, chunks, B), kCgBlock, 0, st>>>(dA, 1);
    SDGP_CHECK_LAUNCH();
  }
  k_cg_init_fin<NI><<<grid, kCgBlock, 0, st>>>(dA);
  SDGP_CHECK_LAUNCH();
}

void cg_iteration(int NI, hipStream_t st, const CgArgs* dA, const CgArgs& h0, dim3 grid, int chunks, int B,
                  Ctx* c) {
  switch (NI) {
    case 0: launch_cg_iteration<0>(st, dA, h0, grid, chunks, B, c); break;
    case 8: launch_cg_iteration<8>(st, dA, h0, grid, chunks, B, c); break;
    case 16: launch_cg_iteration<16>(st, dA, h0, grid, chunks, B, c); break;
    case 32: launch_cg_iteration<32>(st, dA, h0, grid, chunks, B, c); break;
    default: launch_cg_iteration<64>(st, dA, h0, grid, chunks, B, c); break;
  }
}

}  // namespace

Precond lowrank_precond(Ctx* c, const Sorted& s, const KParams& kp, const Bumps& b) {
  Precond pc;
  const int n1 = kp.n1;
  const int64_t n = s.n;
  const double psi0 = kp.core == SDGP_CORE_KSTAT ? 0.26596152026762178529 : 1.0;
  pc.c = kp.sigma2 * psi0 + kp.noise;
  require(pc.c > 0.0, "the low-rank preconditioner needs sigma2 psi(0) + noise_var > 0");
  pc.n1 = n1;
  pc.F = b.F;
  if (n1 == 0) {
    pc.logdetM = (double)n * std::log(pc.c);
    return pc;
  }
  const int64_t nbk = std::min<int64_t>(256, (n + 4095) / 4096);
  const int64_t slab = (n + nbk - 1) / nbk;
  const int np = n1 * n1;
  double* part = c->get<double>(S_PC_PART, (size_t)nbk * np);
  k_gram<<<(unsigned)nbk, 256, 0, c->stream>>>(b.F, n, n1, slab, part);
  SDGP_CHECK_LAUNCH();
  std::vector<double> hp((size_t)nbk * np);
  SDGP_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  // S = c I + F^T F; Cholesky S = L L^T; ln det S; S^{-1}
  std::vector<double> S((size_t)np, 0.0), L((size_t)np, 0.0), Si((size_t)np, 0.0);
  for (int64_t bb = 0; bb < nbk; ++bb)
    for (int q = 0; q < np; ++q) S[q] += hp[bb * np + q];
  for (int i = 0; i < n1; ++i) S[i * n1 + i] += pc.c;
  double logdetS = 0.0;
  for (int j = 0; j < n1; ++j) {
    double d = S[j * n1 + j];
    for (int k = 0; k < j; ++k) d -= L[j * n1 + k] * L[j * n1 + k];
    require(d > 0.0, "preconditioner factor is not positive definite");
    const double ljj = std::sqrt(d);
    L[j * n1 + j] = ljj;
    logdetS += 2.0 * std::log(ljj);
    for (int i = j + 1; i < n1; ++i) {
      double v = S[i * n1 + j];
      for (int k = 0; k < j; ++k) v -= L[i * n1 + k] * L[j * n1 + k];
      L[i * n1 + j] = v / ljj;
    }
  }
  for (int col = 0; col < n1; ++col) {  // solve L L^T x = e_col
    std::vector<double> y(n1, 0.0);
    for (int i = 0; i < n1; ++i) {
      double v = (i == col) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) v -= L[i * n1 + k] * y[k];
      y[i] = v / L[i * n1 + i];
    }
    for (int i = n1 - 1; i >= 0; --i) {
      double v = y[i];
      for (int k = i + 1; k < n1; ++k) v -= L[k * n1 + i] * Si[k * n1 + col];
      Si[i * n1 + col] = v / L[i * n1 + i];
    }
  }
  double* dSi = c->get<double>(S_PC_SINV, np);
  SDGP_HIP(hipMemcpyAsync(dSi, Si.data(), np * sizeof(double), hipMemcpyHostToDevice, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  pc.Sinv = dSi;
  pc.logdetM = (double)(n - n1) * std::log(pc.c) + logdetS;
  return pc;
}

std::vector<CgResult> block_cg_multi(Ctx* c, const std::vector<CgMember>& mem, const Sorted& s, const double* ys,
                                     int kind, int P, uint64_t seed, double rtol, int max_iter,
                                     const double* dense_rhs, int dense_R, bool keep_v, bool use_graph) {
  const int B = (int)mem.size();
  require(B >= 1 && B <= 65535, "1..65535 members");
  const int64_t n = s.n;
  int R;
  if (kind == PK_DENSE) R = dense_R;
  else if (kind == PK_IDENTITY) R = (int)(1 + n);
  else if (kind == PK_NONE) R = 1;
  else R = 1 + P;
  require(R >= 1, "no right-hand sides");
  require(max_iter >= 1, "cg_max_iter must be >= 1");
  require(rtol > 0.0 && std::isfinite(rtol), "cg_rtol must be > 0");
  require(kind != PK_DENSE || B == 1, "dense right-hand sides take one member");
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
  const int NI = n1 == 0 ? 0 : (n1 <= 8 ? 8 : (n1 <= 16 ? 16 : (n1 <= 32 ? 32 : 64)));
  const size_t NR = (size_t)n * R;
  const int nb = cg_nb(n, R);
  const int chunks = (R + kWave - 1) / kWave;
  double* X = c->get<double>(S_CG_X, NR * B);
  double* Rr = c->get<double>(S_CG_R, NR * B);
  double* Pp = c->get<double>(S_CG_P, NR * B);
  double* Q = c->get<double>(S_CG_Q, NR * B);
  double* V = (use_pc && keep_v) ? c->get<double>(S_CG_V, NR * B) : nullptr;
  double* part = c->get<double>(S_CG_PART, (size_t)nb * R * B);
  double* part2 = c->get<double>(S_CG_PART2, (size_t)nb * R * B);
  double* partg = n1 > 0 ? c->get<double>(S_CG_PARTG, (size_t)nb * n1 * R * B) : nullptr;
  double* g = use_pc ? c->get<double>(S_CG_G, (size_t)n1 * R * B) : nullptr;
  double* gp = use_lr ? c->get<double>(S_CG_GP, (size_t)n1 * R * B) : nullptr;
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
    A.R = R;
    A.row_ptr = Am.row_ptr;
    A.col = Am.col;
    A.val = Am.val;
    A.X = X + m * NR;
    A.Rr = Rr + m * NR;
    A.P = Pp + m * NR;
    A.Q = Q + m * NR;
    A.V = V ? V + m * NR : nullptr;
    A.sched = s.sched;
    A.part = part + (size_t)m * nb * R;
    A.part2 = part2 + (size_t)m * nb * R;
    A.partg = partg ? partg + (size_t)m * nb * n1 * R : nullptr;
    A.g = g ? g + (size_t)m * n1 * R : nullptr;
    A.gp = gp ? gp + (size_t)m * n1 * R : nullptr;
    A.n1 = n1;
    A.use_pc = use_pc ? 1 : 0;
    A.lowrank_op = use_lr ? 1 : 0;
    A.F = n1 > 0 ? p->F : nullptr;
    A.Sinv = use_pc ? p->Sinv : nullptr;
    A.inv_c = use_pc ? 1.0 / p->c : 1.0;
    A.sqrt_c = use_pc ? std::sqrt(p->c) : 1.0;
    A.nb = nb;
    A.max_iter = max_iter;
    A.rtol2 = rtol * rtol;
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
  {
    const int64_t tot = (int64_t)NR;
    const int64_t gx = (tot + 255) / 256;
    require(gx < 0x7fffffff, "n*R too large");
    k_cg_init<<<dim3((unsigned)gx, 1, B), 256, 0, c->stream>>>(dA, ys, s.perm, kind, seed, dense_rhs);
    SDGP_CHECK_LAUNCH();
  }
  dim3 grid(nb, chunks, B);
  switch (NI) {
    case 0: launch_cg_init<0>(c->stream, dA, hA[0], grid, chunks, B); break;
    case 8: launch_cg_init<8>(c->stream, dA, hA[0], grid, chunks, B); break;
    case 16: launch_cg_init<16>(c->stream, dA, hA[0], grid, chunks, B); break;
    case 32: launch_cg_init<32>(c->stream, dA, hA[0], grid, chunks, B); break;
    default: launch_cg_init<64>(c->stream, dA, hA[0], grid, chunks, B); break;
  }
  // iterate; poll the per-member flags now and then
  std::vector<int32_t> flags((size_t)3 * B);
  auto poll = [&](hipStream_t st) -> bool {
    for (int m = 0; m < B; ++m)
      SDGP_HIP(hipMemcpyAsync(&flags[3 * m], hA[m].st.done, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SDGP_HIP(hipStreamSynchronize(st));
    for (int m = 0; m < B; ++m)
      if (flags[3 * m] == 0 && flags[3 * m + 2] < max_iter) return false;
    return true;
  };
  c->spmm_events.clear();
  int launched = 0;
  if (use_graph) {
    // capture k iterations once and replay them: the iteration counters live
    // on the device, so every replay advances the solve; kernels of members
    // that are done, or past max_iter, return at once
    const int k = 8;
    hipStream_t gs = c->graph_stream();
    hipEvent_t ready = c->event();
    SDGP_HIP(hipEventRecord(ready, c->stream));
    SDGP_HIP(hipStreamWaitEvent(gs, ready, 0));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    SDGP_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
    for (int q = 0; q < k; ++q) cg_iteration(NI, gs, dA, hA[0], grid, chunks, B, nullptr);
    SDGP_HIP(hipStreamEndCapture(gs, &graph));
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
      (void)hipGraphDestroy(graph);
      throw Error(SDGP_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    }
    int every = 1;
    bool fin = false;
    while (!fin && launched < max_iter) {
      for (int q = 0; q < every && launched < max_iter; ++q) {
        SDGP_HIP(hipGraphLaunch(exec, gs));
        launched += k;
      }
      fin = poll(gs);
      every = std::min(every * 2, 8);
    }
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    hipEvent_t back = c->event();
    SDGP_HIP(hipEventRecord(back, gs));
    SDGP_HIP(hipStreamWaitEvent(c->stream, back, 0));
  } else {
    int check = 8;
    bool fin = false;
    while (!fin && launched < max_iter) {
      const int upto = std::min(max_iter, launched + check);
      for (; launched < upto; ++launched) cg_iteration(NI, c->stream, dA, hA[0], grid, chunks, B, c);
      fin = poll(c->stream);
      check = std::min(check * 2, 64);
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
    res.X = A.X;
    res.V = A.V;
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
  return out;
}

CgResult block_cg(Ctx* c, const Csr& Am, const Sorted& s, const double* ys, int kind, int P, uint64_t seed,
                  double rtol, int max_iter, const double* dense_rhs, int dense_R, const Precond* pc,
                  bool keep_v, PhaseTimer* t) {
  (void)t;
  std::vector<CgMember> mem(1);
  mem[0].A = Am;
  mem[0].pc = pc;
  return block_cg_multi(c, mem, s, ys, kind, P, seed, rtol, max_iter, dense_rhs, dense_R, keep_v,
                        c->use_graph)[0];
}

namespace {

// Number of eigenvalues of the symmetric tridiagonal T (d, e) below x
// (Sturm sequence of the LDL^T pivots of T - xI).
int sturm_count(const std::vector<double>& d, const std::vector<double>& e, double x) {
  const int m = (int)d.size();
  int cnt = 0;
  double q = d[0] - x;
  if (q < 0.0) ++cnt;
  for (int k = 1; k < m; ++k) {
    if (q == 0.0) q = 1e-300;
    q = d[k] - x - e[k - 1] * e[k - 1] / q;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// e_1^T ln(T) e_1 for the symmetric positive definite tridiagonal T by the
// integral ln(theta) = int_0^inf [1/(1+t) - 1/(theta+t)] dt applied to the
// spectral measure of e_1: with t = exp(s),
//   e_1^T ln(T) e_1 = int_R t [1/(1+t) - e_1^T (T + tI)^{-1} e_1] ds.
// The integrand is analytic in the strip |Im s| < pi (poles at
// s = ln(theta_j) + i pi), so the trapezoidal rule with step h converges like
// exp(-2 pi^2 / h); the tails decay like exp(-|s|) beyond the spectrum.
// e_1^T (T + tI)^{-1} e_1 is the continued fraction of the bottom-up
// pivots of T + tI (O(m) per node).  Returns NaN if T is not positive
// definite; lo/hi receive the extreme Ritz values (bisection).
double quad_log_tridiag(const std::vector<double>& d, const std::vector<double>& e, double* lo, double* hi) {
  const int m = (int)d.size();
  // Gershgorin interval
  double glo = INFINITY, ghi = -INFINITY;
  for (int k = 0; k < m; ++k) {
    const double r = (k > 0 ? std::fabs(e[k - 1]) : 0.0) + (k + 1 < m ? std::fabs(e[k]) : 0.0);
    glo = std::min(glo, d[k] - r);
    ghi = std::max(ghi, d[k] + r);
  }
  if (!(ghi > 0.0) || !std::isfinite(glo) || !std::isfinite(ghi)) return NAN;
  if (sturm_count(d, e, 0.0) != 0) return NAN;          // some theta <= 0
  // extreme eigenvalues by bisection (relative accuracy 1e-10)
  double a = std::max(glo, 0.0), b = ghi;
  for (int it = 0; it < 200 && b - a > 1e-10 * b; ++it) {
    const double mid = 0.5 * (a + b);
    if (sturm_count(d, e, mid) >= 1) b = mid; else a = mid;
  }
  const double tmin = b;
  a = std::max(glo, 0.0);
  b = ghi;
  for (int it = 0; it < 200 && b - a > 1e-10 * b; ++it) {
    const double mid = 0.5 * (a + b);
    if (sturm_count(d, e, mid) >= m) b = mid; else a = mid;
  }
  const double tmax = b;
  *lo = tmin;
  *hi = tmax;
  if (!(tmin > 0.0)) return NAN;
  const double h = 0.4;
  const double s0 = std::log(tmin) - 42.0, s1 = std::log(tmax) + 42.0;
  const int nodes = (int)std::ceil((s1 - s0) / h);
  double acc = 0.0;
  for (int j = 0; j <= nodes; ++j) {
    const double t = std::exp(s0 + j * h);
    double f = d[m - 1] + t;
    for (int k = m - 2; k >= 0; --k) f = d[k] + t - e[k] * e[k] / f;
    acc += t * (1.0 / (1.0 + t) - 1.0 / f);
  }
  return h * acc;
}

}  // namespace

void slq_from_cg(Ctx* c, const CgResult& cg, int kind, int P, int64_t n, int lanczos_steps, double* logdet,
                 double* stderr_out, double* ritz_min, double* ritz_max) {
  (void)P;
  (void)n;
  const int ncols = cg.R - 1;
  if (ncols <= 0) {
    *logdet = 0.0; *stderr_out = 0.0; *ritz_min = 0.0; *ritz_max = 0.0;
    return;
  }
  std::vector<int32_t> its(cg.R);
  std::vector<double> w0(cg.R);
  SDGP_HIP(hipMemcpyAsync(its.data(), cg.col_iters, cg.R * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipMemcpyAsync(w0.data(), cg.rz0, cg.R * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  int mmax = 0;
  for (int r = 1; r < cg.R; ++r) mmax = std::max(mmax, its[r]);
  if (lanczos_steps > 0) mmax = std::min(mmax, lanczos_steps);
  // coefficient history rows 0..mmax-1 (all columns) to the host
  std::vector<double> ha((size_t)std::max(mmax, 1) * cg.R), hb((size_t)std::max(mmax, 1) * cg.R);
  if (mmax > 0) {
    SDGP_HIP(hipMemcpyAsync(ha.data(), cg.hist_a, (size_t)mmax * cg.R * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
    SDGP_HIP(hipMemcpyAsync(hb.data(), cg.hist_b, (size_t)mmax * cg.R * sizeof(double), hipMemcpyDeviceToHost,
                            c->stream));
    SDGP_HIP(hipStreamSynchronize(c->stream));
  }
  std::vector<double> q(ncols), lo(ncols), hi(ncols);
  auto work = [&](int p) {
    const int r = 1 + p;
    int m = its[r];
    if (lanczos_steps > 0) m = std::min(m, lanczos_steps);
    if (m <= 0) { q[p] = 0.0; lo[p] = INFINITY; hi[p] = -INFINITY; return; }
    std::vector<double> d(m), e(std::max(m - 1, 1), 0.0);
    for (int k = 0; k < m; ++k) {
      const double ak = ha[(size_t)k * cg.R + r];
      double dk = 1.0 / ak;
      if (k > 0) dk += hb[(size_t)(k - 1) * cg.R + r] / ha[(size_t)(k - 1) * cg.R + r];
      d[k] = dk;
      if (k + 1 < m) e[k] = std::sqrt(hb[(size_t)k * cg.R + r]) / ak;
    }
    q[p] = quad_log_tridiag(d, e, &lo[p], &hi[p]);
  };
  unsigned hw = std::thread::hardware_concurrency();
  int nt = (int)std::max(1u, std::min(hw == 0 ? 1u : hw, 16u));
  nt = std::min(nt, ncols);
  if (nt <= 1) {
    for (int p = 0; p < ncols; ++p) work(p);
  } else {
    std::vector<std::thread> th;
    std::atomic<int> next(0);
    for (int t = 0; t < nt; ++t)
      th.emplace_back([&] {
        for (int p = next.fetch_add(1); p < ncols; p = next.fetch_add(1)) work(p);
      });
    for (auto& t : th) t.join();
  }
  // weight of probe p: |M^{-1/2} b_p|^2 = b_p^T M^{-1} b_p (|z|^2 without a
  // preconditioner: n for Rademacher, 1 for unit vectors)
  double sum = 0.0, sum2 = 0.0, mn = INFINITY, mx = -INFINITY;
  bool bad = false;
  for (int p = 0; p < ncols; ++p) {
    const double v = w0[1 + p] * q[p];
    if (!std::isfinite(v)) bad = true;
    sum += v;
    sum2 += v * v;
    mn = std::min(mn, lo[p]);
    mx = std::max(mx, hi[p]);
  }
  if (bad) throw Error(SDGP_ERR_NOT_SPD, "Lanczos quadrature met a non-positive Ritz value");
  if (kind == PK_IDENTITY) {
    *logdet = cg.logdetM + sum;
    *stderr_out = 0.0;
  } else {
    const double mean = sum / ncols;
    *logdet = cg.logdetM + mean;
    const double var = ncols > 1 ? std::max(0.0, (sum2 - ncols * mean * mean) / (ncols - 1)) : 0.0;
    *stderr_out = ncols > 1 ? std::sqrt(var / ncols) : NAN;
  }
  *ritz_min = mn;
  *ritz_max = mx;
}

}  // namespace sdgp
