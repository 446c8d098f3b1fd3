// Sparse covariance assembly of the sparsity-discovering kernel
// (Section 2.2 kernel, Section 2.3 sparse assembly) for gfx950.
//
// Points are sorted into a grid of cells whose side is at least the core
// radius, so every core neighbour of a point lies in the 3^dim block of
// cells around it.  For each cell the candidate columns are a sorted list of
// disjoint point intervals: the x-runs of the neighbouring cells, merged
// (SUM combine) with the cell runs of every bump function whose support
// touches the cell.  One wavefront per row sweeps its cell's intervals 64
// columns at a time, tests the support predicate, and compacts the kept
// columns with a ballot + lane prefix count, so rows come out with ascending
// columns and coalesced stores, and no dense block is ever formed.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>

#include "kernel_math.hpp"
#include "sdgp_internal.hpp"

namespace sdgp {

namespace {

constexpr int kBlock = 256;

inline int grid_for(int64_t work, int per_block) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > 0x7fffffff) throw Error(SDGP_ERR_INVALID_ARG, "problem too large for one launch");
  return (int)g;
}

// ---------------------------------------------------------------- ordering
__global__ void k_bbox(const double* __restrict__ x, int64_t n, int dim, double* __restrict__ part) {
  __shared__ double smin[kBlock][kMaxDim];
  __shared__ double smax[kBlock][kMaxDim];
  double lo[kMaxDim], hi[kMaxDim];
  for (int k = 0; k < kMaxDim; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
  for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < n;
       a += (int64_t)gridDim.x * blockDim.x) {
    for (int k = 0; k < dim; ++k) {
      double v = x[a * dim + k];
      lo[k] = fmin(lo[k], v);
      hi[k] = fmax(hi[k], v);
    }
  }
  for (int k = 0; k < kMaxDim; ++k) { smin[threadIdx.x][k] = lo[k]; smax[threadIdx.x][k] = hi[k]; }
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int k = 0; k < kMaxDim; ++k) {
        smin[threadIdx.x][k] = fmin(smin[threadIdx.x][k], smin[threadIdx.x + s][k]);
        smax[threadIdx.x][k] = fmax(smax[threadIdx.x][k], smax[threadIdx.x + s][k]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < kMaxDim; ++k) {
      part[blockIdx.x * 2 * kMaxDim + k] = smin[0][k];
      part[blockIdx.x * 2 * kMaxDim + kMaxDim + k] = smax[0][k];
    }
}

__device__ __forceinline__ int cell_coord(double v, double lo, double inv, int G) {
  double t = (v - lo) * inv;
  int c = (int)t;
  if (t < 0.0) c = 0;
  return c >= G ? G - 1 : c;
}

__global__ void k_cell_keys(const double* __restrict__ x, int64_t n, Grid g,
                            uint32_t* __restrict__ keys, int32_t* __restrict__ idx) {
  int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= n) return;
  int64_t key = 0;
  for (int k = g.dim - 1; k >= 0; --k)
    key = key * g.G[k] + cell_coord(x[a * g.dim + k], g.lo[k], g.inv_side[k], g.G[k]);
  keys[a] = (uint32_t)key;
  idx[a] = (int32_t)a;
}

__global__ void k_cell_start(const uint32_t* __restrict__ keys, int64_t n, int64_t n_cells,
                             int32_t* __restrict__ cell_start) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  int64_t key = keys[s];
  int64_t prev = s > 0 ? (int64_t)keys[s - 1] : -1;
  for (int64_t c = prev + 1; c <= key; ++c) cell_start[c] = (int32_t)s;
  if (s == n - 1)
    for (int64_t c = key + 1; c <= n_cells; ++c) cell_start[c] = (int32_t)n;
}

__global__ void k_gather_points(const double* __restrict__ x, const int32_t* __restrict__ perm,
                                int64_t n, int dim, double4* __restrict__ xs) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  int64_t a = perm[s];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < dim; ++k) v[k] = x[a * dim + k];
  xs[s] = make_double4(v[0], v[1], v[2], v[3]);
}

__global__ void k_gather_vec(const double* __restrict__ src, const int32_t* __restrict__ perm,
                             int64_t n, double* __restrict__ dst) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s < n) dst[s] = src[perm[s]];
}

// Processing schedule: cells in Morton (bit-interleaved) order of their grid
// coordinates, rows of each cell in storage order.  Kernels that gather
// neighbour rows walk this schedule so that consecutive work stays inside a
// compact 3-D block (the storage order itself is untouched).
__device__ __forceinline__ uint64_t spread_bits(uint64_t v, int dim, int nb) {
  uint64_t out = 0;
  for (int b = 0; b < nb; ++b) out |= ((v >> b) & 1ull) << (b * dim);
  return out;
}

struct MortonQ {
  int dim, bits;
  double lo[kMaxDim], scale[kMaxDim];
};

// Morton key of sorted point s: its quantised coordinates, bits interleaved.
__global__ void k_point_morton(const double4* __restrict__ xs, int64_t n, MortonQ q, uint64_t* __restrict__ keys,
                               int32_t* __restrict__ ids) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double4 p = xs[s];
  const double xk[4] = {p.x, p.y, p.z, p.w};
  const double top = (double)((1 << q.bits) - 1);
  uint64_t key = 0;
  for (int k = 0; k < q.dim; ++k) {
    const double t = fmin(fmax((xk[k] - q.lo[k]) * q.scale[k], 0.0), top);
    key |= spread_bits((uint64_t)t, q.dim, q.bits) << k;
  }
  keys[s] = key;
  ids[s] = (int32_t)s;
}

// ------------------------------------------------------------ bump values
// F[s, i] = sum_j a_ij exp(beta_ij - beta_ij / (1 - q_ij(x_s))) over the
// balls that strictly contain x_s (q < 1, decided as |x-c|^2 < r^2), and the
// membership mask M[s] (bit i: x_s inside some ball of bump function i).
// One block of kBlock points: each thread evaluates its point's F values
// 16 bump functions at a time into an LDS tile, and the block writes the
// tile out row-contiguously (16 consecutive lanes per 128-byte row piece),
// so F is written in whole cache lines instead of one 8-byte word per lane
// at a stride of n1 doubles.
constexpr int kFT = 16;   // bump functions per tile

__device__ __forceinline__ void bumps_block(const double4* __restrict__ xs, int64_t n, int dim, int n1, int n2,
                                            const double* __restrict__ bp, double* __restrict__ F,
                                            uint64_t* __restrict__ M) {
  __shared__ double tile[kBlock][kFT + 1];
  const int t = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * kBlock;
  const int64_t s = s0 + t;
  const bool live = s < n;
  const double4 p = live ? xs[s] : make_double4(0.0, 0.0, 0.0, 0.0);
  const int stride = 3 + dim;
  uint64_t m = 0;
  for (int i0 = 0; i0 < n1; i0 += kFT) {
    const int wt = min(kFT, n1 - i0);
    for (int ii = 0; ii < wt; ++ii) {
      const int i = i0 + ii;
      double f = 0.0;
      // balls unrolled by 4 and the axes fully, so the balls' parameter
      // loads are issued together (0.127 -> 0.084 ms at 1M); each sum keeps
      // its order
#pragma unroll 4
      for (int j = 0; j < n2; ++j) {
        const double* q = bp + (i * n2 + j) * stride;
        double d2 = 0.0;
#pragma unroll
        for (int k = 0; k < kMaxDim; ++k) {
          if (k < dim) {
            double d = comp(p, k) - q[3 + k];
            d2 += d * d;
          }
        }
        const double r2 = q[2] * q[2];
        if (d2 < r2) {
          const double qq = d2 / r2;
          f += q[0] * exp(q[1] - q[1] / (1.0 - qq));
          m |= (1ull << i);
        }
      }
      tile[t][ii] = f;
    }
    __syncthreads();
    for (int e = t; e < kBlock * wt; e += kBlock) {
      const int r = e / wt, cc = e - r * wt;
      if (s0 + r < n) F[(s0 + r) * n1 + i0 + cc] = tile[r][cc];
    }
    __syncthreads();
  }
  if (live) M[s] = m;
}

__global__ __launch_bounds__(kBlock) void k_bumps(const double4* __restrict__ xs, int64_t n, int dim, int n1,
                                                  int n2, const double* __restrict__ bp, double* __restrict__ F,
                                                  uint64_t* __restrict__ M) {
  bumps_block(xs, n, dim, n1, n2, bp, F, M);
}

// Per-member storage of the population assembly: every population kernel
// runs member blockIdx.z on its own bump parameters and outputs.
struct PopMember {
  const double* bp;          // bump parameters
  double* F;                 // [n, n1]
  uint64_t* M;               // [n]
  uint64_t* cm;              // [n_cells] cell masks
  const int32_t* run_ptr;    // [n1 + 1], offsets into runs
  const int4* runs;          // bump-function cell runs of all members
  int32_t* iv_cnt;           // [n_cells + 1]
  const int32_t* iv_ptr;     // [n_cells + 1]
  int2* iv;                  // candidate intervals
  int64_t* row_nnz;          // [n + 1]
  const int64_t* row_ptr;    // [n + 1]
  int32_t* col;
  double* val;
  unsigned long long* cand;  // candidate-pair counter
};

__global__ __launch_bounds__(kBlock) void k_bumps_pop(const double4* __restrict__ xs, int64_t n, int dim, int n1,
                                                      int n2, const PopMember* __restrict__ pm) {
  const PopMember& P = pm[blockIdx.z];
  bumps_block(xs, n, dim, n1, n2, P.bp, P.F, P.M);
}

// ---------------------------------------------------------------- pruning
__global__ void k_cellmask(const int32_t* __restrict__ cell_start, int64_t n_cells,
                           const uint64_t* __restrict__ M, uint64_t* __restrict__ cm) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= n_cells) return;
  uint64_t m = 0;
  for (int32_t s = cell_start[c]; s < cell_start[c + 1]; ++s) m |= M[s];
  cm[c] = m;
}

__global__ void k_cellmask_pop(const int32_t* __restrict__ cell_start, int64_t n_cells,
                               const PopMember* __restrict__ pm) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= n_cells) return;
  const PopMember& P = pm[blockIdx.z];
  uint64_t m = 0;
  for (int32_t s = cell_start[c]; s < cell_start[c + 1]; ++s) m |= P.M[s];
  P.cm[c] = m;
}

// Runs of consecutive cells whose mask has bit i, for every bump function
// (grid y) of every member (grid z), all in parallel: k_run_flags marks the
// cells that start a run, one exclusive scan over the flags of all
// (member, function, cell) triples gives every run its slot, and
// k_run_write puts a run's first cell at its slot and its last cell at the
// slot of the run it closes (the number of run starts up to and including
// that cell, minus one).  The runs of function i of member z are
// runs[pos[(z n1 + i) nc] .. pos[(z n1 + i + 1) nc]).
__device__ __forceinline__ bool cell_bit(const uint64_t* __restrict__ cm, int64_t c, int i) {
  return (cm[c] >> i) & 1ull;
}

__global__ void k_run_flags(const uint64_t* __restrict__ cm, int64_t nc, int n1, int32_t* __restrict__ flag) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const int i = blockIdx.y;
  const uint64_t* m = cm + (int64_t)blockIdx.z * nc;
  const bool f = cell_bit(m, c, i);
  const bool fp = c > 0 && cell_bit(m, c - 1, i);
  flag[((int64_t)blockIdx.z * n1 + i) * nc + c] = (f && !fp) ? 1 : 0;
}

__global__ void k_run_write(const uint64_t* __restrict__ cm, int64_t nc, int n1, const int32_t* __restrict__ pos,
                            const int32_t* __restrict__ cell_start, int4* __restrict__ runs) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const int i = blockIdx.y;
  const uint64_t* m = cm + (int64_t)blockIdx.z * nc;
  if (!cell_bit(m, c, i)) return;
  const bool fp = c > 0 && cell_bit(m, c - 1, i);
  const bool fn = c + 1 < nc && cell_bit(m, c + 1, i);
  const int32_t p = pos[((int64_t)blockIdx.z * n1 + i) * nc + c];
  if (!fp) {
    runs[p].x = (int)c;
    runs[p].z = cell_start[c];
  }
  if (!fn) {
    runs[fp ? p - 1 : p].y = (int)c;
    runs[fp ? p - 1 : p].w = cell_start[c + 1];
  }
}

// run_ptr[z (n1 + 1) + i] = pos[(z n1 + i) nc] for i <= n1 (offsets into
// the one run array of all members).
__global__ void k_run_ptr(const int32_t* __restrict__ pos, int64_t nc, int n1, int B,
                          int32_t* __restrict__ run_ptr) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)B * (n1 + 1)) return;
  const int64_t z = e / (n1 + 1), i = e % (n1 + 1);
  run_ptr[e] = pos[(z * n1 + i) * nc];
}

struct IvArgs {
  Grid g;
  const int32_t* cell_start;
  const uint64_t* cm;
  const int32_t* run_ptr;   // [n1 + 1], null for PRODUCT
  const int4* runs;         // cell runs (first cell, last cell) with their point bounds
  int use_bumps;
  int n1 = 0;               // bump functions (0: the runs are not staged in LDS)
};

// Bump-function runs staged in LDS by the interval kernels (when they fit).
constexpr int kRunLds = 2048;

// Merged candidate intervals of one query (a training cell, or a test point
// placed in its clamped cell).  Lists: the x-runs of the neighbouring cells
// (ascending by construction) and, when bumps are used, the runs of every
// bump function in `mask`.  A k-way merge emits maximal disjoint point
// intervals in ascending order; returns their number and, when kFill, writes
// them to out.  Every run carries its point bounds (bump runs from their
// construction, core runs loaded when the merge reaches them), so a merged
// cell run is converted to points without further loads.  The bump runs are
// read from `runs` at A.run_ptr offsets minus run_base (A.runs itself, or a
// copy staged in LDS); up to kRegLists bump lists (all but rare cells) are
// merged with their positions and next runs in registers (the general
// path's per-list arrays live in scratch memory).
template <bool kFill>
__device__ int merge_intervals(const IvArgs& A, const int* cc, uint64_t mask, const int4* runs, int run_base,
                               int2* __restrict__ out) {
  const int dim = A.g.dim;
  // core x-runs enumerated with the highest axis outermost -> ascending
  int n_off = 1;
  for (int k = 1; k < dim; ++k) n_off *= 3;
  const int xlo = cc[0] > 0 ? cc[0] - 1 : 0;
  const int xhi = cc[0] + 1 < A.g.G[0] ? cc[0] + 1 : A.g.G[0] - 1;

  // bump lists of the query
  constexpr int kRegLists = 4;
  const int nl = A.use_bumps ? __popcll(mask) : 0;
  const bool in_regs = nl <= kRegLists;
  int lst_pos[kMaxN1], lst_end[kMaxN1];    // more than kRegLists lists
  int rpos[kRegLists], rend[kRegLists];    // up to kRegLists lists
  int4 rhead[kRegLists];
  {
    uint64_t m = mask;
#pragma unroll
    for (int l = 0; l < kRegLists; ++l) {
      rpos[l] = rend[l] = 0;
      rhead[l] = make_int4(0, 0, 0, 0);
      if (in_regs && l < nl) {
        const int i = __builtin_ctzll(m);
        m &= m - 1;
        rpos[l] = A.run_ptr[i] - run_base;
        rend[l] = A.run_ptr[i + 1] - run_base;
        if (rpos[l] < rend[l]) rhead[l] = runs[rpos[l]];
      }
    }
    if (!in_regs) {
      m = mask;
      for (int l = 0; l < nl; ++l) {
        const int i = __builtin_ctzll(m);
        m &= m - 1;
        lst_pos[l] = A.run_ptr[i] - run_base;
        lst_end[l] = A.run_ptr[i + 1] - run_base;
      }
    }
  }
  int core_k = 0;  // next core offset index
  auto core_run = [&](int k, int64_t& lo, int64_t& hi) -> bool {
    // offset digits (base 3) for axes 1..dim-1, lowest axis fastest
    int64_t base = 0;
    int64_t mul = A.g.G[0];
    int t = k;
    for (int ax = 1; ax < dim; ++ax) {
      const int o = t % 3 - 1;
      t /= 3;
      const int v = cc[ax] + o;
      if (v < 0 || v >= A.g.G[ax]) return false;
      base += (int64_t)v * mul;
      mul *= A.g.G[ax];
    }
    lo = base + xlo;
    hi = base + xhi;
    return true;
  };
  int64_t next_core_lo = -1, next_core_hi = -1;
  int32_t next_core_s = 0, next_core_e = 0;
  auto advance_core = [&]() {
    next_core_lo = -1;
    while (core_k < n_off) {
      int64_t lo, hi;
      const bool ok = core_run(core_k, lo, hi);
      ++core_k;
      if (ok) {
        next_core_lo = lo;
        next_core_hi = hi;
        next_core_s = A.cell_start[lo];
        next_core_e = A.cell_start[hi + 1];
        return;
      }
    }
  };
  advance_core();

  int count = 0;
  int64_t cur_lo = -1, cur_hi = -1;        // current merged cell run
  int32_t cur_s = 0, cur_e = 0;            // its point bounds
  int32_t last_s = -1, last_e = -1;        // last point interval (pending)
  auto flush_point = [&](int32_t s, int32_t e) {
    if (e <= s) return;
    if (last_e == s) { last_e = e; return; }
    if (last_s >= 0) {
      if (kFill) out[count] = make_int2(last_s, last_e);
      ++count;
    }
    last_s = s;
    last_e = e;
  };
  for (;;) {
    // pick the list whose next run starts lowest
    int64_t best_lo = -1, best_hi = -1;
    int32_t best_s = 0, best_e = 0;
    int best = -2;
    if (next_core_lo >= 0) {
      best_lo = next_core_lo;
      best_hi = next_core_hi;
      best_s = next_core_s;
      best_e = next_core_e;
      best = -1;
    }
    if (in_regs) {
#pragma unroll
      for (int l = 0; l < kRegLists; ++l) {
        if (rpos[l] < rend[l] && (best == -2 || rhead[l].x < best_lo)) {
          best_lo = rhead[l].x;
          best_hi = rhead[l].y;
          best_s = rhead[l].z;
          best_e = rhead[l].w;
          best = l;
        }
      }
    } else {
      for (int l = 0; l < nl; ++l) {
        if (lst_pos[l] < lst_end[l]) {
          const int4 r = runs[lst_pos[l]];
          if (best == -2 || r.x < best_lo) {
            best_lo = r.x;
            best_hi = r.y;
            best_s = r.z;
            best_e = r.w;
            best = l;
          }
        }
      }
    }
    if (best == -2) break;
    if (best == -1) {
      advance_core();
    } else if (in_regs) {
#pragma unroll
      for (int l = 0; l < kRegLists; ++l)
        if (l == best && ++rpos[l] < rend[l]) rhead[l] = runs[rpos[l]];
    } else {
      ++lst_pos[best];
    }
    if (cur_lo < 0) {
      cur_lo = best_lo; cur_hi = best_hi; cur_s = best_s; cur_e = best_e;
    } else if (best_lo <= cur_hi + 1) {
      if (best_hi > cur_hi) { cur_hi = best_hi; cur_e = best_e; }
    } else {
      flush_point(cur_s, cur_e);
      cur_lo = best_lo; cur_hi = best_hi; cur_s = best_s; cur_e = best_e;
    }
  }
  if (cur_lo >= 0) flush_point(cur_s, cur_e);
  if (last_s >= 0) {
    if (kFill) out[count] = make_int2(last_s, last_e);
    ++count;
  }
  return count;
}

// The bump runs A.runs[A.run_ptr[0] .. A.run_ptr[n1]) in LDS when they fit
// (every thread of the block calls this); returns the runs to read and sets
// base to the offset to subtract from run_ptr values.
__device__ __forceinline__ const int4* stage_runs(const IvArgs& A, int4* lds, int& base) {
  base = 0;
  if (!A.use_bumps || A.n1 <= 0) return A.runs;
  const int b0 = A.run_ptr[0], total = A.run_ptr[A.n1] - b0;
  if (total > kRunLds) return A.runs;
  for (int e = threadIdx.x; e < total; e += blockDim.x) lds[e] = A.runs[b0 + e];
  __syncthreads();
  base = b0;
  return lds;
}

template <bool kFill>
__global__ void k_cell_intervals(IvArgs A, int32_t* __restrict__ iv_cnt,
                                 const int32_t* __restrict__ iv_ptr, int2* __restrict__ iv) {
  __shared__ int4 sruns[kRunLds];
  int base = 0;
  const int4* runs = stage_runs(A, sruns, base);
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= A.g.n_cells) return;
  int cc[kMaxDim];
  {
    int64_t r = c;
    for (int k = 0; k < A.g.dim; ++k) { cc[k] = (int)(r % A.g.G[k]); r /= A.g.G[k]; }
  }
  const uint64_t mask = A.use_bumps ? A.cm[c] : 0ull;
  if (mask != 0) return;                      // k_cell_intervals_wave's cell
  const int cnt = merge_intervals<kFill>(A, cc, mask, runs, base, kFill ? iv + iv_ptr[c] : nullptr);
  if (!kFill) iv_cnt[c] = cnt;
}

// Cell run k of the 3^(dim-1) core runs of cell cc (x-runs xlo..xhi of the
// neighbouring rows, the highest axis outermost: ascending in k); false when
// the row lies outside the grid.
__device__ __forceinline__ bool core_run_of(const IvArgs& A, const int* cc, int xlo, int xhi, int k, int64_t& lo,
                                            int64_t& hi) {
  int64_t base = 0;
  int64_t mul = A.g.G[0];
  int t = k;
  for (int ax = 1; ax < A.g.dim; ++ax) {
    const int o = t % 3 - 1;
    t /= 3;
    const int v = cc[ax] + o;
    if (v < 0 || v >= A.g.G[ax]) return false;
    base += (int64_t)v * mul;
    mul *= A.g.G[ax];
  }
  lo = base + xlo;
  hi = base + xhi;
  return true;
}

// Inclusive prefix maximum over the wavefront's lanes.
__device__ __forceinline__ int64_t wave_incl_max(int64_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t u = __shfl_up(v, o, kWave);
    if (lane >= o) v = u > v ? u : v;
  }
  return v;
}

// The merged candidate intervals of one cell by a whole wavefront (every
// lane calls it), with the serial merge's result: the cell's core runs and
// bump lists (runs with their point bounds) are gathered into buf (LDS,
// kWaveRuns entries), sorted by first cell (bitonic), merged into cell runs
// by a prefix maximum of the last cells (a run starts a new merged run when
// it begins more than one cell after every earlier run ends), and the merged
// runs' point intervals are chained where they touch.  Returns -1 when the
// runs do not fit in buf.
constexpr int kWaveRuns = 512;
template <bool kFill>
__device__ int merge_wave(const IvArgs& A, const int* cc, uint64_t mask, int4* buf, int2* __restrict__ out) {
  const int lane = lane_id();
  int n_off = 1;
  for (int k = 1; k < A.g.dim; ++k) n_off *= 3;
  const int xlo = cc[0] > 0 ? cc[0] - 1 : 0;
  const int xhi = cc[0] + 1 < A.g.G[0] ? cc[0] + 1 : A.g.G[0] - 1;
  int T = n_off;                               // upper bound first: every core run
  for (uint64_t m = mask; m; m &= m - 1) {
    const int i = __builtin_ctzll(m);
    T += A.run_ptr[i + 1] - A.run_ptr[i];
  }
  if (T > kWaveRuns) return -1;
  // 1. gather: the core runs that exist, then every bump list
  T = 0;
  {
    int64_t lo = 0, hi = 0;
    const bool ok = lane < n_off && core_run_of(A, cc, xlo, xhi, lane, lo, hi);   // n_off <= 27
    const uint64_t bal = ballot64(ok);
    if (ok) buf[lanes_below(bal)] = make_int4((int)lo, (int)hi, A.cell_start[lo], A.cell_start[hi + 1]);
    T = __popcll(bal);
  }
  for (uint64_t m = mask; m; m &= m - 1) {
    const int i = __builtin_ctzll(m);
    const int p0 = A.run_ptr[i], len = A.run_ptr[i + 1] - p0;
    for (int e = lane; e < len; e += kWave) buf[T + e] = A.runs[p0 + e];
    T += len;
  }
  // 2. bitonic sort by first cell over a power of two, padded with runs past every cell
  int P = 1;
  while (P < T) P <<= 1;
  for (int e = T + lane; e < P; e += kWave) buf[e] = make_int4(0x7fffffff, 0x7fffffff, 0, 0);
  __builtin_amdgcn_wave_barrier();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < P; i += kWave) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const int4 a = buf[i], b = buf[ixj];
          if ((a.x > b.x) == ((i & k) == 0)) {
            buf[i] = b;
            buf[ixj] = a;
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  // 3. merged cell runs, written over buf from the front (group g <= run i):
  // key = (last cell, its end point bound) so the maximum carries the bound
  int64_t kmax = INT64_MIN;                    // over all runs so far (uniform)
  int ng = 0;                                  // merged runs so far (uniform)
  for (int c0 = 0; c0 < T; c0 += kWave) {
    const int i = c0 + lane;
    const bool valid = i < T;
    const int4 r = valid ? buf[i] : make_int4(0, 0, 0, 0);
    const int64_t key = valid ? ((int64_t)r.y << 32 | (uint32_t)r.w) : INT64_MIN;
    const int64_t incl = wave_incl_max(key);
    int64_t excl = __shfl_up(incl, 1, kWave);
    if (lane == 0) excl = INT64_MIN;
    if (kmax > excl) excl = kmax;
    const bool start = valid && (excl == INT64_MIN || (excl >> 32) < (int64_t)r.x - 1);
    const uint64_t sb = ballot64(start);
    const int g = ng + lanes_below(sb);        // this run's merged run when it starts one
    __builtin_amdgcn_wave_barrier();           // every run of the chunk is read
    if (start) {
      buf[g].x = r.x;                          // first cell and first point
      buf[g].z = r.z;
      if (g > 0) {                             // the previous merged run ends here
        buf[g - 1].y = (int)(excl >> 32);
        buf[g - 1].w = (int)(uint32_t)excl;
      }
    }
    ng += __popcll(sb);
    const int64_t cm = (int64_t)readlane_u64((uint64_t)incl, kWave - 1);
    if (cm > kmax) kmax = cm;
    __builtin_amdgcn_wave_barrier();
  }
  if (lane == 0 && ng > 0) {
    buf[ng - 1].y = (int)(kmax >> 32);
    buf[ng - 1].w = (int)(uint32_t)kmax;
  }
  __builtin_amdgcn_wave_barrier();
  // 4. point intervals: empty merged runs dropped, touching ones chained
  int64_t last_e = -1;                         // end of the last non-empty merged run (uniform)
  int nout = 0;
  for (int g0 = 0; g0 < ng; g0 += kWave) {
    const int g = g0 + lane;
    const bool valid = g < ng;
    const int4 q = valid ? buf[g] : make_int4(0, 0, 0, 0);
    const bool nonempty = valid && q.w > q.z;
    const int64_t v = nonempty ? (int64_t)q.w : -1;
    const int64_t incl = wave_incl_max(v);
    int64_t excl = __shfl_up(incl, 1, kWave);
    if (lane == 0) excl = -1;
    if (last_e > excl) excl = last_e;
    const bool start = nonempty && excl != (int64_t)q.z;
    const uint64_t sb = ballot64(start);
    const int o = nout + lanes_below(sb);
    if (kFill && start) {
      out[o].x = q.z;
      if (o > 0) out[o - 1].y = (int)excl;
    }
    nout += __popcll(sb);
    const int64_t cm = (int64_t)readlane_u64((uint64_t)incl, kWave - 1);
    if (cm > last_e) last_e = cm;
  }
  if (kFill && lane == 0 && nout > 0) out[nout - 1].y = (int)last_e;
  return nout;
}

// Cells with bump lists: one wavefront per cell (kWaveCells cells per
// wavefront, in turn; one keeps the slowest wavefront at one cell), the
// merge shared by the wavefront; cells whose runs do not fit in LDS are
// merged serially by lane 0.
constexpr int kWaveCells = 1;
template <bool kFill>
__device__ __forceinline__ void bump_cells_wave(const IvArgs& A, int32_t* __restrict__ iv_cnt,
                                                const int32_t* __restrict__ iv_ptr, int2* __restrict__ iv,
                                                int4* buf) {
  const int lane = lane_id();
  const int64_t c0 = ((int64_t)blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6)) * kWaveCells;
  for (int u = 0; u < kWaveCells; ++u) {
    const int64_t c = c0 + u;
    if (c >= A.g.n_cells) break;
    const uint64_t mask = A.cm[c];
    if (mask == 0) continue;
    int cc[kMaxDim];
    {
      int64_t r = c;
      for (int k = 0; k < A.g.dim; ++k) { cc[k] = (int)(r % A.g.G[k]); r /= A.g.G[k]; }
    }
    int2* out = kFill ? iv + iv_ptr[c] : nullptr;
    int cnt = merge_wave<kFill>(A, cc, mask, buf, out);
    if (cnt < 0) {
      if (lane == 0) cnt = merge_intervals<kFill>(A, cc, mask, A.runs, 0, out);
      cnt = readlane_i32(cnt, 0);
    }
    if (!kFill && lane == 0) iv_cnt[c] = cnt;
    __builtin_amdgcn_wave_barrier();           // buf is the next cell's
  }
}

template <bool kFill>
__global__ __launch_bounds__(kBlock) void k_cell_intervals_wave(IvArgs A, int32_t* __restrict__ iv_cnt,
                                                                const int32_t* __restrict__ iv_ptr,
                                                                int2* __restrict__ iv) {
  __shared__ int4 buf[kBlock / kWave][kWaveRuns];
  bump_cells_wave<kFill>(A, iv_cnt, iv_ptr, iv, buf[threadIdx.x >> 6]);
}

template <bool kFill>
__global__ __launch_bounds__(kBlock) void k_cell_intervals_wave_pop(IvArgs A, const PopMember* __restrict__ pm) {
  __shared__ int4 buf[kBlock / kWave][kWaveRuns];
  const PopMember& P = pm[blockIdx.z];
  A.cm = P.cm;
  A.run_ptr = P.run_ptr;
  A.runs = P.runs;
  bump_cells_wave<kFill>(A, P.iv_cnt, P.iv_ptr, P.iv, buf[threadIdx.x >> 6]);
}

static unsigned wave_cell_grid(int64_t nc) {
  const int64_t per_block = (int64_t)(kBlock / kWave) * kWaveCells;
  return (unsigned)((nc + per_block - 1) / per_block);
}

// Population form: member z's intervals with its own masks and runs (the
// cell grid is shared).
template <bool kFill>
__global__ void k_cell_intervals_pop(IvArgs A, const PopMember* __restrict__ pm) {
  __shared__ int4 sruns[kRunLds];
  const PopMember& P = pm[blockIdx.z];
  A.cm = P.cm;
  if (A.use_bumps) {
    A.run_ptr = P.run_ptr;
    A.runs = P.runs;
  }
  int base = 0;
  const int4* runs = stage_runs(A, sruns, base);
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= A.g.n_cells) return;
  int cc[kMaxDim];
  {
    int64_t r = c;
    for (int k = 0; k < A.g.dim; ++k) { cc[k] = (int)(r % A.g.G[k]); r /= A.g.G[k]; }
  }
  const uint64_t mask = A.use_bumps ? A.cm[c] : 0ull;
  if (mask != 0) return;                      // k_cell_intervals_wave_pop's cell
  const int cnt = merge_intervals<kFill>(A, cc, mask, runs, base, kFill ? P.iv + P.iv_ptr[c] : nullptr);
  if (!kFill) P.iv_cnt[c] = cnt;
}

// Candidate intervals of test points: the clamped cell of each point (a
// training point within the core radius lies at most one cell away per axis
// also after clamping) and the bump functions whose support holds the point.
template <bool kFill>
__global__ void k_query_intervals(IvArgs A, const double4* __restrict__ q, const uint64_t* __restrict__ qm,
                                  int64_t nq, int32_t* __restrict__ iv_cnt, const int32_t* __restrict__ iv_ptr,
                                  int2* __restrict__ iv) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nq) return;
  const double4 p = q[t];
  int cc[kMaxDim];
  for (int k = 0; k < A.g.dim; ++k) cc[k] = cell_coord(comp(p, k), A.g.lo[k], A.g.inv_side[k], A.g.G[k]);
  const uint64_t mask = A.use_bumps ? qm[t] : 0ull;
  const int cnt = merge_intervals<kFill>(A, cc, mask, A.runs, 0, kFill ? iv + iv_ptr[t] : nullptr);
  if (!kFill) iv_cnt[t] = cnt;
}

// ------------------------------------------------------------ count / fill
struct RowArgs {
  const double4* xs;
  const uint64_t* M;
  const double* F;
  const int32_t* cell_of;
  const int32_t* cell_start;
  const int32_t* iv_ptr;
  const int2* iv;
  int64_t n;
  int dim, n1, core, combine, add_noise;
  int core_only;   // keep only the core part (+ diagonal), values without B
  double sigma2, r_core, rc2, noise;
  // keep masks of the count (one 64-bit word per row and 64-candidate step;
  // cell c's words start at mask_ptr[c], step-major over the cell's rows),
  // read by the masked fill; null: not recorded
  const int64_t* mask_ptr = nullptr;
  uint64_t* mask = nullptr;
};

// Count / fill with LDS-staged point tiles: one workgroup per cell.  All rows
// of a cell share the cell's candidate intervals, so the candidates' points
// and bump masks are staged in LDS once per chunk of 512 candidates and every
// row of the cell (one wavefront per row, rows dealt to the four wavefronts)
// tests them from there: a candidate point is read from memory once per cell
// instead of once per row.  The cell's intervals are read in windows of 256
// (one per thread) with their exclusive length prefix from a block scan, so
// every thread finds its candidate of a chunk by a binary search in LDS.
// Each wavefront holds its rows' points, bump masks and output positions in
// registers (one row per lane) and broadcasts them row by row.
// Columns stay ascending (chunks follow the sorted disjoint intervals); each
// row's output position persists in LDS across chunks.  Cells with more
// than 64 rows are processed in row groups.
constexpr int kCC = 512;      // staged candidates per chunk
constexpr int kCRows = 64;    // rows per row group
constexpr int kIvWin = kBlock;  // intervals per window

// Value of a stored entry (row a with bump values Fa, column b): the kernel
// of the stored-pattern predicate's pair, plus the noise on the diagonal.
// kDim: the points' dimension, which fixes the Wendland exponent
// (l = d / 2 + 2).
template <int kDim>
__device__ __forceinline__ double entry_value(const RowArgs& A, int64_t a, const double* Fa, int32_t b, double d2,
                                              uint64_t mm) {
  constexpr int kEll = kDim / 2 + 2;
  double psi = 0.0;
  if (d2 < A.rc2) psi = core_psi(sqrt(d2) / A.r_core, A.core, kEll);
  double B = 0.0;
  const double* Fb = A.F + (int64_t)b * A.n1;
  while (mm) {
    const int i = __builtin_ctzll(mm);
    mm &= mm - 1;
    B += Fa[i] * Fb[i];
  }
  double kv = A.combine == 0 ? A.sigma2 * psi * B : A.sigma2 * psi + B;
  if (b == a && A.add_noise) kv += A.noise;
  return kv;
}

// LDS of the row kernels.  The fill needs the compaction buffers (kCB = 2
// wavefronts' worth of entries per wavefront); the count uses one entry.
template <bool kFill, bool kList, int kDim>
struct CellLds {
  typedef hipcub::BlockScan<int, kBlock> Scan;
  static constexpr int kCB = kFill ? 2 * kWave : 1;
  static constexpr int kKL = kList ? kCC : 1;
  typename Scan::TempStorage scan_tmp;
  double sx[kDim][kCC];      // candidate coordinates, one array per axis
  uint64_t sm[kCC];
  int32_t sb[kCC];
  int32_t wb[kIvWin];        // window: first point of each interval
  int32_t wpre[kIvWin + 1];  // window: exclusive prefix of the lengths
  // fill: per wavefront, the kept entries of the current row compacted in
  // order (column, squared distance, common bump mask), so that values are
  // computed and stored 64 at a time with every lane busy
  int32_t kb_col[kBlock / kWave][kCB];
  double kb_d2[kBlock / kWave][kCB];
  uint64_t kb_mm[kBlock / kWave][kCB];
  // masked fill: per wavefront, the staged indices of the current row's
  // kept candidates of the chunk, in order
  int16_t kl[kBlock / kWave][kKL];
};

// Squared distance from a to staged candidate k (axis arrays in LDS: lanes
// read consecutive doubles, free of bank conflicts), in the order of dist2.
template <int kDim>
__device__ __forceinline__ double dist2_lds(const double4& a, const double (&s)[kDim][kCC], int k) {
  double dx = a.x - s[0][k];
  double d2 = dx * dx;
  if constexpr (kDim > 1) { double d = a.y - s[1][k]; d2 += d * d; }
  if constexpr (kDim > 2) { double d = a.z - s[2][k]; d2 += d * d; }
  if constexpr (kDim > 3) { double d = a.w - s[3][k]; d2 += d * d; }
  return d2;
}

// Modes of the row body: the count (row_nnz[a] = stored entries of row a,
// keep masks recorded when A.mask is set; the candidate tests as three
// wavefront masks combined in scalar registers, over chunks padded to
// whole 64-candidate steps), the fill that tests every candidate again
// (compacting each row's kept entries in LDS), and the fill from the
// count's keep masks (the masks' set bits are listed per row in LDS and
// every lane takes one listed entry: no candidate is tested twice).  The
// candidate pairs are counted apart from these kernels (k_mask_words): one
// counter updated by every cell's workgroup serialised the whole count.
constexpr int kRowCount = 0, kRowFillTest = 1, kRowFillMasked = 2;

// Rows of cell c in mode kMode for points of kDim coordinates.  L: the
// block's LDS (a fill-sized one serves every mode).
template <int kMode, int kDim, class Lds>
__device__ __forceinline__ void cell_rows_body(const RowArgs& A, int64_t c, Lds& L, int64_t* __restrict__ row_nnz,
                                               const int64_t* __restrict__ row_ptr,
                                               int32_t* __restrict__ col, double* __restrict__ val) {
  constexpr bool kFill = kMode != kRowCount;
  typedef typename Lds::Scan Scan;
  auto& scan_tmp = L.scan_tmp;
  auto& sx = L.sx;
  auto& sm = L.sm;
  auto& sb = L.sb;
  auto& wb = L.wb;
  auto& wpre = L.wpre;
  auto& kb_col = L.kb_col;
  auto& kb_d2 = L.kb_d2;
  auto& kb_mm = L.kb_mm;
  const int32_t r0 = A.cell_start[c], r1 = A.cell_start[c + 1];
  if (r1 <= r0) return;                       // uniform: empty cell
  const int32_t i0 = A.iv_ptr[c], i1 = A.iv_ptr[c + 1];
  const int t = threadIdx.x, lane = lane_id(), w = t >> 6;
  constexpr int kWaves = kBlock / kWave;
  const int64_t nrc = r1 - r0;                // rows of the cell (mask stride)
  const int64_t mbase = A.mask ? A.mask_ptr[c] : 0;
  // stored-pattern predicate as two uniform flags: a core pair is kept
  // unless the bumps must agree too (PRODUCT), a bump pair alone only
  // under SUM; the diagonal always
  const bool core_keeps = A.core_only || A.combine != 0;
  const bool bump_keeps = !A.core_only && A.combine != 0;
  for (int32_t g0 = r0; g0 < r1; g0 += kCRows) {
    const int nr = min(r1 - g0, kCRows);
    int st0 = 0;                              // 64-candidate steps before the chunk (uniform)
    // rows of the group are dealt to the wavefronts in turn: this one's are
    // g0 + w + kWaves * i for i < nrw, row i's point, bump mask and output
    // position (fill) or kept count (count) held by lane i
    const int nrw = nr > w ? (nr - w + kWaves - 1) / kWaves : 0;
    double4 xr = make_double4(0.0, 0.0, 0.0, 0.0);
    uint64_t mr = 0;
    int64_t pr = 0;
    if (lane < nrw) {
      const int32_t a = g0 + w + kWaves * lane;
      xr = A.xs[a];
      mr = A.M[a];
      if (kFill) pr = row_ptr[a];
    }
    // row i's point, uniform over the wavefront
    auto row_point = [&](int i) {
      double4 p;
      p.x = readlane_f64(xr.x, i);
      p.y = kDim > 1 ? readlane_f64(xr.y, i) : 0.0;
      p.z = kDim > 2 ? readlane_f64(xr.z, i) : 0.0;
      p.w = kDim > 3 ? readlane_f64(xr.w, i) : 0.0;
      return p;
    };
    for (int32_t q0 = i0; q0 < i1; q0 += kIvWin) {
      const int nw = min(i1 - q0, kIvWin);
      int len = 0;
      if (t < nw) {
        const int2 iv = A.iv[q0 + t];
        wb[t] = iv.x;
        len = iv.y - iv.x;
      }
      int pre = 0, tot = 0;
      Scan(scan_tmp).ExclusiveSum(len, pre, tot);
      if (t < nw) wpre[t] = pre;
      if (t == 0) wpre[nw] = tot;
      __syncthreads();
      for (int k0 = 0; k0 < tot; k0 += kCC) {
        const int filled = min(kCC, tot - k0);
        for (int k = t; k < filled; k += kBlock) {
          const int kk = k0 + k;
          int lo = 0, hi = nw;                // wpre[lo] <= kk < wpre[hi]
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (wpre[mid] <= kk) lo = mid; else hi = mid;
          }
          const int32_t b = wb[lo] + (kk - wpre[lo]);
          const double4 p = A.xs[b];
          sx[0][k] = p.x;
          if constexpr (kDim > 1) sx[1][k] = p.y;
          if constexpr (kDim > 2) sx[2][k] = p.z;
          if constexpr (kDim > 3) sx[3][k] = p.w;
          sm[k] = A.M[b];
          sb[k] = b;
        }
        // pad the last 64-candidate step with candidates that are never
        // kept (NaN distance, no bumps, no point index)
        const int padded = min(kCC, (filled + kWave - 1) / kWave * kWave);
        for (int k = filled + t; k < padded; k += kBlock) {
          sx[0][k] = __builtin_nan("");
          sm[k] = 0;
          sb[k] = -1;
        }
        __syncthreads();
        const int nsteps = (filled + kWave - 1) / kWave;   // <= kCC / 64
        if constexpr (kMode == kRowCount) {
          for (int i = 0; i < nrw; ++i) {
            const int r = w + kWaves * i;
            const int32_t a = g0 + r;
            const double4 xa = row_point(i);
            const uint64_t Ma = readlane_u64(mr, i);
            int64_t kept = 0;                 // uniform
            uint64_t mw = 0;                  // lane q: keep mask of step q
            for (int q = 0; q < nsteps; ++q) {
              const int k = q * kWave + lane; // a staged or padding candidate
              const double d2 = dist2_lds<kDim>(xa, sx, k);
              // the three tests as wavefront masks, combined in scalar registers
              const uint64_t bd = ballot64(sb[k] == a);
              const uint64_t bc = ballot64(d2 < A.rc2);
              const uint64_t bb = ballot64((Ma & sm[k]) != 0);
              const uint64_t bal = bd | (bc & (core_keeps ? ~0ull : bb)) | (bump_keeps ? bb : 0ull);
              kept += __popcll(bal);
              mw = lane == q ? bal : mw;
            }
            if (A.mask && lane < nsteps) A.mask[mbase + (int64_t)(st0 + lane) * nrc + (g0 - r0 + r)] = mw;
            if (lane == i) pr += kept;
          }
          st0 += nsteps;
          __syncthreads();
          continue;
        }
        if constexpr (kMode == kRowFillMasked) {
          for (int i = 0; i < nrw; ++i) {
            const int r = w + kWaves * i;
            const int64_t a = (int64_t)g0 + r;
            const double4 xa = row_point(i);
            const uint64_t Ma = A.core_only ? 0 : readlane_u64(mr, i);
            const double* Fa = A.F + a * (int64_t)A.n1;
            const int64_t pos = (int64_t)readlane_u64((uint64_t)pr, i);
            const uint64_t mw = lane < nsteps ? A.mask[mbase + (int64_t)(st0 + lane) * nrc + (g0 - r0 + r)] : 0;
            int nkeep = 0;                    // uniform
            for (int q = 0; q < nsteps; ++q) {
              const uint64_t mq = readlane_u64(mw, q);
              if (mq >> lane & 1) L.kl[w][nkeep + lanes_below(mq)] = (int16_t)(q * kWave + lane);
              nkeep += __popcll(mq);
            }
            __builtin_amdgcn_wave_barrier();
            for (int e = lane; e < nkeep; e += kWave) {
              const int k = L.kl[w][e];
              const int32_t b = sb[k];
              const double d2 = dist2_lds<kDim>(xa, sx, k);
              col[pos + e] = b;
              val[pos + e] = entry_value<kDim>(A, a, Fa, b, d2, Ma & sm[k]);
            }
            __builtin_amdgcn_wave_barrier();  // the list is the next row's
            if (lane == i) pr = pos + nkeep;
          }
          st0 += nsteps;
          __syncthreads();
          continue;
        }
        for (int i = 0; i < nrw; ++i) {
          const int64_t a = (int64_t)g0 + w + kWaves * i;
          const double4 xa = row_point(i);
          const uint64_t Ma = readlane_u64(mr, i);
          const double* Fa = A.F + a * (int64_t)A.n1;
          int64_t pos = (int64_t)readlane_u64((uint64_t)pr, i);
          int nk = 0;                         // compacted kept entries (fill; uniform)
          for (int j0 = 0; j0 < filled; j0 += kWave) {
            const int k = j0 + lane;
            bool keep = false, core = false;
            double d2 = 0.0;
            uint64_t mm = 0;
            int32_t b = 0;
            if (k < filled) {
              b = sb[k];
              d2 = dist2_lds<kDim>(xa, sx, k);
              core = d2 < A.rc2;
              mm = Ma & sm[k];
              const bool bump = mm != 0;
              keep = (b == a) | (core & (core_keeps | bump)) | (bump_keeps & bump);
              if (A.core_only) mm = 0;
            }
            const uint64_t bal = ballot64(keep);
            if (keep) {
              const int q = nk + lanes_below(bal);
              kb_col[w][q] = b;
              kb_d2[w][q] = d2;
              kb_mm[w][q] = mm;
            }
            nk += __popcll(bal);
            if (nk >= kWave) {                // 64 buffered: values and stores with every lane
              __builtin_amdgcn_wave_barrier();
              const int32_t bb = kb_col[w][lane];
              col[pos + lane] = bb;
              val[pos + lane] = entry_value<kDim>(A, a, Fa, bb, kb_d2[w][lane], kb_mm[w][lane]);
              pos += kWave;
              nk -= kWave;
              __builtin_amdgcn_wave_barrier();
              int32_t mc = 0;
              double md = 0.0;
              uint64_t mb = 0;
              if (lane < nk) {
                mc = kb_col[w][kWave + lane];
                md = kb_d2[w][kWave + lane];
                mb = kb_mm[w][kWave + lane];
              }
              __builtin_amdgcn_wave_barrier();
              if (lane < nk) {
                kb_col[w][lane] = mc;
                kb_d2[w][lane] = md;
                kb_mm[w][lane] = mb;
              }
            }
          }
          if (kFill && nk > 0) {              // the rest of the row's kept entries of this chunk
            __builtin_amdgcn_wave_barrier();
            if (lane < nk) {
              const int32_t bb = kb_col[w][lane];
              col[pos + lane] = bb;
              val[pos + lane] = entry_value<kDim>(A, a, Fa, bb, kb_d2[w][lane], kb_mm[w][lane]);
            }
            pos += nk;
          }
          if (lane == i) pr = pos;
        }
        st0 += nsteps;
        __syncthreads();
      }
      __syncthreads();                        // window storage and scan storage free again
    }
    if (!kFill && lane < nrw) row_nnz[g0 + w + kWaves * lane] = pr;
  }
}

template <int kMode, int kDim>
__global__ __launch_bounds__(kBlock) void k_cell_rows(RowArgs A, int64_t* __restrict__ row_nnz,
                                                      const int64_t* __restrict__ row_ptr,
                                                      int32_t* __restrict__ col, double* __restrict__ val) {
  __shared__ CellLds<kMode == kRowFillTest, kMode == kRowFillMasked, kDim> L;
  cell_rows_body<kMode, kDim>(A, blockIdx.x, L, row_nnz, row_ptr, col, val);
}

// Population form: member z's rows (RowArgs[z] holds its kernel
// parameters and inputs, PopMember[z] its outputs).
template <bool kFill, int kDim>
__global__ __launch_bounds__(kBlock) void k_cell_rows_pop(const RowArgs* __restrict__ ra,
                                                          const PopMember* __restrict__ pm) {
  const PopMember& P = pm[blockIdx.z];
  __shared__ CellLds<kFill, false, kDim> L;
  cell_rows_body<kFill ? kRowFillTest : kRowCount, kDim>(ra[blockIdx.z], blockIdx.x, L, P.row_nnz, P.row_ptr,
                                                         P.col, P.val);
}

// Row-kernel launches for points of `dim` coordinates (1 to kMaxDim), one
// workgroup per cell.
template <int kMode>
static void launch_cell_rows(int dim, unsigned grid, hipStream_t st, const RowArgs& A, int64_t* row_nnz,
                             const int64_t* row_ptr, int32_t* col, double* val) {
  switch (dim) {
    case 1: k_cell_rows<kMode, 1><<<grid, kBlock, 0, st>>>(A, row_nnz, row_ptr, col, val); break;
    case 2: k_cell_rows<kMode, 2><<<grid, kBlock, 0, st>>>(A, row_nnz, row_ptr, col, val); break;
    case 3: k_cell_rows<kMode, 3><<<grid, kBlock, 0, st>>>(A, row_nnz, row_ptr, col, val); break;
    default: k_cell_rows<kMode, 4><<<grid, kBlock, 0, st>>>(A, row_nnz, row_ptr, col, val); break;
  }
}

template <bool kFill>
static void launch_cell_rows_pop(int dim, dim3 grid, hipStream_t st, const RowArgs* ra, const PopMember* pm) {
  switch (dim) {
    case 1: k_cell_rows_pop<kFill, 1><<<grid, kBlock, 0, st>>>(ra, pm); break;
    case 2: k_cell_rows_pop<kFill, 2><<<grid, kBlock, 0, st>>>(ra, pm); break;
    case 3: k_cell_rows_pop<kFill, 3><<<grid, kBlock, 0, st>>>(ra, pm); break;
    default: k_cell_rows_pop<kFill, 4><<<grid, kBlock, 0, st>>>(ra, pm); break;
  }
}

// row_ptr of every member from one scan over the members' concatenated
// count arrays (each [n + 1] with a zero last entry): subtract the
// member's base.
__global__ void k_rebase_pop(const int64_t* __restrict__ scan, int64_t n, int64_t* __restrict__ out) {
  const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a > n) return;
  const int64_t o = (int64_t)blockIdx.z * (n + 1);
  out[o + a] = scan[o + a] - scan[o];
}


// ------------------------------------------------------- cross covariance
// Rows are test points (caller order), columns sorted training points; the
// stored predicate has no diagonal rule (the sets are distinct).
struct CrossArgs {
  const double4* xs;
  const uint64_t* M;
  const double* F;
  const double4* q;
  const uint64_t* qm;
  const double* qF;
  const int32_t* iv_ptr;
  const int2* iv;
  int64_t nq;
  int dim, n1, core, ell, combine;
  double sigma2, r_core, rc2;
};

template <bool kFill>
__global__ __launch_bounds__(kBlock) void k_cross_rows(CrossArgs A, int64_t* __restrict__ row_nnz,
                                                       const int64_t* __restrict__ row_ptr,
                                                       int32_t* __restrict__ col, double* __restrict__ val) {
  const int64_t t = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  if (t >= A.nq) return;
  const int lane = lane_id();
  const double4 xt = A.q[t];
  const uint64_t Mt = A.qm[t];
  const double* Ft = A.qF + t * (int64_t)A.n1;
  int64_t pos = kFill ? row_ptr[t] : 0;
  int64_t cnt = 0;
  for (int32_t k = A.iv_ptr[t]; k < A.iv_ptr[t + 1]; ++k) {
    const int2 r = A.iv[k];
    for (int32_t b0 = r.x; b0 < r.y; b0 += kWave) {
      const int32_t b = b0 + lane;
      bool keep = false, core = false;
      double d2 = 0.0;
      uint64_t mm = 0;
      if (b < r.y) {
        d2 = dist2(xt, A.xs[b], A.dim);
        core = d2 < A.rc2;
        mm = Mt & A.M[b];
        keep = A.combine == 0 ? (core && mm != 0) : (core || mm != 0);
      }
      const uint64_t bal = ballot64(keep);
      if (kFill) {
        if (keep) {
          const double psi = core ? core_psi(sqrt(d2) / A.r_core, A.core, A.ell) : 0.0;
          double B = 0.0;
          const double* Fb = A.F + (int64_t)b * A.n1;
          uint64_t m = mm;
          while (m) {
            const int i = __builtin_ctzll(m);
            m &= m - 1;
            B += Ft[i] * Fb[i];
          }
          const int64_t o = pos + lanes_below(bal);
          col[o] = b;
          val[o] = A.combine == 0 ? A.sigma2 * psi * B : A.sigma2 * psi + B;
        }
        pos += __popcll(bal);
      } else {
        cnt += __popcll(bal);
      }
    }
  }
  if (!kFill && lane == 0) row_nnz[t] = cnt;
}

// Prior variance k(x0, x0) of each test point.
__global__ void k_prior_diag(const uint64_t* __restrict__ qm, const double* __restrict__ qF, int64_t nq, int n1,
                             int core, int ell, int combine, double sigma2, double* __restrict__ kxx) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nq) return;
  double B = 0.0;
  uint64_t m = qm[t];
  while (m) {
    const int i = __builtin_ctzll(m);
    m &= m - 1;
    const double f = qF[t * (int64_t)n1 + i];
    B += f * f;
  }
  const double psi0 = core_psi(0.0, core, ell);
  kxx[t] = combine == 0 ? sigma2 * psi0 * B : sigma2 * psi0 + B;
}

__global__ void k_pack_points(const double* __restrict__ x, int64_t n, int dim, double4* __restrict__ out) {
  const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= n) return;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < dim; ++k) v[k] = x[a * dim + k];
  out[a] = make_double4(v[0], v[1], v[2], v[3]);
}

// ---------------------------------------------------------- canonical CSR
__global__ void k_canon_len(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ perm,
                            int64_t n, int64_t* __restrict__ len) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s < n) len[perm[s]] = row_ptr[s + 1] - row_ptr[s];
  if (s == 0) len[n] = 0;
}

__global__ void k_canon_copy(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                             const double* __restrict__ val, const int32_t* __restrict__ perm,
                             int64_t n, const int64_t* __restrict__ out_ptr,
                             int32_t* __restrict__ col2, double* __restrict__ val2) {
  const int64_t s = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  if (s >= n) return;
  const int lane = lane_id();
  const int64_t src = row_ptr[s], len = row_ptr[s + 1] - src;
  const int64_t dst = out_ptr[perm[s]];
  for (int64_t k = lane; k < len; k += kWave) {
    col2[dst + k] = perm[col[src + k]];
    val2[dst + k] = val[src + k];
  }
}

__global__ void k_iota_i64(int64_t* p, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

// =========================================================== host side
KParams make_params(const sdgp_kernel_desc& d, const double* h) {
  KParams k;
  k.dim = d.dim; k.n1 = d.n1; k.n2 = d.n2; k.core = d.core; k.combine = d.combine;
  k.sigma2 = h[0];
  k.r_core = h[1];
  k.rc2 = h[1] * h[1];
  k.inv_rc = 1.0 / h[1];
  k.noise = h[2 + (int64_t)d.n1 * d.n2 * (3 + d.dim)];
  return k;
}

void validate_shape(const sdgp_kernel_desc& d, int64_t n) {
  require(d.dim >= 1 && d.dim <= kMaxDim, "dim must be in 1..4");
  require(d.n1 >= 0 && d.n1 <= kMaxN1, "n1 must be in 0..64");
  require(d.n1 == 0 || d.n2 >= 1, "n2 must be >= 1");
  require(d.core == SDGP_CORE_WENDLAND_C2 || d.core == SDGP_CORE_KSTAT, "unknown core");
  require(d.combine == SDGP_COMBINE_PRODUCT || d.combine == SDGP_COMBINE_SUM, "unknown combine");
  require(n >= 1 && n < (int64_t)0x7fffffff, "n must be in 1..2^31-2");
}

void validate(const sdgp_kernel_desc& d, const double* h, int64_t n) {
  validate_shape(d, n);
  require(h != nullptr, "h is NULL");
  const int64_t nh = 2 + (int64_t)d.n1 * d.n2 * (3 + d.dim) + 1;
  for (int64_t i = 0; i < nh; ++i) require(std::isfinite(h[i]), "hyperparameters must be finite");
  require(h[0] >= 0.0, "sigma2 must be >= 0");
  require(h[1] > 0.0, "core radius must be > 0");
  require(h[nh - 1] >= 0.0, "noise variance must be >= 0");
  for (int i = 0; i < d.n1; ++i)
    for (int j = 0; j < d.n2; ++j) {
      const double* q = h + 2 + (int64_t)(i * d.n2 + j) * (3 + d.dim);
      require(q[2] > 0.0, "bump radius must be > 0");
      require(q[1] >= 0.0, "bump shape beta must be >= 0");
    }
}

Sorted order_points(Ctx* c, const double* x, int64_t n, int dim, double r_cell, bool with_schedule) {
  Sorted s;
  s.n = n;
  s.sched = nullptr;
  // bounding box
  const int nb = std::min<int64_t>(1024, (n + kBlock - 1) / kBlock);
  double* part = c->get<double>(S_BBOX, (size_t)nb * 2 * kMaxDim);
  k_bbox<<<nb, kBlock, 0, c->stream>>>(x, n, dim, part);
  SDGP_CHECK_LAUNCH();
  std::vector<double> hp((size_t)nb * 2 * kMaxDim);
  SDGP_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  double lo[kMaxDim], hi[kMaxDim];
  for (int k = 0; k < kMaxDim; ++k) { lo[k] = INFINITY; hi[k] = -INFINITY; }
  for (int b = 0; b < nb; ++b)
    for (int k = 0; k < dim; ++k) {
      lo[k] = std::min(lo[k], hp[b * 2 * kMaxDim + k]);
      hi[k] = std::max(hi[k], hp[b * 2 * kMaxDim + kMaxDim + k]);
    }
  for (int k = 0; k < dim; ++k) require(std::isfinite(lo[k]) && std::isfinite(hi[k]), "x must be finite");
  // grid: side >= r_cell (1 + 1e-9) so any pair closer than r_cell is at most
  // one cell apart per axis; capped at ~2 cells per point
  Grid g;
  g.dim = dim;
  const double side = r_cell * (1.0 + 1e-9);
  double G[kMaxDim];
  for (int k = 0; k < dim; ++k) {
    const double ext = hi[k] - lo[k];
    G[k] = std::max(1.0, std::floor(ext / side));
    G[k] = std::min(G[k], 1e6);
  }
  const double cap = std::max<double>(1024.0, 2.0 * (double)n);
  for (;;) {
    double tot = 1.0;
    for (int k = 0; k < dim; ++k) tot *= G[k];
    if (tot <= cap) break;
    int kmax = 0;
    for (int k = 1; k < dim; ++k) if (G[k] > G[kmax]) kmax = k;
    G[kmax] = std::max(1.0, std::floor(G[kmax] / 2.0));
  }
  g.n_cells = 1;
  for (int k = 0; k < kMaxDim; ++k) {
    if (k < dim) {
      g.G[k] = (int)G[k];
      g.lo[k] = lo[k];
      const double ext = hi[k] - lo[k];
      g.inv_side[k] = ext > 0.0 ? G[k] / ext : 0.0;
      g.n_cells *= g.G[k];
    } else {
      g.G[k] = 1; g.lo[k] = 0.0; g.inv_side[k] = 0.0;
    }
  }
  s.grid = g;
  // keys + radix sort (stable: equal cells keep caller order)
  uint32_t* keys = c->get<uint32_t>(S_KEYS, n);
  uint32_t* keys_out = c->get<uint32_t>(S_KEYS_ALT, n);
  int32_t* idx = c->get<int32_t>(S_IDX, n);
  int32_t* perm = c->get<int32_t>(S_PERM, n);
  k_cell_keys<<<grid_for(n, kBlock), kBlock, 0, c->stream>>>(x, n, g, keys, idx);
  SDGP_CHECK_LAUNCH();
  int bits = 1;
  while (((int64_t)1 << bits) < g.n_cells) ++bits;
  size_t tb = 0;
  SDGP_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, keys, keys_out, idx, perm, (int)n, 0, bits, c->stream));
  void* tmp = c->get<char>(S_SORT_TMP, tb);
  SDGP_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, keys, keys_out, idx, perm, (int)n, 0, bits, c->stream));
  int32_t* cell_start = c->get<int32_t>(S_CELL_START, g.n_cells + 1);
  k_cell_start<<<grid_for(n, kBlock), kBlock, 0, c->stream>>>(keys_out, n, g.n_cells, cell_start);
  SDGP_CHECK_LAUNCH();
  double4* xs = c->get<double4>(S_XS, n);
  k_gather_points<<<grid_for(n, kBlock), kBlock, 0, c->stream>>>(x, perm, n, dim, xs);
  SDGP_CHECK_LAUNCH();
  // Row schedule: the sorted points in Morton (Z-curve) order of their
  // coordinates quantised to 2^mb steps per axis; consecutive schedule
  // positions are spatial neighbours at every scale, so a window of rows in
  // flight gathers from a compact neighbourhood.  Only the solver and the
  // adjoint walk it; assembly alone does not need it.
  if (with_schedule) {
    MortonQ mq;
    mq.dim = dim;
    mq.bits = std::min(16, 62 / dim);
    const double steps = (double)((1 << mq.bits) - 1);
    for (int k = 0; k < kMaxDim; ++k) {
      mq.lo[k] = k < dim ? lo[k] : 0.0;
      const double ext = k < dim ? hi[k] - lo[k] : 0.0;
      mq.scale[k] = ext > 0.0 ? steps / ext : 0.0;
    }
    uint64_t* mk = c->get<uint64_t>(S_MORTON_KEYS, n);
    uint64_t* mk2 = c->get<uint64_t>(S_MORTON_KEYS2, n);
    int32_t* ids = c->get<int32_t>(S_MORTON_IDS, n);
    int32_t* sched = c->get<int32_t>(S_SCHED, n);
    k_point_morton<<<grid_for(n, kBlock), kBlock, 0, c->stream>>>(xs, n, mq, mk, ids);
    SDGP_CHECK_LAUNCH();
    size_t tb2 = 0;
    const int kbits = mq.bits * dim;
    SDGP_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb2, mk, mk2, ids, sched, (int)n, 0, kbits, c->stream));
    void* tmp2 = c->get<char>(S_SORT_TMP, tb2);
    SDGP_HIP(hipcub::DeviceRadixSort::SortPairs(tmp2, tb2, mk, mk2, ids, sched, (int)n, 0, kbits, c->stream));
    s.sched = sched;
  }
  s.perm = perm;
  s.xs = xs;
  s.cell_start = cell_start;
  s.cell_of = reinterpret_cast<int32_t*>(keys_out);
  return s;
}

void gather_vector(Ctx* c, const Sorted& s, const double* src, double* dst) {
  k_gather_vec<<<grid_for(s.n, kBlock), kBlock, 0, c->stream>>>(src, s.perm, s.n, dst);
  SDGP_CHECK_LAUNCH();
}

Bumps bump_precompute(Ctx* c, const Sorted& s, const KParams& kp, const double* h) {
  Bumps b;
  const int n1 = kp.n1;
  const int64_t np = (int64_t)kp.n1 * kp.n2 * (3 + kp.dim);
  b.bp = c->get<double>(S_BP, np > 0 ? np : 1);
  if (np > 0)
    SDGP_HIP(hipMemcpyAsync(b.bp, h + 2, np * sizeof(double), hipMemcpyHostToDevice, c->stream));
  b.F = c->get<double>(S_F, (size_t)s.n * (n1 > 0 ? n1 : 1));
  b.M = c->get<uint64_t>(S_M, s.n);
  k_bumps<<<grid_for(s.n, kBlock), kBlock, 0, c->stream>>>(s.xs, s.n, kp.dim, n1, kp.n2, b.bp, b.F, b.M);
  SDGP_CHECK_LAUNCH();
  return b;
}

// Bump-function cell runs of B members (masks cm[z nc + c]) with no host
// round trip: flags, one scan, run pointers and runs (storage sized for the
// most runs a function can have, ceil(nc / 2)).
static void bump_runs(Ctx* c, const uint64_t* cm, const int32_t* cell_start, int64_t nc, int n1, int B,
                      Slot s_flag, Slot s_pos, Slot s_ptr, Slot s_runs, int32_t** run_ptr_out, int4** runs_out) {
  const int64_t nflag = (int64_t)B * n1 * nc + 1;
  require(nflag < 0x7fffffffLL, "too many (member, bump function, cell) triples");
  int32_t* flag = c->get<int32_t>(s_flag, nflag);
  int32_t* pos = c->get<int32_t>(s_pos, nflag);
  SDGP_HIP(hipMemsetAsync(flag + nflag - 1, 0, sizeof(int32_t), c->stream));
  const unsigned gc = (unsigned)grid_for(nc, kBlock);
  k_run_flags<<<dim3(gc, n1, B), kBlock, 0, c->stream>>>(cm, nc, n1, flag);
  SDGP_CHECK_LAUNCH();
  size_t tb = 0;
  SDGP_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, flag, pos, (int)nflag, c->stream));
  void* tmp = c->get<char>(S_SORT_TMP, tb);
  SDGP_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, flag, pos, (int)nflag, c->stream));
  int32_t* run_ptr = c->get<int32_t>(s_ptr, (size_t)B * (n1 + 1));
  k_run_ptr<<<(unsigned)grid_for((int64_t)B * (n1 + 1), kBlock), kBlock, 0, c->stream>>>(pos, nc, n1, B, run_ptr);
  SDGP_CHECK_LAUNCH();
  int4* runs = c->get<int4>(s_runs, (size_t)B * n1 * ((nc + 1) / 2) + 1);
  k_run_write<<<dim3(gc, n1, B), kBlock, 0, c->stream>>>(cm, nc, n1, pos, cell_start, runs);
  SDGP_CHECK_LAUNCH();
  *run_ptr_out = run_ptr;
  *runs_out = runs;
}

void prune(Ctx* c, const Sorted& s, const KParams& kp, const Bumps& b, int32_t** iv_ptr_out,
           int2** iv_out, bool core_only) {
  const int64_t nc = s.grid.n_cells;
  uint64_t* cm = c->get<uint64_t>(S_CELLMASK, nc);
  k_cellmask<<<grid_for(nc, kBlock), kBlock, 0, c->stream>>>(s.cell_start, nc, b.M, cm);
  SDGP_CHECK_LAUNCH();
  IvArgs A;
  A.g = s.grid;
  A.cell_start = s.cell_start;
  A.cm = cm;
  A.run_ptr = nullptr;
  A.runs = nullptr;
  A.use_bumps = (kp.combine == SDGP_COMBINE_SUM && kp.n1 > 0 && !core_only) ? 1 : 0;
  A.n1 = kp.n1;
  if (A.use_bumps) {
    int32_t* run_ptr = nullptr;
    int4* runs = nullptr;
    bump_runs(c, cm, s.cell_start, nc, kp.n1, 1, S_RUN_CNT, S_RUN_POS, S_RUN_PTR, S_RUNS, &run_ptr, &runs);
    A.run_ptr = run_ptr;
    A.runs = runs;
  }
  int32_t* iv_cnt = c->get<int32_t>(S_IV_CNT, nc + 1);
  k_cell_intervals<false><<<grid_for(nc, kBlock), kBlock, 0, c->stream>>>(A, iv_cnt, nullptr, nullptr);
  SDGP_CHECK_LAUNCH();
  if (A.use_bumps) {
    k_cell_intervals_wave<false><<<wave_cell_grid(nc), kBlock, 0, c->stream>>>(A, iv_cnt, nullptr, nullptr);
    SDGP_CHECK_LAUNCH();
  }
  int32_t* iv_ptr = c->get<int32_t>(S_IV_PTR, nc + 1);
  size_t tb = 0;
  SDGP_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, iv_cnt, iv_ptr, (int)(nc + 1), c->stream));
  void* tmp = c->get<char>(S_SORT_TMP, tb);
  // iv_cnt[nc] is scratch: zero it so the scan's last entry is the total
  SDGP_HIP(hipMemsetAsync(iv_cnt + nc, 0, sizeof(int32_t), c->stream));
  SDGP_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, iv_cnt, iv_ptr, (int)(nc + 1), c->stream));
  int32_t total = 0;
  SDGP_HIP(hipMemcpyAsync(&total, iv_ptr + nc, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  int2* iv = c->get<int2>(S_IV, total > 0 ? total : 1);
  k_cell_intervals<true><<<grid_for(nc, kBlock), kBlock, 0, c->stream>>>(A, nullptr, iv_ptr, iv);
  SDGP_CHECK_LAUNCH();
  if (A.use_bumps) {
    k_cell_intervals_wave<true><<<wave_cell_grid(nc), kBlock, 0, c->stream>>>(A, nullptr, iv_ptr, iv);
    SDGP_CHECK_LAUNCH();
  }
  *iv_ptr_out = iv_ptr;
  *iv_out = iv;
}

static RowArgs row_args(const Sorted& s, const KParams& kp, const Bumps& b, const int32_t* iv_ptr,
                        const int2* iv, bool add_noise, bool core_only) {
  RowArgs A;
  A.xs = s.xs; A.M = b.M; A.F = b.F; A.cell_of = s.cell_of; A.cell_start = s.cell_start;
  A.iv_ptr = iv_ptr; A.iv = iv;
  A.n = s.n; A.dim = kp.dim; A.n1 = kp.n1; A.core = kp.core;
  A.combine = kp.combine; A.add_noise = add_noise ? 1 : 0; A.core_only = core_only ? 1 : 0;
  A.sigma2 = kp.sigma2; A.r_core = kp.r_core; A.rc2 = kp.rc2; A.noise = kp.noise;
  return A;
}

// Keep-mask words of each cell: its rows times its 64-candidate steps (the
// row body walks the cell's intervals in windows of kIvWin and each
// window's candidates in chunks of kCC, a multiple of 64, so a window of
// `tot` candidates takes ceil(tot / 64) steps); words[nc] = 0.  Also the
// candidate pairs (rows times candidates) of all cells, added to cand_total
// once per wavefront (null words: the sum alone).
__global__ void k_mask_words(const int32_t* __restrict__ cell_start, const int32_t* __restrict__ iv_ptr,
                             const int2* __restrict__ iv, int64_t nc, int64_t* __restrict__ words,
                             unsigned long long* __restrict__ cand_total) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t pairs = 0;
  if (c < nc) {
    const int32_t i0 = iv_ptr[c], i1 = iv_ptr[c + 1];
    const int64_t rows = cell_start[c + 1] - cell_start[c];
    int64_t steps = 0, cands = 0;
    for (int32_t q0 = i0; q0 < i1; q0 += kIvWin) {
      const int32_t q1 = min(i1, q0 + kIvWin);
      int64_t tot = 0;
      for (int32_t q = q0; q < q1; ++q) tot += iv[q].y - iv[q].x;
      steps += (tot + kWave - 1) / kWave;
      cands += tot;
    }
    if (words) words[c] = rows * steps;
    pairs = rows * cands;
  } else if (c == nc && words) {
    words[nc] = 0;
  }
  pairs = wave_sum_i64(pairs);
  if (lane_id() == 0 && pairs > 0) atomicAdd(cand_total, (unsigned long long)pairs);
}

// Population form: member z's candidate pairs (its own intervals).
__global__ void k_cell_cands_pop(const int32_t* __restrict__ cell_start, int64_t nc,
                                 const PopMember* __restrict__ pm) {
  const PopMember& P = pm[blockIdx.z];
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t pairs = 0;
  if (c < nc) {
    int64_t cands = 0;
    for (int32_t q = P.iv_ptr[c]; q < P.iv_ptr[c + 1]; ++q) cands += P.iv[q].y - P.iv[q].x;
    pairs = (int64_t)(cell_start[c + 1] - cell_start[c]) * cands;
  }
  pairs = wave_sum_i64(pairs);
  if (lane_id() == 0 && pairs > 0) atomicAdd(P.cand, (unsigned long long)pairs);
}

// Count (recording keep masks), device-wide scan, host read of nnz, fill
// from the masks.
static Csr assemble_two_pass(Ctx* c, const Sorted& s, RowArgs A, int64_t* candidates, PhaseTimer* t,
                             const CsrOut* out) {
  const int64_t n = s.n;
  const int64_t ncell = s.grid.n_cells;
  // keep masks of the count for the fill: offsets per cell, then storage;
  // the candidate pairs on the way
  int64_t* mwords = c->get<int64_t>(S_MASK_CNT, ncell + 1);
  unsigned long long* cand = c->get<unsigned long long>(S_COUNTER, 4);
  SDGP_HIP(hipMemsetAsync(cand, 0, sizeof(unsigned long long), c->stream));
  k_mask_words<<<grid_for(ncell + 1, kBlock), kBlock, 0, c->stream>>>(s.cell_start, A.iv_ptr, A.iv, ncell, mwords,
                                                                      cand);
  SDGP_CHECK_LAUNCH();
  int64_t* mptr = c->get<int64_t>(S_MASK_PTR, ncell + 1);
  size_t tbm = 0;
  SDGP_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tbm, mwords, mptr, (int)(ncell + 1), c->stream));
  SDGP_HIP(hipcub::DeviceScan::ExclusiveSum(c->get<char>(S_SORT_TMP, tbm), tbm, mwords, mptr, (int)(ncell + 1),
                                            c->stream));
  int64_t nwords = 0;
  SDGP_HIP(hipMemcpyAsync(&nwords, mptr + ncell, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  A.mask_ptr = mptr;
  A.mask = c->get<uint64_t>(S_MASK, nwords > 0 ? nwords : 1);
  int64_t* row_nnz = c->get<int64_t>(S_ROW_NNZ, n + 1);
  SDGP_HIP(hipMemsetAsync(row_nnz + n, 0, sizeof(int64_t), c->stream));
  launch_cell_rows<kRowCount>(A.dim, (unsigned)ncell, c->stream, A, row_nnz, nullptr, nullptr, nullptr);
  SDGP_CHECK_LAUNCH();
  int64_t* row_ptr = out ? out->row_ptr : c->get<int64_t>(S_ROW_PTR, n + 1);
  size_t tb = 0;
  SDGP_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, row_nnz, row_ptr, (int)(n + 1), c->stream));
  void* tmp = c->get<char>(S_SORT_TMP, tb);
  SDGP_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, row_nnz, row_ptr, (int)(n + 1), c->stream));
  int64_t nnz = 0;
  unsigned long long ncand = 0;
  SDGP_HIP(hipMemcpyAsync(&nnz, row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipMemcpyAsync(&ncand, cand, sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  if (candidates) *candidates = (int64_t)ncand;
  if (t) t->mark(4);
  Csr k;
  if (out && nnz > out->capacity) {   // the caller's arrays are too small: no fill
    k.n = n; k.nnz = nnz; k.row_ptr = row_ptr; k.col = nullptr; k.val = nullptr;
    return k;
  }
  int32_t* col = out ? out->col : c->get<int32_t>(S_COL, nnz);
  double* val = out ? out->val : c->get<double>(S_VAL, nnz);
  launch_cell_rows<kRowFillMasked>(A.dim, (unsigned)ncell, c->stream, A, nullptr, row_ptr, col, val);
  SDGP_CHECK_LAUNCH();
  k.n = n; k.nnz = nnz; k.row_ptr = row_ptr; k.col = col; k.val = val;
  return k;
}

Csr assemble_sorted(Ctx* c, const Sorted& s, const KParams& kp, const Bumps& b, const int32_t* iv_ptr,
                    const int2* iv, bool add_noise, int64_t* candidates, PhaseTimer* t, bool core_only,
                    const CsrOut* out) {
  require(s.grid.n_cells < 0x7fffffff, "too many cells");
  RowArgs A = row_args(s, kp, b, iv_ptr, iv, add_noise, core_only);
  return assemble_two_pass(c, s, A, candidates, t, out);
}

std::vector<PopAssembled> assemble_population(Ctx* c, const Sorted& s, const sdgp_kernel_desc& d,
                                              const std::vector<const double*>& h, bool add_noise) {
  const int B = (int)h.size();
  require(B >= 1 && B <= 65535, "1..65535 members");
  const int64_t n = s.n;
  const int64_t nc = s.grid.n_cells;
  require(nc < 0x7fffffff, "too many cells");
  const int n1 = d.n1;
  const int n1s = n1 > 0 ? n1 : 1;
  const int64_t np = (int64_t)n1 * d.n2 * (3 + d.dim);
  const int64_t nps = np > 0 ? np : 1;
  std::vector<PopAssembled> out(B);
  std::vector<double> hbp((size_t)B * nps, 0.0);
  for (int m = 0; m < B; ++m) {
    out[m].kp = make_params(d, h[m]);
    for (int64_t k = 0; k < np; ++k) hbp[(size_t)m * nps + k] = h[m][2 + k];
  }
  double* bp = c->get<double>(S_POP_BP, hbp.size());
  SDGP_HIP(hipMemcpyAsync(bp, hbp.data(), hbp.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  double* F = c->get<double>(S_POP_F, (size_t)B * n * n1s);
  uint64_t* M = c->get<uint64_t>(S_POP_M, (size_t)B * n);
  uint64_t* cm = c->get<uint64_t>(S_POP_CM, (size_t)B * nc);
  std::vector<PopMember> pm(B);
  for (int m = 0; m < B; ++m) {
    PopMember& P = pm[m];
    std::memset(&P, 0, sizeof(P));
    P.bp = bp + (size_t)m * nps;
    P.F = F + (size_t)m * n * n1s;
    P.M = M + (size_t)m * n;
    P.cm = cm + (size_t)m * nc;
    out[m].b.bp = const_cast<double*>(P.bp);
    out[m].b.F = P.F;
    out[m].b.M = P.M;
  }
  PopMember* dpm = c->get<PopMember>(S_POP_ARGS, B);
  // each upload copies from a snapshot that lives until the function's
  // last synchronisation, so pm may change while a copy is pending
  std::deque<std::vector<PopMember>> snaps;
  auto upload = [&]() {
    snaps.push_back(pm);
    SDGP_HIP(hipMemcpyAsync(dpm, snaps.back().data(), B * sizeof(PopMember), hipMemcpyHostToDevice, c->stream));
  };
  upload();
  const unsigned gn = (unsigned)grid_for(n, kBlock), gc = (unsigned)grid_for(nc, kBlock);
  // bump values and masks, cell masks
  k_bumps_pop<<<dim3(gn, 1, B), kBlock, 0, c->stream>>>(s.xs, n, d.dim, n1, d.n2, dpm);
  SDGP_CHECK_LAUNCH();
  k_cellmask_pop<<<dim3(gc, 1, B), kBlock, 0, c->stream>>>(s.cell_start, nc, dpm);
  SDGP_CHECK_LAUNCH();
  // bump-function cell runs (SUM)
  IvArgs A;
  A.g = s.grid;
  A.cell_start = s.cell_start;
  A.cm = nullptr;
  A.run_ptr = nullptr;
  A.runs = nullptr;
  A.use_bumps = (d.combine == SDGP_COMBINE_SUM && n1 > 0) ? 1 : 0;
  A.n1 = n1;
  if (A.use_bumps) {
    int32_t* run_ptr = nullptr;
    int4* runs = nullptr;
    bump_runs(c, cm, s.cell_start, nc, n1, B, S_POP_RUNCNT, S_POP_RUNPOS, S_POP_RUNPTR, S_POP_RUNS, &run_ptr,
              &runs);
    for (int m = 0; m < B; ++m) {
      pm[m].run_ptr = run_ptr + (size_t)m * (n1 + 1);
      pm[m].runs = runs;                     // run pointers index the one array of all members
    }
  }
  // candidate intervals per cell: counts, one scan over all members'
  // concatenated counts (global offsets into one interval array), fill
  int32_t* iv_cnt = c->get<int32_t>(S_POP_IVCNT, (size_t)B * (nc + 1));
  SDGP_HIP(hipMemsetAsync(iv_cnt, 0, (size_t)B * (nc + 1) * sizeof(int32_t), c->stream));
  int32_t* iv_ptr = c->get<int32_t>(S_POP_IVPTR, (size_t)B * (nc + 1));
  for (int m = 0; m < B; ++m) {
    pm[m].iv_cnt = iv_cnt + (size_t)m * (nc + 1);
    pm[m].iv_ptr = iv_ptr + (size_t)m * (nc + 1);
  }
  upload();
  k_cell_intervals_pop<false><<<dim3(gc, 1, B), kBlock, 0, c->stream>>>(A, dpm);
  SDGP_CHECK_LAUNCH();
  if (A.use_bumps) {
    k_cell_intervals_wave_pop<false><<<dim3(wave_cell_grid(nc), 1, B), kBlock, 0, c->stream>>>(A, dpm);
    SDGP_CHECK_LAUNCH();
  }
  require((int64_t)B * (nc + 1) < 0x7fffffffLL, "population too large for one interval scan");
  {
    size_t tb = 0;
    SDGP_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, iv_cnt, iv_ptr, (int)(B * (nc + 1)), c->stream));
    void* tmp = c->get<char>(S_SORT_TMP, tb);
    SDGP_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, iv_cnt, iv_ptr, (int)(B * (nc + 1)), c->stream));
  }
  int32_t iv_total = 0;
  SDGP_HIP(hipMemcpyAsync(&iv_total, iv_ptr + (size_t)B * (nc + 1) - 1, sizeof(int32_t), hipMemcpyDeviceToHost,
                          c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  require(iv_total >= 0, "too many candidate intervals");
  int2* iv = c->get<int2>(S_POP_IV, (size_t)std::max<int32_t>(iv_total, 1));
  for (int m = 0; m < B; ++m) pm[m].iv = iv;
  upload();
  k_cell_intervals_pop<true><<<dim3(gc, 1, B), kBlock, 0, c->stream>>>(A, dpm);
  SDGP_CHECK_LAUNCH();
  if (A.use_bumps) {
    k_cell_intervals_wave_pop<true><<<dim3(wave_cell_grid(nc), 1, B), kBlock, 0, c->stream>>>(A, dpm);
    SDGP_CHECK_LAUNCH();
  }
  // count: row lengths of every member; one scan; row pointers rebased per
  // member so that each member's CSR starts at 0
  int64_t* row_nnz = c->get<int64_t>(S_POP_ROWNNZ, (size_t)B * (n + 1));
  SDGP_HIP(hipMemsetAsync(row_nnz, 0, (size_t)B * (n + 1) * sizeof(int64_t), c->stream));
  unsigned long long* cand = c->get<unsigned long long>(S_POP_CAND, B);
  SDGP_HIP(hipMemsetAsync(cand, 0, B * sizeof(unsigned long long), c->stream));
  std::vector<RowArgs> ra(B);
  for (int m = 0; m < B; ++m) {
    Bumps bm;
    bm.F = pm[m].F;
    bm.M = pm[m].M;
    bm.bp = const_cast<double*>(pm[m].bp);
    ra[m] = row_args(s, out[m].kp, bm, pm[m].iv_ptr, iv, add_noise, false);
    pm[m].row_nnz = row_nnz + (size_t)m * (n + 1);
    pm[m].cand = cand + m;
  }
  RowArgs* dra = c->get<RowArgs>(S_POP_RARGS, B);
  SDGP_HIP(hipMemcpyAsync(dra, ra.data(), B * sizeof(RowArgs), hipMemcpyHostToDevice, c->stream));
  upload();
  k_cell_cands_pop<<<dim3(gc, 1, B), kBlock, 0, c->stream>>>(s.cell_start, nc, dpm);
  SDGP_CHECK_LAUNCH();
  launch_cell_rows_pop<false>(s.grid.dim, dim3((unsigned)nc, 1, B), c->stream, dra, dpm);
  SDGP_CHECK_LAUNCH();
  int64_t* scan = c->get<int64_t>(S_POP_SCAN, (size_t)B * (n + 1));
  require((int64_t)B * (n + 1) < 0x7fffffffLL, "population too large for one row scan");
  {
    size_t tb = 0;
    SDGP_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, row_nnz, scan, (int)(B * (n + 1)), c->stream));
    void* tmp = c->get<char>(S_SORT_TMP, tb);
    SDGP_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, row_nnz, scan, (int)(B * (n + 1)), c->stream));
  }
  int64_t* row_ptr = c->get<int64_t>(S_POP_ROWPTR, (size_t)B * (n + 1));
  k_rebase_pop<<<dim3((unsigned)grid_for(n + 1, kBlock), 1, B), kBlock, 0, c->stream>>>(scan, n, row_ptr);
  SDGP_CHECK_LAUNCH();
  std::vector<int64_t> base((size_t)B + 1);
  for (int m = 0; m < B; ++m)
    SDGP_HIP(hipMemcpyAsync(&base[m], scan + (size_t)m * (n + 1), sizeof(int64_t), hipMemcpyDeviceToHost,
                            c->stream));
  SDGP_HIP(hipMemcpyAsync(&base[B], scan + (size_t)B * (n + 1) - 1, sizeof(int64_t), hipMemcpyDeviceToHost,
                          c->stream));
  std::vector<unsigned long long> hcand(B);
  SDGP_HIP(hipMemcpyAsync(hcand.data(), cand, B * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  const int64_t total = base[B];
  int32_t* col = c->get<int32_t>(S_POP_COL, (size_t)std::max<int64_t>(total, 1));
  double* val = c->get<double>(S_POP_VAL, (size_t)std::max<int64_t>(total, 1));
  for (int m = 0; m < B; ++m) {
    pm[m].row_ptr = row_ptr + (size_t)m * (n + 1);
    pm[m].col = col + base[m];
    pm[m].val = val + base[m];
    Csr& K = out[m].A;
    K.n = n;
    K.nnz = base[m + 1] - base[m];
    K.row_ptr = row_ptr + (size_t)m * (n + 1);
    K.col = pm[m].col;
    K.val = pm[m].val;
    out[m].candidates = (int64_t)hcand[m];
  }
  upload();
  SDGP_HIP(hipStreamSynchronize(c->stream));   // the host copies (snapshots, bp, row arguments) are done
  launch_cell_rows_pop<true>(s.grid.dim, dim3((unsigned)nc, 1, B), c->stream, dra, dpm);
  SDGP_CHECK_LAUNCH();
  return out;
}

Csr assemble_cross(Ctx* c, const Sorted& s, const KParams& kp, const Bumps& b, const double* x0, int64_t n0,
                   const double* h, double** kxx_out) {
  require(x0 != nullptr, "x0 is NULL");
  require(n0 >= 1 && n0 < (int64_t)0x7fffffff, "n0 must be in 1..2^31-2");
  const int dim = kp.dim;
  // finiteness of the test points
  {
    const int nb = std::min<int64_t>(1024, (n0 + kBlock - 1) / kBlock);
    double* part = c->get<double>(S_BBOX, (size_t)nb * 2 * kMaxDim);
    k_bbox<<<nb, kBlock, 0, c->stream>>>(x0, n0, dim, part);
    SDGP_CHECK_LAUNCH();
    std::vector<double> hp((size_t)nb * 2 * kMaxDim);
    SDGP_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    SDGP_HIP(hipStreamSynchronize(c->stream));
    for (int bb = 0; bb < nb; ++bb)
      for (int k = 0; k < dim; ++k)
        require(std::isfinite(hp[bb * 2 * kMaxDim + k]) && std::isfinite(hp[bb * 2 * kMaxDim + kMaxDim + k]),
                "x0 must be finite");
  }
  double4* q = c->get<double4>(S_X0S, n0);
  k_pack_points<<<grid_for(n0, kBlock), kBlock, 0, c->stream>>>(x0, n0, dim, q);
  SDGP_CHECK_LAUNCH();
  const int n1 = kp.n1;
  double* qF = c->get<double>(S_QF, (size_t)n0 * (n1 > 0 ? n1 : 1));
  uint64_t* qm = c->get<uint64_t>(S_QM, n0);
  k_bumps<<<grid_for(n0, kBlock), kBlock, 0, c->stream>>>(q, n0, dim, n1, kp.n2, b.bp, qF, qm);
  SDGP_CHECK_LAUNCH();
  double* kxx = c->get<double>(S_KXX, n0);
  k_prior_diag<<<grid_for(n0, kBlock), kBlock, 0, c->stream>>>(qm, qF, n0, n1, kp.core, dim / 2 + 2, kp.combine,
                                                               kp.sigma2, kxx);
  SDGP_CHECK_LAUNCH();
  // candidate intervals per test point (runs of the last prune())
  IvArgs A;
  A.g = s.grid;
  A.cell_start = s.cell_start;
  A.cm = c->buf[S_CELLMASK].as<uint64_t>();
  A.use_bumps = (kp.combine == SDGP_COMBINE_SUM && kp.n1 > 0) ? 1 : 0;
  A.run_ptr = A.use_bumps ? c->buf[S_RUN_PTR].as<int32_t>() : nullptr;
  A.runs = A.use_bumps ? c->buf[S_RUNS].as<int4>() : nullptr;
  int32_t* iv_cnt = c->get<int32_t>(S_QIV_CNT, n0 + 1);
  SDGP_HIP(hipMemsetAsync(iv_cnt + n0, 0, sizeof(int32_t), c->stream));
  k_query_intervals<false><<<grid_for(n0, kBlock), kBlock, 0, c->stream>>>(A, q, qm, n0, iv_cnt, nullptr, nullptr);
  SDGP_CHECK_LAUNCH();
  int32_t* iv_ptr = c->get<int32_t>(S_QIV_PTR, n0 + 1);
  size_t tb = 0;
  SDGP_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, iv_cnt, iv_ptr, (int)(n0 + 1), c->stream));
  void* tmp = c->get<char>(S_SORT_TMP, tb);
  SDGP_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, iv_cnt, iv_ptr, (int)(n0 + 1), c->stream));
  int32_t total = 0;
  SDGP_HIP(hipMemcpyAsync(&total, iv_ptr + n0, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  int2* iv = c->get<int2>(S_QIV, total > 0 ? total : 1);
  k_query_intervals<true><<<grid_for(n0, kBlock), kBlock, 0, c->stream>>>(A, q, qm, n0, nullptr, iv_ptr, iv);
  SDGP_CHECK_LAUNCH();
  // count, scan, fill
  CrossArgs X;
  X.xs = s.xs; X.M = b.M; X.F = b.F; X.q = q; X.qm = qm; X.qF = qF; X.iv_ptr = iv_ptr; X.iv = iv;
  X.nq = n0; X.dim = dim; X.n1 = n1; X.core = kp.core; X.ell = dim / 2 + 2; X.combine = kp.combine;
  X.sigma2 = kp.sigma2; X.r_core = kp.r_core; X.rc2 = kp.rc2;
  int64_t* rn = c->get<int64_t>(S_QROW_NNZ, n0 + 1);
  SDGP_HIP(hipMemsetAsync(rn + n0, 0, sizeof(int64_t), c->stream));
  const int rpb = kBlock / kWave;
  k_cross_rows<false><<<grid_for(n0, rpb), kBlock, 0, c->stream>>>(X, rn, nullptr, nullptr, nullptr);
  SDGP_CHECK_LAUNCH();
  int64_t* rp = c->get<int64_t>(S_QROW_PTR, n0 + 1);
  tb = 0;
  SDGP_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, rn, rp, (int)(n0 + 1), c->stream));
  tmp = c->get<char>(S_SORT_TMP, tb);
  SDGP_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, rn, rp, (int)(n0 + 1), c->stream));
  int64_t nnz = 0;
  SDGP_HIP(hipMemcpyAsync(&nnz, rp + n0, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  int32_t* col = c->get<int32_t>(S_QCOL, nnz);
  double* val = c->get<double>(S_QVAL, nnz);
  k_cross_rows<true><<<grid_for(n0, rpb), kBlock, 0, c->stream>>>(X, nullptr, rp, col, val);
  SDGP_CHECK_LAUNCH();
  Csr k;
  k.n = n0; k.nnz = nnz; k.row_ptr = rp; k.col = col; k.val = val;
  *kxx_out = kxx;
  (void)h;
  return k;
}

void canonicalize(Ctx* c, const Sorted& s, const Csr& k, int64_t* row_ptr, int32_t* col, double* val) {
  const int64_t n = s.n;
  require(k.nnz < (int64_t)0x7fffffff, "canonical CSR output needs nnz < 2^31");
  int64_t* len = c->get<int64_t>(S_ROWLEN2, n + 1);
  k_canon_len<<<grid_for(n, kBlock), kBlock, 0, c->stream>>>(k.row_ptr, s.perm, n, len);
  SDGP_CHECK_LAUNCH();
  size_t tb = 0;
  SDGP_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, len, row_ptr, (int)(n + 1), c->stream));
  void* tmp = c->get<char>(S_SORT_TMP, tb);
  SDGP_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, len, row_ptr, (int)(n + 1), c->stream));
  int32_t* col2 = c->get<int32_t>(S_COL2, k.nnz);
  double* val2 = c->get<double>(S_VAL2, k.nnz);
  k_canon_copy<<<grid_for(n, kBlock / kWave), kBlock, 0, c->stream>>>(k.row_ptr, k.col, k.val, s.perm, n,
                                                                       row_ptr, col2, val2);
  SDGP_CHECK_LAUNCH();
  int bits = 1;
  while (((int64_t)1 << bits) < n) ++bits;
  tb = 0;
  SDGP_HIP(hipcub::DeviceSegmentedRadixSort::SortPairs(nullptr, tb, col2, col, val2, val, (int)k.nnz, (int)n,
                                                       row_ptr, row_ptr + 1, 0, bits, c->stream));
  tmp = c->get<char>(S_SORT_TMP, tb);
  SDGP_HIP(hipcub::DeviceSegmentedRadixSort::SortPairs(tmp, tb, col2, col, val2, val, (int)k.nnz, (int)n,
                                                       row_ptr, row_ptr + 1, 0, bits, c->stream));
}

}  // namespace sdgp
