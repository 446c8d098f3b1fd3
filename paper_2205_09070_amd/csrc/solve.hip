// Solver helpers on the sparse covariance (Section 2.5): SpMV / SpMM,
// dot products, the low-rank preconditioner, the posterior variance and
// Taylor log-det drivers, and stochastic Lanczos quadrature of ln det A
// from the CG coefficients, for gfx950.  The block CG itself is in cg.hip.
//
// Caller-facing SpMM on row-major [n][R] blocks: R == 1 takes the SpMV
// kernel (16 lanes per row), even R the 32-column slab kernel of cg.hip,
// odd R a one-wavefront-per-row kernel whose 64 lanes hold 64 consecutive
// columns.  Reductions are deterministic (fixed-order block partials).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>
#include <vector>

#include "kernel_math.hpp"
#include "sdgp_internal.hpp"

namespace sdgp {

namespace {

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

// SpMV (one right-hand side): 32 lanes per row, 8 rows per 256-thread block;
// each lane loads 4 of its row's (column, value) pairs (stride 32) and then
// issues their 4 gathers together.  Rows are dealt XCD-aware as in RowSweep;
// many small blocks (about four row groups each) keep the tail short.
constexpr int kSpmvLanes = 32;
constexpr int kSpmvU = 4;
__global__ __launch_bounds__(256) void k_spmv(int64_t n, const int64_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col, const double* __restrict__ val,
                                              const double* __restrict__ x, double* __restrict__ y) {
  constexpr int G = 256 / kSpmvLanes;
  const int sub = threadIdx.x & (kSpmvLanes - 1);
  const int r = threadIdx.x / kSpmvLanes;
  const int xcd = blockIdx.x & 7;
  const int64_t bi = blockIdx.x >> 3, nbx = gridDim.x >> 3;
  const int64_t nx = (n + 7) >> 3, lo = xcd * nx, hi = min(n, lo + nx);
  for (int64_t base = lo + bi * G; base < hi; base += nbx * G) {
    const int64_t a = base + r;
    double acc = 0.0;
    if (a < hi) {
      const int64_t k1 = row_ptr[a + 1];
      for (int64_t k0 = row_ptr[a] + sub; k0 < k1; k0 += kSpmvLanes * kSpmvU) {
        int cj[kSpmvU];
        double vj[kSpmvU];
#pragma unroll
        for (int u = 0; u < kSpmvU; ++u) {
          const int64_t k = k0 + kSpmvLanes * u;
          cj[u] = k < k1 ? col[k] : 0;
          vj[u] = k < k1 ? val[k] : 0.0;
        }
        double xv[kSpmvU];
#pragma unroll
        for (int u = 0; u < kSpmvU; ++u) xv[u] = x[cj[u]];
#pragma unroll
        for (int u = 0; u < kSpmvU; ++u) acc += vj[u] * xv[u];
      }
    }
#pragma unroll
    for (int o = kSpmvLanes / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kSpmvLanes);
    if (a < hi && sub == 0) y[a] = acc;
  }
}

// SpMV with paired loads: 32 lanes per row, two rows per wavefront, 8 rows
// per 256-thread block (measured at 1M points, ~90 entries per row: 32
// lanes 0.341 ms, 16 lanes 0.366, 8 lanes 0.479, 64 lanes 0.383; two rows
// per lane group or more pairs in flight no faster).  A row's entries are
// read in 16-byte-aligned pairs
// (one 8-byte column pair and one 16-byte value pair per lane; pair halves
// outside the row are masked), two pairs per lane in flight and their four
// gathers issued together.  A pair is only loaded whole when its second
// entry exists in the arrays (nnz = row_ptr[n]); the last entry of the
// matrix is read alone.  Needs val 16-byte and col 8-byte aligned.
constexpr int kSpw = 32;
__global__ __launch_bounds__(256) void k_spmv_w(int64_t n, const int64_t* __restrict__ row_ptr,
                                                const int32_t* __restrict__ col, const double* __restrict__ val,
                                                const double* __restrict__ x, double* __restrict__ y) {
  constexpr int G = 256 / kSpw;
  const int64_t nnz = row_ptr[n];
  const int sub = threadIdx.x & (kSpw - 1);
  const int r = threadIdx.x / kSpw;
  const int xcd = blockIdx.x & 7;
  const int64_t bi = blockIdx.x >> 3, nbx = gridDim.x >> 3;
  const int64_t nx = (n + 7) >> 3, lo = xcd * nx, hi = min(n, lo + nx);
  for (int64_t base = lo + bi * G; base < hi; base += nbx * G) {
    const int64_t a = base + r;
    double acc = 0.0;
    if (a < hi) {
      const int64_t k0 = row_ptr[a], k1 = row_ptr[a + 1];
      for (int64_t e = (k0 & ~(int64_t)1) + 2 * sub; e < k1; e += 4 * kSpw) {
        int cj[4] = {0, 0, 0, 0};
        double vj[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int64_t ep = e + 2 * kSpw * h;
          if (ep < k1) {
            if (ep + 1 < nnz) {
              const int2 cc = *reinterpret_cast<const int2*>(col + ep);
              const double2 vv = *reinterpret_cast<const double2*>(val + ep);
              cj[2 * h] = cc.x;
              cj[2 * h + 1] = cc.y;
              vj[2 * h] = ep >= k0 ? vv.x : 0.0;
              vj[2 * h + 1] = ep + 1 < k1 ? vv.y : 0.0;
            } else {
              cj[2 * h] = col[ep];
              vj[2 * h] = ep >= k0 ? val[ep] : 0.0;
            }
          }
        }
        double xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = x[cj[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += vj[u] * xv[u];
      }
    }
#pragma unroll
    for (int o = kSpw / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kSpw);
    if (a < hi && sub == 0) y[a] = acc;
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
    const bool aligned = (reinterpret_cast<uintptr_t>(A.val) % 16) == 0 && (reinterpret_cast<uintptr_t>(A.col) % 8) == 0;
    if (aligned) {
      // 8 rows per block step, up to 65528 blocks
      int64_t blocks = std::min<int64_t>((A.n + 7) / 8, 65528);
      blocks = std::max<int64_t>(8, (blocks + 7) / 8 * 8);
      k_spmv_w<<<(unsigned)blocks, 256, 0, c->stream>>>(A.n, A.row_ptr, A.col, A.val, X, Y);
      SDGP_CHECK_LAUNCH();
      return;
    }
    // 8 rows per block step, up to 32768 blocks
    int64_t blocks = std::min<int64_t>((A.n + 7) / 8, 32768);
    blocks = std::max<int64_t>(8, (blocks + 7) / 8 * 8);
    k_spmv<<<(unsigned)blocks, 256, 0, c->stream>>>(A.n, A.row_ptr, A.col, A.val, X, Y);
    SDGP_CHECK_LAUNCH();
    return;
  }
  if (R % 2 == 0 && (reinterpret_cast<uintptr_t>(X) % 16) == 0 && (reinterpret_cast<uintptr_t>(Y) % 16) == 0) {
    spmm_slab(c, A, X, R, Y);
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
  // population form: member blockIdx.z's F (stride n * n1) and partials
  F += (int64_t)blockIdx.z * n * n1;
  part += (int64_t)blockIdx.z * gridDim.x * n1 * n1;
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

}  // namespace

namespace {

// c and ln det M of the low-rank preconditioner, without the bump part.
Precond lowrank_base(const KParams& kp, int64_t n, const double* F) {
  Precond pc;
  const double psi0 = kp.core == SDGP_CORE_KSTAT ? 0.26596152026762178529 : 1.0;
  pc.c = kp.sigma2 * psi0 + kp.noise;
  require(pc.c > 0.0, "the low-rank preconditioner needs sigma2 psi(0) + noise_var > 0");
  pc.n1 = kp.n1;
  pc.F = F;
  if (kp.n1 == 0) pc.logdetM = (double)n * std::log(pc.c);
  return pc;
}

// From the Gram partials hp[nbk][n1*n1]: S = c I + F^T F, its Cholesky
// factor, ln det M and S^{-1} (into Si, host).
void lowrank_finish(Precond& pc, int64_t n, int64_t nbk, const double* hp, std::vector<double>& Si) {
  const int n1 = pc.n1;
  const int np = n1 * n1;
  std::vector<double> S((size_t)np, 0.0), L((size_t)np, 0.0);
  Si.assign((size_t)np, 0.0);
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
  pc.logdetM = (double)(n - n1) * std::log(pc.c) + logdetS;
}

}  // namespace

Precond lowrank_precond(Ctx* c, const Sorted& s, const KParams& kp, const Bumps& b) {
  const int64_t n = s.n;
  Precond pc = lowrank_base(kp, n, b.F);
  const int n1 = kp.n1;
  if (n1 == 0) return pc;
  const int64_t nbk = std::min<int64_t>(256, (n + 4095) / 4096);
  const int64_t slab = (n + nbk - 1) / nbk;
  const int np = n1 * n1;
  double* part = c->get<double>(S_PC_PART, (size_t)nbk * np);
  k_gram<<<(unsigned)nbk, 256, 0, c->stream>>>(b.F, n, n1, slab, part);
  SDGP_CHECK_LAUNCH();
  std::vector<double> hp((size_t)nbk * np);
  SDGP_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  std::vector<double> Si;
  lowrank_finish(pc, n, nbk, hp.data(), Si);
  double* dSi = c->get<double>(S_PC_SINV, np);
  SDGP_HIP(hipMemcpyAsync(dSi, Si.data(), np * sizeof(double), hipMemcpyHostToDevice, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  pc.Sinv = dSi;
  return pc;
}

std::vector<Precond> lowrank_precond_pop(Ctx* c, const Sorted& s, const std::vector<KParams>& kp,
                                         const double* F0, std::vector<std::string>* failed) {
  const int B = (int)kp.size();
  const int64_t n = s.n;
  const int n1 = B > 0 ? kp[0].n1 : 0;
  const int n1s = n1 > 0 ? n1 : 1;
  std::vector<Precond> pcs(B);
  failed->assign(B, std::string());
  for (int m = 0; m < B; ++m) {
    try {
      pcs[m] = lowrank_base(kp[m], n, F0 + (size_t)m * n * n1s);
    } catch (const Error& e) {
      (*failed)[m] = e.what();
    }
  }
  if (n1 == 0 || B == 0) return pcs;
  const int64_t nbk = std::min<int64_t>(256, (n + 4095) / 4096);
  const int64_t slab = (n + nbk - 1) / nbk;
  const int np = n1 * n1;
  double* part = c->get<double>(S_POP_GRAM, (size_t)B * nbk * np);
  k_gram<<<dim3((unsigned)nbk, 1, B), 256, 0, c->stream>>>(F0, n, n1, slab, part);
  SDGP_CHECK_LAUNCH();
  std::vector<double> hp((size_t)B * nbk * np);
  SDGP_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  std::vector<double> all((size_t)B * np), Si;
  for (int m = 0; m < B; ++m) {
    if (!(*failed)[m].empty()) continue;
    try {
      lowrank_finish(pcs[m], n, nbk, hp.data() + (size_t)m * nbk * np, Si);
      std::copy(Si.begin(), Si.end(), all.begin() + (size_t)m * np);
    } catch (const Error& e) {
      (*failed)[m] = e.what();
    }
  }
  double* dSi = c->get<double>(S_POP_SINV, all.size());
  SDGP_HIP(hipMemcpyAsync(dSi, all.data(), all.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  for (int m = 0; m < B; ++m) pcs[m].Sinv = dSi + (size_t)m * np;
  return pcs;
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
