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
#include <cmath>
#include <vector>

#include "kernel_math.hpp"
#include "sdgp_internal.hpp"

namespace sdgp {

namespace {

constexpr int kCgBlock = 1024;             // 16 wavefronts
constexpr int kCgWaves = kCgBlock / kWave;

// y = sum_k val[k] X[col[k], rc] over one CSR row (the calling wave's row).
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
    for (; j + 4 <= cnt; j += 4) {
      const int c0 = readlane_i32(cj, j), c1 = readlane_i32(cj, j + 1);
      const int c2 = readlane_i32(cj, j + 2), c3 = readlane_i32(cj, j + 3);
      const double x0 = Xc[(int64_t)c0 * R], x1 = Xc[(int64_t)c1 * R];
      const double x2 = Xc[(int64_t)c2 * R], x3 = Xc[(int64_t)c3 * R];
      acc += readlane_f64(vj, j) * x0;
      acc += readlane_f64(vj, j + 1) * x1;
      acc += readlane_f64(vj, j + 2) * x2;
      acc += readlane_f64(vj, j + 3) * x3;
    }
    for (; j < cnt; ++j) acc += readlane_f64(vj, j) * Xc[(int64_t)readlane_i32(cj, j) * R];
  }
  return acc;
}

// Plain SpMM: Y = A X (one wave per row, lanes over a 64-column chunk).
__global__ __launch_bounds__(256) void k_spmm(int64_t n, const int64_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col, const double* __restrict__ val,
                                              const double* __restrict__ X, int R, double* __restrict__ Y) {
  const int64_t a = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  if (a >= n) return;
  const int rc = blockIdx.y * kWave + lane_id();
  const int rcc = rc < R ? rc : R - 1;
  const double v = row_dot(row_ptr[a], row_ptr[a + 1], col, val, X + rcc, R);
  if (rc < R) Y[a * (int64_t)R + rc] = v;
}

struct CgState {
  double* rr;       // [2][R] parity buffers of r.r
  int32_t* act;     // [2][R] active flags
  int32_t* failed;  // [R] p^T A p <= 0 met
  double* bnorm2;   // [R]
  int32_t* iters;   // [R]
  int32_t* done;    // [1]
  int32_t* not_spd; // [1]
  double* hist_a;   // [max_iter][R]
  double* hist_b;   // [max_iter][R]
};

// Fixed-order reduction of per-block partials part[b][r] (b < nb) for the
// 64-column chunk of this block into sh[0..63].  All blocks get identical
// values.
__device__ void chunk_reduce(const double* __restrict__ part, int nb, int R, double* sh, double* scratch) {
  const int t = threadIdx.x;
  const int l = t & 63, w = t >> 6;
  const int rc = blockIdx.y * kWave + l;
  double s = 0.0;
  if (rc < R)
    for (int b = w; b < nb; b += kCgWaves) s += part[(int64_t)b * R + rc];
  scratch[w * kWave + l] = s;
  __syncthreads();
  if (t < kWave) {
    double tot = 0.0;
    for (int q = 0; q < kCgWaves; ++q) tot += scratch[q * kWave + t];
    sh[t] = tot;
  }
  __syncthreads();
}

// Block partial of per-lane values over the block's waves.
__device__ void block_partial(double v, double* scratch, double* part, int R) {
  const int t = threadIdx.x;
  const int l = t & 63, w = t >> 6;
  scratch[w * kWave + l] = v;
  __syncthreads();
  if (t < kWave) {
    double tot = 0.0;
    for (int q = 0; q < kCgWaves; ++q) tot += scratch[q * kWave + t];
    const int rc = blockIdx.y * kWave + t;
    if (rc < R) part[(int64_t)blockIdx.x * R + rc] = tot;
  }
}

struct CgArgs {
  int64_t n;
  int R;
  const int64_t* row_ptr;
  const int32_t* col;
  const double* val;
  double *X, *Rr, *P, *Q;
  double* part;     // [nb][R]
  int nb;
  CgState st;
  double rtol2;
};

// Q = A P, partial p.q per column.
__global__ __launch_bounds__(kCgBlock) void k_cg_spmm(CgArgs A) {
  if (*A.st.done) return;
  __shared__ double scratch[kCgBlock];
  const int lane = lane_id();
  const int rc = blockIdx.y * kWave + lane;
  const int rcc = rc < A.R ? rc : A.R - 1;
  const int64_t R = A.R;
  const int64_t W = (int64_t)gridDim.x * kCgWaves;
  double pq = 0.0;
  for (int64_t a = blockIdx.x * (int64_t)kCgWaves + (threadIdx.x >> 6); a < A.n; a += W) {
    const double q = row_dot(A.row_ptr[a], A.row_ptr[a + 1], A.col, A.val, A.P + rcc, R);
    if (rc < A.R) {
      A.Q[a * R + rc] = q;
      pq += A.P[a * R + rc] * q;
    }
  }
  block_partial(pq, scratch, A.part, A.R);
}

// alpha = r.r / p.q; x += alpha p; r -= alpha q; partial r.r.
__global__ __launch_bounds__(kCgBlock) void k_cg_update_xr(CgArgs A, int it) {
  if (*A.st.done) return;
  __shared__ double scratch[kCgBlock];
  __shared__ double pAp[kWave];
  chunk_reduce(A.part, A.nb, A.R, pAp, scratch);
  const int lane = lane_id();
  const int rc = blockIdx.y * kWave + lane;
  const int par = it & 1;
  double alpha = 0.0;
  bool act = false;
  if (rc < A.R) {
    act = A.st.act[par * A.R + rc] != 0;
    if (act) {
      const double d = pAp[lane];
      if (d > 0.0 && isfinite(d)) alpha = A.st.rr[par * A.R + rc] / d;
      else act = false;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < kWave && rc < A.R) {
    const bool was = A.st.act[par * A.R + rc] != 0;
    if (was) A.st.hist_a[(int64_t)it * A.R + rc] = alpha;
    if (was && !act) { A.st.failed[rc] = 1; *A.st.not_spd = 1; }
  }
  __syncthreads();
  const int64_t R = A.R;
  const int64_t W = (int64_t)gridDim.x * kCgWaves;
  double rr = 0.0;
  for (int64_t a = blockIdx.x * (int64_t)kCgWaves + (threadIdx.x >> 6); a < A.n; a += W) {
    if (act) {
      const int64_t o = a * R + rc;
      A.X[o] += alpha * A.P[o];
      const double r = A.Rr[o] - alpha * A.Q[o];
      A.Rr[o] = r;
      rr += r * r;
    }
  }
  __syncthreads();
  block_partial(rr, scratch, A.part, A.R);
}

// beta = r.r_new / r.r; convergence test; p = r + beta p.
__global__ __launch_bounds__(kCgBlock) void k_cg_update_p(CgArgs A, int it) {
  if (*A.st.done) return;
  __shared__ double scratch[kCgBlock];
  __shared__ double rrn[kWave];
  chunk_reduce(A.part, A.nb, A.R, rrn, scratch);
  const int lane = lane_id();
  const int rc = blockIdx.y * kWave + lane;
  const int par = it & 1, nxt = par ^ 1;
  double beta = 0.0;
  bool cont = false;
  bool act = false;
  double rr_new = 0.0, rr_old = 0.0;
  if (rc < A.R) {
    act = A.st.act[par * A.R + rc] != 0 && A.st.failed[rc] == 0;
    rr_old = A.st.rr[par * A.R + rc];
    rr_new = rrn[lane];
    if (act) {
      beta = rr_new / rr_old;
      cont = !(rr_new <= A.rtol2 * A.st.bnorm2[rc]);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < kWave && rc < A.R) {
    A.st.rr[nxt * A.R + rc] = act ? rr_new : rr_old;
    A.st.act[nxt * A.R + rc] = cont ? 1 : 0;
    if (act) {
      A.st.hist_b[(int64_t)it * A.R + rc] = beta;
      A.st.iters[rc] += 1;
    }
  }
  const int64_t R = A.R;
  const int64_t W = (int64_t)gridDim.x * kCgWaves;
  for (int64_t a = blockIdx.x * (int64_t)kCgWaves + (threadIdx.x >> 6); a < A.n; a += W) {
    if (cont) {
      const int64_t o = a * R + rc;
      A.P[o] = A.Rr[o] + beta * A.P[o];
    }
  }
}

// Records the executed iteration count in done when no column is active
// (one block, after update_p).
__global__ void k_cg_check(CgArgs A, int it) {
  const int nxt = (it & 1) ^ 1;
  __shared__ int left;
  if (threadIdx.x == 0) left = 0;
  __syncthreads();
  int mine = 0;
  for (int r = threadIdx.x; r < A.R; r += blockDim.x) mine |= A.st.act[nxt * A.R + r];
  if (mine) atomicOr(&left, 1);
  __syncthreads();
  if (threadIdx.x == 0 && !left) *A.st.done = it + 1;
}

// Right-hand sides and CG initial state (x = 0, r = p = b).
__global__ void k_cg_init(CgArgs A, const double* __restrict__ ys, const int32_t* __restrict__ perm,
                          int kind, uint64_t seed, const double* __restrict__ dense) {
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
    const uint64_t k = ((uint64_t)(r - 1) << 32) + (uint64_t)perm[a] + 1ull;
    b = (splitmix64_at(seed, k) >> 63) ? -1.0 : 1.0;
  }
  A.X[idx] = 0.0;
  A.Rr[idx] = b;
  A.P[idx] = b;
}

// Column norms of b (fixed-order partials then one block).
__global__ __launch_bounds__(kCgBlock) void k_cg_norm_part(CgArgs A) {
  __shared__ double scratch[kCgBlock];
  const int rc = blockIdx.y * kWave + lane_id();
  const int64_t R = A.R;
  const int64_t W = (int64_t)gridDim.x * kCgWaves;
  double s = 0.0;
  if (rc < A.R)
    for (int64_t a = blockIdx.x * (int64_t)kCgWaves + (threadIdx.x >> 6); a < A.n; a += W) {
      const double v = A.Rr[a * R + rc];
      s += v * v;
    }
  block_partial(s, scratch, A.part, A.R);
}

__global__ __launch_bounds__(kCgBlock) void k_cg_norm_fin(CgArgs A) {
  __shared__ double scratch[kCgBlock];
  __shared__ double nrm[kWave];
  chunk_reduce(A.part, A.nb, A.R, nrm, scratch);
  if (blockIdx.x != 0) return;
  const int t = threadIdx.x;
  const int rc = blockIdx.y * kWave + t;
  if (t < kWave && rc < A.R) {
    A.st.bnorm2[rc] = nrm[t];
    A.st.rr[rc] = nrm[t];
    A.st.rr[A.R + rc] = nrm[t];
    A.st.act[rc] = nrm[t] > 0.0 ? 1 : 0;
    A.st.act[A.R + rc] = 0;
    A.st.failed[rc] = 0;
    A.st.iters[rc] = 0;
  }
}

// ------------------------------------------------------------------- SLQ
// One thread per probe column: build the Lanczos tridiagonal from the CG
// coefficients (T_00 = 1/a_0, T_kk = 1/a_k + b_{k-1}/a_{k-1},
// T_k,k+1 = sqrt(b_k)/a_k), diagonalise it by the implicit QL method with
// Wilkinson shifts (Bowdler, Martin, Reinsch, Wilkinson 1968), carrying only
// the first row of the eigenvector matrix, and return
// e_1^T ln(T) e_1 = sum_j tau_j^2 ln theta_j and the extreme Ritz values.
__global__ void k_slq(const double* __restrict__ ha, const double* __restrict__ hb,
                      const int32_t* __restrict__ iters, int R, int col0, int ncols, int mcap,
                      int64_t stride, double* __restrict__ d, double* __restrict__ e,
                      double* __restrict__ z, double* __restrict__ out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ncols) return;
  const int r = col0 + p;
  int m = iters[r];
  if (mcap > 0 && m > mcap) m = mcap;
  double* D = d + p;
  double* E = e + p;
  double* Z = z + p;
#define AT(arr, k) arr[(int64_t)(k) * stride]
  if (m <= 0) {
    out[p * 4 + 0] = 0.0; out[p * 4 + 1] = 0.0; out[p * 4 + 2] = INFINITY; out[p * 4 + 3] = -INFINITY;
    return;
  }
  for (int k = 0; k < m; ++k) {
    const double ak = ha[(int64_t)k * R + r];
    double dk = 1.0 / ak;
    if (k > 0) dk += hb[(int64_t)(k - 1) * R + r] / ha[(int64_t)(k - 1) * R + r];
    AT(D, k) = dk;
    AT(E, k) = (k + 1 < m) ? sqrt(hb[(int64_t)k * R + r]) / ak : 0.0;
    AT(Z, k) = (k == 0) ? 1.0 : 0.0;
  }
  bool ok = true;
  for (int l = 0; l < m && ok; ++l) {
    for (int iter = 0;; ++iter) {
      int mm = l;
      for (; mm < m - 1; ++mm) {
        const double dd = fabs(AT(D, mm)) + fabs(AT(D, mm + 1));
        if (fabs(AT(E, mm)) <= 1e-16 * dd) break;
      }
      if (mm == l) break;
      if (iter >= 60) { ok = false; break; }
      double g = (AT(D, l + 1) - AT(D, l)) / (2.0 * AT(E, l));
      double rr = hypot(g, 1.0);
      g = AT(D, mm) - AT(D, l) + AT(E, l) / (g + copysign(rr, g));
      double s = 1.0, c = 1.0, pp = 0.0;
      bool deflated = false;
      for (int i = mm - 1; i >= l; --i) {
        double f = s * AT(E, i);
        const double b = c * AT(E, i);
        rr = hypot(f, g);
        AT(E, i + 1) = rr;
        if (rr == 0.0) {
          AT(D, i + 1) -= pp;
          AT(E, mm) = 0.0;
          deflated = true;
          break;
        }
        s = f / rr;
        c = g / rr;
        g = AT(D, i + 1) - pp;
        rr = (AT(D, i) - g) * s + 2.0 * c * b;
        pp = s * rr;
        AT(D, i + 1) = g + pp;
        g = c * rr - b;
        f = AT(Z, i + 1);
        AT(Z, i + 1) = s * AT(Z, i) + c * f;
        AT(Z, i) = c * AT(Z, i) - s * f;
      }
      if (deflated) continue;
      AT(D, l) -= pp;
      AT(E, l) = g;
      AT(E, mm) = 0.0;
    }
  }
  double q = 0.0, lo = INFINITY, hi = -INFINITY;
  bool pos = ok;
  for (int k = 0; k < m; ++k) {
    const double th = AT(D, k);
    const double tau = AT(Z, k);
    if (!(th > 0.0)) pos = false;
    lo = fmin(lo, th);
    hi = fmax(hi, th);
    q += tau * tau * log(th);
  }
#undef AT
  out[p * 4 + 0] = pos ? q : NAN;
  out[p * 4 + 1] = (double)m;
  out[p * 4 + 2] = lo;
  out[p * 4 + 3] = hi;
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

inline int cg_nb(int64_t n, int R) {
  const int chunks = (R + kWave - 1) / kWave;
  int64_t nb = std::max<int64_t>(1, 512 / chunks);
  nb = std::min<int64_t>(nb, (n + kCgWaves - 1) / kCgWaves);
  return (int)std::max<int64_t>(nb, 1);
}

}  // namespace

void spmm(Ctx* c, const Csr& A, const double* X, int R, double* Y) {
  require(R >= 1 && R <= (1 << 20), "R must be in 1..2^20");
  const int64_t blocks = (A.n + 3) / 4;
  require(blocks < 0x7fffffff, "n too large");
  dim3 grid((unsigned)blocks, (unsigned)((R + kWave - 1) / kWave));
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

CgResult block_cg(Ctx* c, const Csr& Am, const Sorted& s, const double* ys, int kind, int P, uint64_t seed,
                  double rtol, int max_iter, const double* dense_rhs, int dense_R, PhaseTimer* t) {
  const int64_t n = Am.n;
  int R;
  if (kind == PK_DENSE) R = dense_R;
  else if (kind == PK_IDENTITY) R = (int)(1 + n);
  else if (kind == PK_NONE) R = 1;
  else R = 1 + P;
  require(R >= 1, "no right-hand sides");
  require(max_iter >= 1, "cg_max_iter must be >= 1");
  require(rtol > 0.0 && std::isfinite(rtol), "cg_rtol must be > 0");
  const size_t NR = (size_t)n * R;
  CgArgs A;
  A.n = n;
  A.R = R;
  A.row_ptr = Am.row_ptr;
  A.col = Am.col;
  A.val = Am.val;
  A.X = c->get<double>(S_CG_X, NR);
  A.Rr = c->get<double>(S_CG_R, NR);
  A.P = c->get<double>(S_CG_P, NR);
  A.Q = c->get<double>(S_CG_Q, NR);
  const int nb = cg_nb(n, R);
  const int chunks = (R + kWave - 1) / kWave;
  A.nb = nb;
  A.part = c->get<double>(S_CG_PART, (size_t)nb * R);
  // state block
  size_t words = 2 * (size_t)R + R + 2 + 2 * (size_t)R + R + 8;
  char* sb = c->get<char>(S_CG_STATE, words * 8 + 64);
  A.st.rr = reinterpret_cast<double*>(sb);
  A.st.bnorm2 = A.st.rr + 2 * (size_t)R;
  int32_t* ib = reinterpret_cast<int32_t*>(A.st.bnorm2 + R);
  A.st.act = ib;
  A.st.failed = ib + 2 * (size_t)R;
  A.st.iters = A.st.failed + R;
  A.st.done = A.st.iters + R;
  A.st.not_spd = A.st.done + 1;
  A.st.hist_a = c->get<double>(S_CG_HIST_A, (size_t)max_iter * R);
  A.st.hist_b = c->get<double>(S_CG_HIST_B, (size_t)max_iter * R);
  A.rtol2 = rtol * rtol;
  SDGP_HIP(hipMemsetAsync(A.st.done, 0, 2 * sizeof(int32_t), c->stream));
  {
    const int64_t tot = (int64_t)NR;
    const int64_t g = (tot + 255) / 256;
    require(g < 0x7fffffff, "n*R too large");
    k_cg_init<<<(unsigned)g, 256, 0, c->stream>>>(A, ys, s.perm, kind, seed, dense_rhs);
    SDGP_CHECK_LAUNCH();
  }
  dim3 grid(nb, chunks);
  k_cg_norm_part<<<grid, kCgBlock, 0, c->stream>>>(A);
  SDGP_CHECK_LAUNCH();
  k_cg_norm_fin<<<dim3(1, chunks), kCgBlock, 0, c->stream>>>(A);
  SDGP_CHECK_LAUNCH();
  // iterate; poll the done flag now and then
  int it = 0;
  int check = 8;
  int32_t flags[2] = {0, 0};
  c->spmm_events.clear();
  while (it < max_iter) {
    const int upto = std::min(max_iter, it + check);
    for (; it < upto; ++it) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (c->timing) { e0 = c->event(); SDGP_HIP(hipEventRecord(e0, c->stream)); }
      k_cg_spmm<<<grid, kCgBlock, 0, c->stream>>>(A);
      SDGP_CHECK_LAUNCH();
      if (c->timing) {
        e1 = c->event();
        SDGP_HIP(hipEventRecord(e1, c->stream));
        c->spmm_events.push_back({e0, e1});
      }
      k_cg_update_xr<<<grid, kCgBlock, 0, c->stream>>>(A, it);
      SDGP_CHECK_LAUNCH();
      k_cg_update_p<<<grid, kCgBlock, 0, c->stream>>>(A, it);
      SDGP_CHECK_LAUNCH();
      k_cg_check<<<1, 256, 0, c->stream>>>(A, it);
      SDGP_CHECK_LAUNCH();
    }
    SDGP_HIP(hipMemcpyAsync(flags, A.st.done, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    SDGP_HIP(hipStreamSynchronize(c->stream));
    if (flags[0] || flags[1]) break;
    check = std::min(check * 2, 64);
  }
  CgResult res;
  res.R = R;
  res.X = A.X;
  res.hist_a = A.st.hist_a;
  res.hist_b = A.st.hist_b;
  res.col_iters = A.st.iters;
  res.not_spd = flags[1] != 0;
  std::vector<int32_t> its(R);
  std::vector<double> rr(2 * (size_t)R), bn(R);
  SDGP_HIP(hipMemcpyAsync(its.data(), A.st.iters, R * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipMemcpyAsync(rr.data(), A.st.rr, 2 * R * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipMemcpyAsync(bn.data(), A.st.bnorm2, R * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  std::vector<int32_t> actv(2 * (size_t)R);
  SDGP_HIP(hipMemcpyAsync(actv.data(), A.st.act, 2 * R * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  int mx = 0;
  double relmax = 0.0;
  bool conv = true;
  const int executed = flags[0] > 0 ? flags[0] : it;
  const int lastpar = executed & 1;  // parity holding the latest rr / act
  for (int r = 0; r < R; ++r) {
    mx = std::max(mx, its[r]);
    const double rel = bn[r] > 0.0 ? std::sqrt(rr[lastpar * R + r] / bn[r]) : 0.0;
    relmax = std::max(relmax, rel);
    if (actv[lastpar * R + r]) conv = false;
  }
  res.iters = executed;
  res.iters_y = its[0];
  res.relres_max = relmax;
  res.converged = conv && !res.not_spd;
  (void)mx;
  (void)t;
  return res;
}

void slq_from_cg(Ctx* c, const CgResult& cg, int kind, int P, int64_t n, int lanczos_steps, double* logdet,
                 double* stderr_out, double* ritz_min, double* ritz_max) {
  const int ncols = cg.R - 1;
  if (ncols <= 0) {
    *logdet = 0.0; *stderr_out = 0.0; *ritz_min = 0.0; *ritz_max = 0.0;
    return;
  }
  std::vector<int32_t> its(cg.R);
  SDGP_HIP(hipMemcpyAsync(its.data(), cg.col_iters, cg.R * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  int mmax = 1;
  for (int r = 1; r < cg.R; ++r) mmax = std::max(mmax, its[r]);
  if (lanczos_steps > 0) mmax = std::min(mmax, lanczos_steps);
  const size_t W = (size_t)ncols * mmax;
  double* work = c->get<double>(S_SLQ_WORK, 3 * W);
  double* out = c->get<double>(S_SLQ_OUT, (size_t)ncols * 4);
  k_slq<<<(ncols + 63) / 64, 64, 0, c->stream>>>(cg.hist_a, cg.hist_b, cg.col_iters, cg.R, 1, ncols,
                                                 lanczos_steps, ncols, work, work + W, work + 2 * W, out);
  SDGP_CHECK_LAUNCH();
  std::vector<double> ho((size_t)ncols * 4);
  SDGP_HIP(hipMemcpyAsync(ho.data(), out, ho.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  const double zz = (kind == PK_IDENTITY) ? 1.0 : (double)n;
  double sum = 0.0, sum2 = 0.0, lo = INFINITY, hi = -INFINITY;
  bool bad = false;
  for (int p = 0; p < ncols; ++p) {
    const double v = zz * ho[p * 4 + 0];
    if (!std::isfinite(v)) bad = true;
    sum += v;
    sum2 += v * v;
    lo = std::min(lo, ho[p * 4 + 2]);
    hi = std::max(hi, ho[p * 4 + 3]);
  }
  if (bad) throw Error(SDGP_ERR_NOT_SPD, "Lanczos quadrature met a non-positive Ritz value");
  if (kind == PK_IDENTITY) {
    *logdet = sum;
    *stderr_out = 0.0;
  } else {
    const double mean = sum / ncols;
    *logdet = mean;
    const double var = ncols > 1 ? std::max(0.0, (sum2 - ncols * mean * mean) / (ncols - 1)) : 0.0;
    *stderr_out = ncols > 1 ? std::sqrt(var / ncols) : NAN;
  }
  *ritz_min = lo;
  *ritz_max = hi;
}

}  // namespace sdgp
