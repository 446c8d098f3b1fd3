// Adjoint gradient of the log marginal likelihood for gfx950.
//
//   d lnL / d theta = sum_ab Omega_ab (dA/dtheta)_ab,
//   Omega_ab = 1/2 alpha_a alpha_b - 1/2 s sum_p 1/2 (w_pa z_pb + w_pb z_pa),
//
// with alpha = A^{-1} y, w_p = A^{-1} z_p from the block CG (s = 1/P for
// Rademacher probes, 1 for the identity set, for which the sum is the exact
// inverse).  dA/dtheta is recomputed for every stored pair and never stored:
// the core terms accumulate directly, and the bump terms go through the
// per-point adjoint G[a, i] = sum_b Omega_ab c_ab F_i(x_b) (c_ab = sigma2 psi
// for PRODUCT, 1 for SUM), so that for a parameter theta of bump (i, j)
//   d lnL / d theta = 2 sum_a d f_ij(x_a)/d theta * G[a, i].
// All sums are fixed-order (wave butterflies, block trees, ordered partial
// lists): results are bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <vector>

#include "kernel_math.hpp"
#include "sdgp_internal.hpp"

namespace sdgp {

namespace {

constexpr int kAdjBlock = 256;
constexpr int kGroup = 8;  // bump functions per G pass

struct AdjArgs {
  const double4* xs;
  const uint64_t* M;
  const double* F;
  const int32_t* perm;
  const int32_t* sched;
  const int64_t* row_ptr;
  const int32_t* col;
  const double* X;      // [n][R]
  const double* V;      // [n][R] M^{-1} b (preconditioned probes) or null
  const uint64_t* zbits;
  int64_t n;
  int R, P, kind;
  int dim, n1, core, ell, combine;
  double sigma2, r_core, rc2, s_scale;
  double* rowacc;       // [n][3]: sigma2, r_core, noise terms
  double* G;            // [n][n1]
  int lowrank;          // core-only pattern; bump adjoint computed separately
};

__global__ __launch_bounds__(kAdjBlock) void k_adjoint_rows(AdjArgs A) {
  const int64_t pos = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  if (pos >= A.n) return;
  const int64_t a = A.sched ? (int64_t)A.sched[pos] : pos;
  const int lane = lane_id();
  const int64_t R = A.R;
  const double4 xa = A.xs[a];
  const uint64_t Ma = A.M[a];
  const double alpha_a = A.X[a * R];
  const double* Fa = A.F + a * (int64_t)A.n1;
  const bool rad = A.kind == PK_RADEMACHER;
  const bool pre = A.V != nullptr;
  uint64_t za = 0;
  double wa = 0.0, va = 0.0;  // lane p holds w_p(a), v_p(a); broadcast by readlane
  if (rad) {
    if (lane < A.P) wa = A.X[a * R + 1 + lane];
    if (pre) {
      if (lane < A.P) va = A.V[a * R + 1 + lane];
    } else {
      za = A.zbits[a];
    }
  }
  const int64_t k0 = A.row_ptr[a], k1 = A.row_ptr[a + 1];
  const int pa = A.perm[a];
  const int nbits = A.lowrank ? 0 : __popcll(Ma);
  double g_s2 = 0.0, g_rc = 0.0, g_nz = 0.0;
  for (int g0 = 0; g0 < (nbits > 0 ? nbits : 1); g0 += kGroup) {
    // bump functions of this pass: the (g0..g0+7)-th set bits of Ma
    int bi[kGroup];
    {
      uint64_t m = Ma;
      for (int q = 0; q < g0 && m; ++q) m &= m - 1;
#pragma unroll
      for (int q = 0; q < kGroup; ++q) {
        bi[q] = m ? __builtin_ctzll(m) : -1;
        if (m) m &= m - 1;
      }
    }
    double gacc[kGroup];
#pragma unroll
    for (int q = 0; q < kGroup; ++q) gacc[q] = 0.0;
    const bool first = g0 == 0;
    for (int64_t kb = k0; kb < k1; kb += kWave) {
      const int64_t k = kb + lane;
      const bool valid = k < k1;
      const int32_t b = valid ? A.col[k] : (int32_t)a;
      const double4 xb = A.xs[b];
      const double d2 = dist2(xa, xb, A.dim);
      const bool core = d2 < A.rc2;
      const uint64_t Mb = A.M[b];
      const uint64_t mm = Ma & Mb;
      const double* Fb = A.F + (int64_t)b * A.n1;
      double psi = 0.0, dpsi_drc = 0.0;
      if (core) {
        const double dd = sqrt(d2);
        const double u = dd / A.r_core;
        psi = core_psi(u, A.core, A.ell);
        dpsi_drc = -(u / A.r_core) * core_dpsi(u, A.core, A.ell);
      }
      double B = 0.0;  // shared-bump product, a factor of the PRODUCT combine only
      if (A.combine == 0) {
        uint64_t t = mm;
        while (t) {
          const int i = __builtin_ctzll(t);
          t &= t - 1;
          B += Fa[i] * Fb[i];
        }
      }
      // trace part of Omega
      double tr;
      if (rad && pre) {
        // pairs (w_p, v_p) = (A^{-1} b_p, M^{-1} b_p)
        const double* Wb = A.X + (int64_t)b * R + 1;
        const double* Vb = A.V + (int64_t)b * R + 1;
        double t1 = 0.0, t2 = 0.0;
        // probes in steps of 8 with a fixed inner count, so that a step's 16
        // loads are issued together (the compiler will not unroll a loop with
        // a run-time count around the readlanes); the sums keep their order
        int p = 0;
        for (; p + 8 <= A.P; p += 8) {
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            t1 += readlane_f64(wa, p + q) * Vb[p + q];
            t2 += Wb[p + q] * readlane_f64(va, p + q);
          }
        }
        for (; p < A.P; ++p) {
          t1 += readlane_f64(wa, p) * Vb[p];
          t2 += Wb[p] * readlane_f64(va, p);
        }
        tr = 0.5 * (t1 + t2);
      } else if (rad) {
        const uint64_t zb = A.zbits[b];
        const double* Wb = A.X + (int64_t)b * R + 1;
        double t1 = 0.0, t2 = 0.0;
        int p = 0;
        for (; p + 8 <= A.P; p += 8) {
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const double wap = readlane_f64(wa, p + q);
            t1 += ((zb >> (p + q)) & 1ull) ? -wap : wap;
            const double wbp = Wb[p + q];
            t2 += ((za >> (p + q)) & 1ull) ? -wbp : wbp;
          }
        }
        for (; p < A.P; ++p) {
          const double wap = readlane_f64(wa, p);
          t1 += ((zb >> p) & 1ull) ? -wap : wap;
          const double wbp = Wb[p];
          t2 += ((za >> p) & 1ull) ? -wbp : wbp;
        }
        tr = 0.5 * (t1 + t2);
      } else {
        tr = 0.5 * (A.X[a * R + 1 + A.perm[b]] + A.X[(int64_t)b * R + 1 + pa]);
      }
      const double om = valid ? 0.5 * alpha_a * A.X[(int64_t)b * R] - 0.5 * A.s_scale * tr : 0.0;
      if (first) {
        if (A.combine == 0) {
          g_s2 += om * psi * B;
          g_rc += om * A.sigma2 * dpsi_drc * B;
        } else {
          g_s2 += om * psi;
          g_rc += om * A.sigma2 * dpsi_drc;
        }
        if (valid && b == a) g_nz += om;
      }
      if (mm && !A.lowrank) {
        const double cab = A.combine == 0 ? A.sigma2 * psi : 1.0;
        const double oc = om * cab;
#pragma unroll
        for (int q = 0; q < kGroup; ++q)
          if (bi[q] >= 0 && ((mm >> bi[q]) & 1ull)) gacc[q] += oc * Fb[bi[q]];
      }
    }
#pragma unroll
    for (int q = 0; q < kGroup; ++q) {
      const double s = wave_sum(gacc[q]);
      if (lane == 0 && bi[q] >= 0) A.G[a * (int64_t)A.n1 + bi[q]] = s;
    }
  }
  g_s2 = wave_sum(g_s2);
  g_rc = wave_sum(g_rc);
  g_nz = wave_sum(g_nz);
  if (lane == 0) {
    A.rowacc[a * 3 + 0] = g_s2;
    A.rowacc[a * 3 + 1] = g_rc;
    A.rowacc[a * 3 + 2] = g_nz;
  }
}

// Fixed-order block tree sum of 256 values; result valid in thread 0.
__device__ double block_sum256(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Partial sums of the three per-row accumulators over row slices.
__global__ __launch_bounds__(256) void k_rowacc_part(const double* __restrict__ rowacc, int64_t n,
                                                     double* __restrict__ part) {
  __shared__ double sh[256];
  double s[3] = {0.0, 0.0, 0.0};
  for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < n; a += (int64_t)gridDim.x * blockDim.x)
    for (int t = 0; t < 3; ++t) s[t] += rowacc[a * 3 + t];
  for (int t = 0; t < 3; ++t) {
    const double r = block_sum256(s[t], sh);
    if (threadIdx.x == 0) part[blockIdx.x * 3 + t] = r;
  }
}

// Bump-parameter gradient: block (c, sl) handles bump centre c = i*n2 + j
// over the points of slice sl; partial[c][sl][t] for t < 3 + dim.
__global__ __launch_bounds__(256) void k_bump_grad(const double4* __restrict__ xs, const uint64_t* __restrict__ M,
                                                   const double* __restrict__ G, const double* __restrict__ bp,
                                                   int64_t n, int dim, int n1, int n2, int nslices,
                                                   double* __restrict__ part) {
  __shared__ double sh[256];
  const int cidx = blockIdx.x;
  const int i = cidx / n2;
  const int sl = blockIdx.y;
  const int stride = 3 + dim;
  const double* q = bp + cidx * stride;
  const double a = q[0], beta = q[1], r = q[2];
  const double r2 = r * r;
  double acc[3 + kMaxDim];
#pragma unroll
  for (int t = 0; t < 3 + kMaxDim; ++t) acc[t] = 0.0;
  const int64_t per = (n + nslices - 1) / nslices;
  const int64_t s0 = sl * per;
  const int64_t s1 = min(n, s0 + per);
  for (int64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
    if (!((M[s] >> i) & 1ull)) continue;
    const double4 p = xs[s];
    double d2 = 0.0;
    for (int k = 0; k < dim; ++k) {
      const double d = comp(p, k) - q[3 + k];
      d2 += d * d;
    }
    if (!(d2 < r2)) continue;
    const double qq = d2 / r2;
    const double omq = 1.0 - qq;
    const double e = exp(beta - beta / omq);
    const double f = a * e;
    const double g2 = 2.0 * G[s * (int64_t)n1 + i];
    const double gb = f * beta / (omq * omq);
    acc[0] += g2 * e;
    acc[1] += g2 * (-f * qq / omq);
    acc[2] += g2 * gb * 2.0 * qq / r;
    for (int k = 0; k < dim; ++k) acc[3 + k] += g2 * gb * 2.0 * (comp(p, k) - q[3 + k]) / r2;
  }
  for (int t = 0; t < stride; ++t) {
    const double v = block_sum256(acc[t], sh);
    if (threadIdx.x == 0) part[((int64_t)cidx * nslices + sl) * stride + t] = v;
  }
}

// Per-block partials of F^T Y (Y: [n][R] row-major), lane = column:
// part[b][i][r]; grid (nb, chunks), 256 threads.  The wavefront's row index is
// made uniform (readfirstlane), so each row of F comes in by scalar loads,
// and when n1 fills the template width four rows are loaded before their
// products are added (each accumulator still adds the rows in order); the
// guarded per-element form serialised one load and wait per F element.
template <int NI>
__global__ __launch_bounds__(256) void k_ft_part(const double* __restrict__ F, const double* __restrict__ Y,
                                                 int64_t n, int n1, int R, double* __restrict__ part) {
  __shared__ double sh[4][kWave];
  const int lane = lane_id(), w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rc = blockIdx.y * kWave + lane;
  double acc[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) acc[i] = 0.0;
  const int64_t st = (int64_t)gridDim.x * 4;
  int64_t a = blockIdx.x * 4 + w;
  if (rc < R && n1 == NI) {
    for (; a + 3 * st < n; a += 4 * st) {
      double y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) y[u] = Y[(a + u * st) * R + rc];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double* Fa = F + (a + u * st) * NI;
#pragma unroll
        for (int i = 0; i < NI; ++i) acc[i] += Fa[i] * y[u];
      }
    }
  }
  if (rc < R)
    for (; a < n; a += st) {
      const double y = Y[a * R + rc];
      const double* Fa = F + a * n1;
#pragma unroll
      for (int i = 0; i < NI; ++i)
        if (i < n1) acc[i] += Fa[i] * y;
    }
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    if (i >= n1) break;
    __syncthreads();
    sh[w][lane] = acc[i];
    __syncthreads();
    if (threadIdx.x < kWave && rc < R)
      part[((int64_t)blockIdx.x * n1 + i) * R + rc] = sh[0][lane] + sh[1][lane] + sh[2][lane] + sh[3][lane];
  }
}

// out[i][r] = sum_b part[b][i][r] in fixed order; grid (n1, chunks).
__global__ void k_ft_reduce(const double* __restrict__ part, int nb, int n1, int R, double* __restrict__ out) {
  const int i = blockIdx.x;
  const int rc = blockIdx.y * kWave + lane_id();
  if (threadIdx.x >= kWave || rc >= R) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[((int64_t)b * n1 + i) * R + rc];
  out[(int64_t)i * R + rc] = s;
}

// Bump part of the per-point adjoint for K = K_core + F F^T:
//   G[a,i] = sum_b Omega_ab F_bi
//          = 1/2 alpha_a (F^T X)[i][0]
//            - 1/4 s sum_p (w_pa (F^T V)[i][1+p] + v_pa (F^T X)[i][1+p]),
// with X = [alpha, w_1..w_P] and V = [., v_1..v_P]; only where x_a lies in
// a support of bump function i (elsewhere dF_ai/dtheta = 0).
__global__ void k_lowrank_G(const double* __restrict__ X, const double* __restrict__ V,
                            const uint64_t* __restrict__ M, const double* __restrict__ FX,
                            const double* __restrict__ FV, int64_t n, int n1, int R, int P, double s_scale,
                            double* __restrict__ G) {
  const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= n) return;
  uint64_t m = M[a];
  const double* Xa = X + a * R;
  const double* Va = V + a * R;
  while (m) {
    const int i = __builtin_ctzll(m);
    m &= m - 1;
    double t = 0.0;
    for (int p = 0; p < P; ++p) t += Xa[1 + p] * FV[(int64_t)i * R + 1 + p] + Va[1 + p] * FX[(int64_t)i * R + 1 + p];
    G[a * n1 + i] = 0.5 * Xa[0] * FX[(int64_t)i * R] - 0.25 * s_scale * t;
  }
}

template <int NI>
void launch_ft(Ctx* c, const double* F, const double* Y, int64_t n, int n1, int R, double* part, int nb,
               double* out) {
  const int chunks = (R + kWave - 1) / kWave;
  k_ft_part<NI><<<dim3(nb, chunks), 256, 0, c->stream>>>(F, Y, n, n1, R, part);
  SDGP_CHECK_LAUNCH();
  k_ft_reduce<<<dim3(n1, chunks), kWave, 0, c->stream>>>(part, nb, n1, R, out);
  SDGP_CHECK_LAUNCH();
}

void lowrank_bump_adjoint(Ctx* c, const Sorted& s, const KParams& kp, const Bumps& b, const CgResult& cg, int P,
                          double s_scale, double* G) {
  const int n1 = kp.n1;
  const int64_t n = s.n;
  const int R = cg.R;
  require(cg.V != nullptr, "the factored operator needs the preconditioned probe solves");
  const int nb = (int)std::min<int64_t>(256, (n + 1023) / 1024);
  double* part = c->get<double>(S_LR_PART, (size_t)nb * n1 * R);
  double* FX = c->get<double>(S_LR_FX, (size_t)n1 * R);
  double* FV = c->get<double>(S_LR_FV, (size_t)n1 * R);
  auto ft = [&](const double* Y, double* out) {
    if (n1 <= 8) launch_ft<8>(c, b.F, Y, n, n1, R, part, nb, out);
    else if (n1 <= 16) launch_ft<16>(c, b.F, Y, n, n1, R, part, nb, out);
    else if (n1 <= 32) launch_ft<32>(c, b.F, Y, n, n1, R, part, nb, out);
    else launch_ft<64>(c, b.F, Y, n, n1, R, part, nb, out);
  };
  ft(cg.X, FX);
  ft(cg.V, FV);
  k_lowrank_G<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(cg.X, cg.V, b.M, FX, FV, n, n1, R, P, s_scale, G);
  SDGP_CHECK_LAUNCH();
}

}  // namespace

void adjoint_gradient(Ctx* c, const Sorted& s, const KParams& kp, const Bumps& b, const Csr& Am,
                      const CgResult& cg, int kind, int P, uint64_t seed, const double* h, double* grad,
                      bool lowrank) {
  const int64_t n = s.n;
  AdjArgs A;
  A.xs = s.xs; A.M = b.M; A.F = b.F; A.perm = s.perm; A.sched = s.sched;
  A.row_ptr = Am.row_ptr; A.col = Am.col; A.X = cg.X; A.V = cg.V;
  A.n = n; A.R = cg.R; A.P = P; A.kind = kind;
  A.dim = kp.dim; A.n1 = kp.n1; A.core = kp.core; A.ell = kp.dim / 2 + 2; A.combine = kp.combine;
  A.sigma2 = kp.sigma2; A.r_core = kp.r_core; A.rc2 = kp.rc2;
  A.s_scale = kind == PK_IDENTITY ? 1.0 : 1.0 / P;
  A.zbits = nullptr;
  if (kind == PK_RADEMACHER && A.V == nullptr) {
    require(P >= 1 && P <= 64, "Rademacher probes must be 1..64");
    uint64_t* zb = c->get<uint64_t>(S_ZBITS, n);
    probe_bits(c, s, P, seed, zb);
    A.zbits = zb;
  }
  A.rowacc = c->get<double>(S_ADJ_ROW, (size_t)n * 3);
  const int n1 = kp.n1;
  A.G = c->get<double>(S_ADJ_G, (size_t)n * (n1 > 0 ? n1 : 1));
  if (n1 > 0) SDGP_HIP(hipMemsetAsync(A.G, 0, (size_t)n * n1 * sizeof(double), c->stream));
  A.lowrank = lowrank ? 1 : 0;
  const int64_t blocks = (n + 3) / 4;
  k_adjoint_rows<<<(unsigned)blocks, kAdjBlock, 0, c->stream>>>(A);
  SDGP_CHECK_LAUNCH();
  if (lowrank && n1 > 0) lowrank_bump_adjoint(c, s, kp, b, cg, P, A.s_scale, A.G);
  // core / noise terms
  const int nbp = (int)std::min<int64_t>(256, (n + 255) / 256);
  double* part = c->get<double>(S_ADJ_PART, (size_t)nbp * 3);
  k_rowacc_part<<<nbp, 256, 0, c->stream>>>(A.rowacc, n, part);
  SDGP_CHECK_LAUNCH();
  std::vector<double> hp((size_t)nbp * 3);
  SDGP_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  // bump terms
  const int nc = kp.n1 * kp.n2;
  const int stride = 3 + kp.dim;
  const int nsl = (int)std::max<int64_t>(1, std::min<int64_t>(64, (n + 4095) / 4096));
  std::vector<double> hb((size_t)nc * nsl * stride);
  if (nc > 0) {
    double* bpart = c->get<double>(S_RED_OUT, hb.size());
    k_bump_grad<<<dim3(nc, nsl), 256, 0, c->stream>>>(s.xs, b.M, A.G, b.bp, n, kp.dim, kp.n1, kp.n2, nsl, bpart);
    SDGP_CHECK_LAUNCH();
    SDGP_HIP(hipMemcpyAsync(hb.data(), bpart, hb.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  }
  SDGP_HIP(hipStreamSynchronize(c->stream));
  double g[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < nbp; ++i)
    for (int t = 0; t < 3; ++t) g[t] += hp[i * 3 + t];
  const int64_t nh = 2 + (int64_t)nc * stride + 1;
  grad[0] = g[0];
  grad[1] = g[1];
  grad[nh - 1] = g[2];
  for (int ci = 0; ci < nc; ++ci)
    for (int t = 0; t < stride; ++t) {
      double v = 0.0;
      for (int sl = 0; sl < nsl; ++sl) v += hb[((size_t)ci * nsl + sl) * stride + t];
      grad[2 + (int64_t)ci * stride + t] = v;
    }
  (void)h;
}

}  // namespace sdgp
