// Block preconditioner of the SUM combine (CG on A = K_core + F F^T + noise I).
//
//   M = B + F F^T,  B = blockdiag(B_t),  B_t = A_csr[T_t, T_t],
//
// where the tiles T_t are 16 consecutive rows of the Morton row schedule
// (spatially compact groups of points) and A_csr is the matrix the CG
// multiplies (the core part with the noise on the diagonal under the
// factored operator, the full K otherwise).  Every B_t is a principal
// submatrix of an SPD matrix, so M is SPD.  With Y = B^{-1} F and
// S = I + F^T Y (n1 x n1):
//   M^{-1} r  = B^{-1} r - Y S^{-1} (Y^T r)           (Woodbury identity)
//   ln det M  = sum_t ln det B_t + ln det S             (determinant lemma)
//   b = L w + F v, B = L L^T blockwise, w, v Rademacher: Cov(b) = M,
// which is what the CG probes, the SLQ weights b^T M^{-1} b and the
// Hutchinson pairs (A^{-1} b, M^{-1} b) of the estimators need (Gardner et
// al. 2018 use the same construction with other preconditioners).
//
// Setup, one wavefront per tile: the dense 16 x 16 block from the CSR (an
// entry (a, c) belongs to the tile when the schedule position of c lies in
// it), Cholesky B_t = L L^T, L^{-1} by forward substitution, B_t^{-1} =
// L^{-T} L^{-1} (each entry one fixed-order sum, so the stored inverse is
// exactly symmetric), ln det B_t = 2 sum ln L_ii and the tile's rows of Y.
// B_t^{-1} and L are stored in the operand order of v_mfma_f64_16x16x4f64:
// element [t][st][lane] = X[lane & 15][4 st + (lane >> 4)], so the CG
// kernels apply them to a 16-row tile with one 512-byte load per K step.
#include <algorithm>
#include <cmath>
#include <vector>

#include "sdgp_internal.hpp"

namespace sdgp {

namespace {

constexpr int kTileRows = 16;
constexpr int kWavesPerBlock = 4;
constexpr int kBS = kTileRows + 1;   // LDS row stride (bank spread)

// pos[sched[p]] = p
__global__ void k_sched_inverse(const int32_t* __restrict__ sched, int64_t n, int32_t* __restrict__ pos) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p < n) pos[sched[p]] = (int32_t)p;
}

__global__ __launch_bounds__(64 * kWavesPerBlock) void k_block_build(
    int64_t n, const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const int32_t* __restrict__ sched, const int32_t* __restrict__ pos,
    const double* __restrict__ F, int n1, int64_t ntile, double* __restrict__ Bt, double* __restrict__ Lt,
    double* __restrict__ Y, double* __restrict__ ld, int32_t* __restrict__ bad) {
  __shared__ double sB[kWavesPerBlock][kTileRows * kBS];
  __shared__ double sL[kWavesPerBlock][kTileRows * kBS];
  __shared__ double sI[kWavesPerBlock][kTileRows * kBS];   // L^{-1}, then B^{-1}
  __shared__ double sF[kWavesPerBlock][kTileRows * kMaxN1];
  __shared__ int64_t sRow[kWavesPerBlock][kTileRows];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * kWavesPerBlock + w;
  const bool live = t < ntile;
  double* B = sB[w];
  double* L = sL[w];
  double* I = sI[w];
  const int64_t p0 = t * kTileRows;
  if (lane < kTileRows) {
    const int64_t p = p0 + lane;
    sRow[w][lane] = (live && p < n) ? (int64_t)sched[p] : -1;
  }
  for (int e = lane; e < kTileRows * kBS; e += 64) {
    B[e] = 0.0;
    L[e] = 0.0;
    I[e] = 0.0;
  }
  __syncthreads();
  // dense block: row i scans its entries, keeping the columns of this tile
  for (int i = 0; i < kTileRows; ++i) {
    const int64_t a = sRow[w][i];
    if (a < 0) {
      if (lane == 0) B[i * kBS + i] = 1.0;   // padding row: identity
      continue;
    }
    const int64_t k0 = row_ptr[a], k1 = row_ptr[a + 1];
    for (int64_t k = k0 + lane; k < k1; k += 64) {
      const int64_t q = pos[col[k]];
      if (q >= p0 && q < p0 + kTileRows) B[i * kBS + (int)(q - p0)] = val[k];
    }
  }
  for (int e = lane; e < kTileRows * kMaxN1; e += 64) {
    const int i = e / kMaxN1, m = e % kMaxN1;
    const int64_t a = sRow[w][i];
    sF[w][e] = (a >= 0 && m < n1) ? F[a * n1 + m] : 0.0;
  }
  __syncthreads();
  // Cholesky B = L L^T (one lane; 16 x 16)
  if (lane == 0 && live) {
    bool ok = true;
    double logdet = 0.0;
    for (int j = 0; j < kTileRows; ++j) {
      double d = B[j * kBS + j];
      for (int k = 0; k < j; ++k) d -= L[j * kBS + k] * L[j * kBS + k];
      if (!(d > 0.0) || !isfinite(d)) {
        ok = false;
        d = 1.0;
      }
      const double ljj = sqrt(d);
      L[j * kBS + j] = ljj;
      logdet += 2.0 * log(ljj);
      for (int i = j + 1; i < kTileRows; ++i) {
        double v = B[i * kBS + j];
        for (int k = 0; k < j; ++k) v -= L[i * kBS + k] * L[j * kBS + k];
        L[i * kBS + j] = v / ljj;
      }
    }
    ld[t] = logdet;
    if (!ok) bad[0] = 1;
  }
  __syncthreads();
  // column c of L^{-1} (lanes c < 16): forward substitution on e_c
  if (lane < kTileRows) {
    const int c = lane;
    for (int i = c; i < kTileRows; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) v -= L[i * kBS + k] * I[k * kBS + c];
      I[i * kBS + c] = v / L[i * kBS + i];
    }
  }
  __syncthreads();
  // B^{-1}[i][j] = sum_{k >= max(i, j)} L^{-1}[k][i] L^{-1}[k][j] (into B)
  for (int e = lane; e < kTileRows * kTileRows; e += 64) {
    const int i = e >> 4, j = e & 15;
    double s = 0.0;
    for (int k = max(i, j); k < kTileRows; ++k) s += I[k * kBS + i] * I[k * kBS + j];
    B[i * kBS + j] = s;
  }
  __syncthreads();
  if (live) {
    double* bt = Bt + t * 256;
    double* lt = Lt + t * 256;
    const int i = lane & 15, kk = lane >> 4;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      bt[st * 64 + lane] = B[i * kBS + 4 * st + kk];
      lt[st * 64 + lane] = L[i * kBS + 4 * st + kk];
    }
    // Y rows of the tile: Y[a_i][m] = sum_k B^{-1}[i][k] F[a_k][m]
    for (int e = lane; e < kTileRows * n1; e += 64) {
      const int r = e / n1, m = e % n1;
      const int64_t a = sRow[w][r];
      if (a < 0) continue;
      double s = 0.0;
      for (int k = 0; k < kTileRows; ++k) s += B[r * kBS + k] * sF[w][k * kMaxN1 + m];
      Y[a * n1 + m] = s;
    }
  }
}

// Per-block partial sums of F^T Y (n1 x n1), rows lo .. hi of the block.
__global__ __launch_bounds__(256) void k_gram_fy(const double* __restrict__ F, const double* __restrict__ Y,
                                                 int64_t n, int n1, int64_t slab, double* __restrict__ part) {
  __shared__ double fr[64 * kMaxN1];
  __shared__ double yr[64 * kMaxN1];
  const int np = n1 * n1;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  const int64_t lo = blockIdx.x * slab, hi = min(n, lo + slab);
  for (int64_t a0 = lo; a0 < hi; a0 += 64) {
    const int cnt = (int)min((int64_t)64, hi - a0);
    __syncthreads();
    for (int idx = threadIdx.x; idx < cnt * n1; idx += blockDim.x) {
      fr[idx] = F[a0 * n1 + idx];
      yr[idx] = Y[a0 * n1 + idx];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int idx = threadIdx.x + q * 256;
      if (idx < np) {
        const int i = idx / n1, j = idx % n1;
        double s = 0.0;
        for (int k = 0; k < cnt; ++k) s += fr[k * n1 + i] * yr[k * n1 + j];
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

Precond block_precond(Ctx* c, const Sorted& s, const Csr& A, const KParams& kp, const Bumps& b) {
  Precond pc;
  const int n1 = kp.n1;
  const int64_t n = s.n;
  require(n1 <= kMaxN1, "too many bump functions");
  require(s.sched != nullptr, "no row schedule");
  const int64_t ntile = (n + kTileRows - 1) / kTileRows;
  int32_t* pos = c->get<int32_t>(S_BP_POS, n);
  double* Bt = c->get<double>(S_BP_BT, (size_t)ntile * 256);
  double* Lt = c->get<double>(S_BP_LT, (size_t)ntile * 256);
  double* Y = c->get<double>(S_BP_Y, (size_t)std::max<int64_t>(1, n * n1));
  double* ld = c->get<double>(S_BP_LD, ntile);
  int32_t* bad = c->get<int32_t>(S_BP_BAD, 1);
  SDGP_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), c->stream));
  k_sched_inverse<<<(unsigned)((n + 255) / 256), 256, 0, c->stream>>>(s.sched, n, pos);
  SDGP_CHECK_LAUNCH();
  const int64_t nblk = (ntile + kWavesPerBlock - 1) / kWavesPerBlock;
  require(nblk < 0x7fffffff, "too many tiles");
  k_block_build<<<(unsigned)nblk, 64 * kWavesPerBlock, 0, c->stream>>>(n, A.row_ptr, A.col, A.val, s.sched, pos,
                                                                        b.F, n1, ntile, Bt, Lt, Y, ld, bad);
  SDGP_CHECK_LAUNCH();
  std::vector<double> hld((size_t)ntile);
  int32_t hbad = 0;
  SDGP_HIP(hipMemcpyAsync(hld.data(), ld, ntile * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  if (hbad) throw Error(SDGP_ERR_NOT_SPD, "a diagonal block of the covariance is not positive definite");
  double logdetB = 0.0;
  for (int64_t t = 0; t < ntile; ++t) logdetB += hld[t];
  pc.block = 1;
  pc.n1 = n1;
  pc.F = b.F;
  pc.Bt = Bt;
  pc.Lt = Lt;
  pc.Y = n1 > 0 ? Y : nullptr;
  pc.logdetM = logdetB;
  if (n1 == 0) return pc;
  // S = I + F^T Y; Cholesky; ln det S; S^{-1}
  const int64_t nbk = std::min<int64_t>(256, (n + 4095) / 4096);
  const int64_t slab = (n + nbk - 1) / nbk;
  const int np = n1 * n1;
  double* part = c->get<double>(S_PC_PART, (size_t)nbk * np);
  k_gram_fy<<<(unsigned)nbk, 256, 0, c->stream>>>(b.F, Y, n, n1, slab, part);
  SDGP_CHECK_LAUNCH();
  std::vector<double> hp((size_t)nbk * np);
  SDGP_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  std::vector<double> S((size_t)np, 0.0), L((size_t)np, 0.0), Si((size_t)np, 0.0);
  for (int64_t bb = 0; bb < nbk; ++bb)
    for (int q = 0; q < np; ++q) S[q] += hp[bb * np + q];
  // F^T B^{-1} F is symmetric; take the mean of the two triangles' sums
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < i; ++j) {
      const double v = 0.5 * (S[i * n1 + j] + S[j * n1 + i]);
      S[i * n1 + j] = S[j * n1 + i] = v;
    }
  for (int i = 0; i < n1; ++i) S[i * n1 + i] += 1.0;
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
  for (int cc = 0; cc < n1; ++cc) {  // S^{-1} e_cc
    std::vector<double> yv(n1, 0.0);
    for (int i = 0; i < n1; ++i) {
      double v = (i == cc) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) v -= L[i * n1 + k] * yv[k];
      yv[i] = v / L[i * n1 + i];
    }
    for (int i = n1 - 1; i >= 0; --i) {
      double v = yv[i];
      for (int k = i + 1; k < n1; ++k) v -= L[k * n1 + i] * Si[k * n1 + cc];
      Si[i * n1 + cc] = v / L[i * n1 + i];
    }
  }
  double* dSi = c->get<double>(S_PC_SINV, np);
  SDGP_HIP(hipMemcpyAsync(dSi, Si.data(), np * sizeof(double), hipMemcpyHostToDevice, c->stream));
  SDGP_HIP(hipStreamSynchronize(c->stream));
  pc.Sinv = dSi;
  pc.logdetM = logdetB + logdetS;
  return pc;
}

}  // namespace sdgp
