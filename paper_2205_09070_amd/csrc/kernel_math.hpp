// Device-side kernel functions of the sparsity-discovering kernel
// (Section 2.2) and wavefront helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sdgp {

// sqrt(2) / (3 sqrt(pi)): prefactor of the compact core of eq:kstat.
constexpr double kKstatC = 0.26596152026762178529;

// Compact core of eq:kstat as a function of u = d / r (u < 1).  The printed
// form c (3u^2 ln(u/(1+S)) + (2u^2+1) S), S = sqrt(1-u^2), cancels as
// u -> 1; there ln(u/(1+S)) = -atanh(S) and atanh's power series give
//   psi / c = sum_{n>=2} 6 S^(2n+1) / (4n^2 - 1),
// summed forward until the terms stop contributing (S <= 0.85 needs at most
// ~130 terms).  psi(0) = c (limit of the printed form).
__device__ __forceinline__ double kstat_psi(double u) {
  const double s = sqrt((1.0 - u) * (1.0 + u));
  if (s <= 0.85) {
    const double s2 = s * s;
    double pw = s2 * s2 * s;  // S^5
    double acc = 0.0;
    for (int n = 2; n < 200; ++n) {
      const double t = pw * (6.0 / (4.0 * n * n - 1.0));
      acc += t;
      if (t <= 1e-18 * acc) break;
      pw *= s2;
    }
    return kKstatC * acc;
  }
  if (u == 0.0) return kKstatC;
  const double u2 = u * u;
  return kKstatC * (3.0 * u2 * log(u / (1.0 + s)) + (2.0 * u2 + 1.0) * s);
}

// d psi / d u = 6 c u (S - atanh S); near S -> 0 the difference is the series
// -sum_{k>=1} S^(2k+1) / (2k+1).
__device__ __forceinline__ double kstat_dpsi(double u) {
  const double s = sqrt((1.0 - u) * (1.0 + u));
  if (s <= 0.85) {
    const double s2 = s * s;
    double pw = s2 * s;  // S^3
    double acc = 0.0;
    for (int k = 1; k < 300; ++k) {
      const double t = pw / (2.0 * k + 1.0);
      acc += t;
      if (t <= 1e-18 * acc) break;
      pw *= s2;
    }
    return -6.0 * kKstatC * u * acc;
  }
  if (u == 0.0) return 0.0;
  return 6.0 * kKstatC * u * (s - log((1.0 + s) / u));
}

// Wendland smoothness-1 function (1-u)^(l+1) ((l+1) u + 1), l = floor(d/2)+2.
__device__ __forceinline__ double wendland_psi(double u, int ell) {
  const double v = 1.0 - u;
  double p = v;
  for (int k = 0; k < ell; ++k) p *= v;  // v^(l+1)
  return p * ((ell + 1) * u + 1.0);
}

__device__ __forceinline__ double wendland_dpsi(double u, int ell) {
  const double v = 1.0 - u;
  double p = 1.0;
  for (int k = 0; k < ell; ++k) p *= v;  // v^l
  return -(double)((ell + 1) * (ell + 2)) * u * p;
}

// core: 0 = Wendland C2, 1 = eq:kstat.  Caller guarantees u < 1.
__device__ __forceinline__ double core_psi(double u, int core, int ell) {
  return core == 1 ? kstat_psi(u) : wendland_psi(u, ell);
}
__device__ __forceinline__ double core_dpsi(double u, int core, int ell) {
  return core == 1 ? kstat_dpsi(u) : wendland_dpsi(u, ell);
}

__device__ __forceinline__ double dist2(const double4& a, const double4& b, int dim) {
  double dx = a.x - b.x;
  double s = dx * dx;
  if (dim > 1) { double d = a.y - b.y; s += d * d; }
  if (dim > 2) { double d = a.z - b.z; s += d * d; }
  if (dim > 3) { double d = a.w - b.w; s += d * d; }
  return s;
}

__device__ __forceinline__ double comp(const double4& a, int k) {
  return k == 0 ? a.x : (k == 1 ? a.y : (k == 2 ? a.z : a.w));
}

// ---- wavefront (64 lanes) helpers ----
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// Number of set bits of `mask` below the calling lane.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Broadcast lane l's value (l uniform across the wave).
__device__ __forceinline__ int readlane_i32(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return (uint64_t)hi << 32 | lo;
}

// Butterfly sum over the 64 lanes (fixed order: deterministic).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// SplitMix64 (Steele, Lea, Flood 2014): output k >= 1 of the stream seeded
// with `seed` is mix(seed + k * golden).
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
  uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace sdgp
