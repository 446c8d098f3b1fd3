// Differential evolution over hyperparameter populations (DE/rand/1/bin,
// Storn and Price, J. Global Optim. 11, 1997): trial generation and
// selection, host code.  Random numbers come from the SplitMix64 counter
// generator (Steele, Lea and Flood, OOPSLA 2014), one draw per key.
#include <cmath>
#include <cstdint>
#include <vector>

#include "sdgp_internal.hpp"

namespace sdgp {

namespace {

uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Uniform double in [0, 1) for draw `d` of member m in generation gen.
struct DeRng {
  uint64_t seed, gen;
  int32_t B, slots;
  double u(int32_t m, int32_t d) const {
    const uint64_t k = ((gen * (uint64_t)B + (uint64_t)m) * (uint64_t)slots + (uint64_t)d) + 1ull;
    return (double)(mix64(seed + k * 0x9E3779B97F4A7C15ull) >> 11) * 0x1.0p-53;
  }
};

}  // namespace

void de_trials(int32_t B, int32_t nh, const double* H, const double* lo, const double* hi, double F, double CR,
               uint64_t seed, uint64_t generation, double* T) {
  require(H && lo && hi && T, "NULL argument");
  require(B >= 4, "differential evolution needs at least 4 members");
  require(nh >= 1, "nh must be >= 1");
  require(F > 0.0 && F <= 2.0, "F must be in (0, 2]");
  require(CR >= 0.0 && CR <= 1.0, "CR must be in [0, 1]");
  for (int32_t j = 0; j < nh; ++j) require(std::isfinite(lo[j]) && std::isfinite(hi[j]) && lo[j] <= hi[j], "bad bounds");
  for (int64_t e = 0; e < (int64_t)B * nh; ++e) {
    const int32_t j = (int32_t)(e % nh);
    require(std::isfinite(H[e]) && H[e] >= lo[j] && H[e] <= hi[j], "population outside its bounds");
  }
  // draws per member: nh crossover draws, nh bound redraws, jrand, then the
  // parent picks (rejection: at most 64 attempts each)
  const int32_t slots = 2 * nh + 1 + 3 * 64;
  const DeRng rng{seed, generation, B, slots};
  for (int32_t m = 0; m < B; ++m) {
    int32_t r[3];
    int32_t d = 2 * nh + 1;
    for (int q = 0; q < 3; ++q) {
      for (int attempt = 0;; ++attempt) {
        int32_t c = (int32_t)(rng.u(m, d++) * B);
        if (c >= B) c = B - 1;
        bool ok = c != m;
        for (int p = 0; p < q; ++p) ok = ok && c != r[p];
        if (ok) { r[q] = c; break; }
        if (attempt == 63) {  // deterministic fallback: next free index
          c = (m + 1) % B;
          for (;;) {
            bool f = c != m;
            for (int p = 0; p < q; ++p) f = f && c != r[p];
            if (f) break;
            c = (c + 1) % B;
          }
          r[q] = c;
          d = 2 * nh + 1 + 64 * (q + 1);
          break;
        }
      }
    }
    int32_t jr = (int32_t)(rng.u(m, 2 * nh) * nh);
    if (jr >= nh) jr = nh - 1;
    const double* xm = H + (int64_t)m * nh;
    double* t = T + (int64_t)m * nh;
    for (int32_t j = 0; j < nh; ++j) {
      if (lo[j] == hi[j]) {
        t[j] = lo[j];
        continue;
      }
      double v = xm[j];
      if (rng.u(m, j) < CR || j == jr) {
        v = H[(int64_t)r[0] * nh + j] + F * (H[(int64_t)r[1] * nh + j] - H[(int64_t)r[2] * nh + j]);
        const double w = rng.u(m, nh + j);
        if (v < lo[j]) v = lo[j] + w * (xm[j] - lo[j]);
        if (v > hi[j]) v = hi[j] - w * (hi[j] - xm[j]);
      }
      t[j] = v;
    }
  }
}

int32_t de_select(int32_t B, int32_t nh, double* H, double* fit, const double* T, const double* ft) {
  require(H && fit && T && ft, "NULL argument");
  require(B >= 1 && nh >= 1, "B and nh must be >= 1");
  int32_t rep = 0;
  for (int32_t m = 0; m < B; ++m) {
    const double a = fit[m], b = ft[m];
    const bool take = !std::isnan(b) && (std::isnan(a) || b >= a);
    if (!take) continue;
    for (int32_t j = 0; j < nh; ++j) H[(int64_t)m * nh + j] = T[(int64_t)m * nh + j];
    fit[m] = b;
    ++rep;
  }
  return rep;
}

}  // namespace sdgp
