// Host helpers shared by the single-instance runtime (meg_api.hip) and the
// batched server (meg_serve.hip).
#pragma once
#include <cmath>
#include <cstdint>
#include <vector>

namespace meg {

// ---- small host PRNG (SplitMix64 + Box-Muller) for the extra start columns
struct SplitMix {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() {
    const double u1 = uniform(), u2 = uniform();
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

// Host basis: columns 0..q-1 = V (n x q col-major), q..k-1 = seeded Gaussian
// columns orthonormalised against all previous ones (two passes of modified
// Gram-Schmidt in FP64).  Output row-major n x k.
inline bool build_basis(int64_t n, int k, int q, const double* V, uint64_t seed, std::vector<double>& out) {
  std::vector<double> B((size_t)n * k);
  for (int j = 0; j < q; ++j)
    for (int64_t i = 0; i < n; ++i) B[(size_t)j * n + i] = V[(size_t)j * n + i];
  SplitMix rng{seed * 0x2545f4914f6cdd1dull + 12345};
  for (int j = q; j < k; ++j) {
    double* b = &B[(size_t)j * n];
    for (int attempt = 0; attempt < 4; ++attempt) {
      for (int64_t i = 0; i < n; ++i) b[i] = rng.normal();
      for (int pass = 0; pass < 2; ++pass)
        for (int l = 0; l < j; ++l) {
          const double* a = &B[(size_t)l * n];
          double s = 0;
          for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
          for (int64_t i = 0; i < n; ++i) b[i] -= s * a[i];
        }
      double nr = 0;
      for (int64_t i = 0; i < n; ++i) nr += b[i] * b[i];
      nr = std::sqrt(nr);
      if (nr > 1e-8) {
        for (int64_t i = 0; i < n; ++i) b[i] /= nr;
        break;
      }
      if (attempt == 3) return false;
    }
  }
  out.assign((size_t)n * k, 0.0);
  for (int j = 0; j < k; ++j)
    for (int64_t i = 0; i < n; ++i) out[(size_t)i * k + j] = B[(size_t)j * n + i];
  return true;
}

}  // namespace meg
