// Host check of the perceptron's GELU tail polynomial
// (paper_2102_05297_amd/csrc/gelu.h) against a long double reference:
//   1. |p(x) - log2 Phi(-x)| over every 16th float32 x in [0, X] (and every
//      float below 2^-10), X = kGeluTailMax, p evaluated in float32 as the
//      kernels do;
//   2. the whole GELU, max(z, 0) - |z| 2^p(min(|z|, X)), with the host's
//      float32 exp2 (within one ulp, as the device's exponential), against
//      z Phi(z) for every 64th float32 z in [-30, 30]: the error must stay
//      within rho |z| Phi(-|z|) + 2^-24 |GELU(z)| (|z| <= X) and
//      2 (1 + rho) |z| Phi(-X) + 2^-24 |GELU(z)| (|z| > X), where
//      rho = 2^delta - 1 + 2^-22 and delta is the bound of part 1.
// Prints the largest errors; exits non-zero when a bound fails.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#define __host__
#define __device__
#define __forceinline__ inline
#include "gelu.h"

static float from_bits(uint32_t u) { float f; std::memcpy(&f, &u, 4); return f; }
static uint32_t bits(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }

static long double phi_neg(long double x) { // Phi(-x)
  return 0.5L * erfcl(x / sqrtl(2.0L));
}

int main() {
  const double delta = 1.15e-4; // the bound asserted in part 1
  const unsigned nt = std::max(1u, std::thread::hardware_concurrency());
  // part 1: polynomial error
  const uint32_t top = bits(cgs::kGeluTailMax);
  std::vector<double> worst1(nt, 0.0);
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      double w = 0.0;
      for (uint32_t b = t; b <= top; b += nt) {
        if (b % 16 != 0 && b > bits(0x1p-10f)) continue;
        const float x = from_bits(b);
        const long double ref = log2l(phi_neg(x));
        const double e = std::fabs((double)((long double)cgs::gelu_tail_log2(x) - ref));
        if (e > w) w = e;
      }
      worst1[t] = w;
    });
  for (auto &x : th) x.join();
  th.clear();
  double e1 = 0.0;
  for (double w : worst1) e1 = std::max(e1, w);
  // part 2: the whole GELU against its bound
  const double rho = std::exp2(delta) - 1.0 + 0x1p-22;
  const long double phi_cut = phi_neg((long double)cgs::kGeluTailMax);
  std::vector<double> worst2(nt, 0.0);
  std::vector<long> bad(nt, 0);
  const uint32_t zmax = bits(30.0f);
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      double w = 0.0;
      for (uint32_t b = 64 * t; b <= zmax; b += 64 * nt) {
        for (int sg = 0; sg < 2; ++sg) {
          const float z = sg ? -from_bits(b) : from_bits(b);
          const float az = std::fabs(z);
          const float e = exp2f(cgs::gelu_tail_log2(std::fmin(az, cgs::kGeluTailMax)));
          const float g = std::fma(-az, e, std::fmax(z, 0.0f));
          const long double tail = (long double)az * phi_neg(az);
          const long double exact = (z > 0 ? (long double)z : 0.0L) - tail;
          const long double err = fabsl((long double)g - exact);
          const long double bound =
              (az <= cgs::kGeluTailMax ? rho * tail : 2.0L * (1.0L + rho) * az * phi_cut) +
              0x1p-24L * fabsl(exact) + 1e-45L;
          if (err > bound) ++bad[t];
          const double rel = (double)(err / bound);
          if (rel > w) w = rel;
        }
      }
      worst2[t] = w;
    });
  for (auto &x : th) x.join();
  double e2 = 0.0;
  long nbad = 0;
  for (unsigned t = 0; t < nt; ++t) {
    e2 = std::max(e2, worst2[t]);
    nbad += bad[t];
  }
  std::printf("log2 error %.3e (bound %.3e); GELU error / bound max %.3f; failures %ld\n", e1,
              delta, e2, nbad);
  return (e1 <= delta && nbad == 0) ? 0 : 1;
}
