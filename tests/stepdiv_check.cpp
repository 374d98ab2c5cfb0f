// Host check of the fixed-divisor division (paper_2102_05297_amd/csrc/stepdiv.h)
// against IEEE float32 division.  Correct rounding depends only on the
// significands while every intermediate is normal, so numerators run over
// every significand in [1, 2) (both signs, one exponent step either way)
// for each divisor significand given; plus operands outside the fast range,
// zeros and non-finite values; and 1 + s / d for numerators below the range
// with divisors of at least kWideDivisorMin.  Prints the number of
// mismatches.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#define __host__
#define __device__
#define __forceinline__ inline
#include "stepdiv.h"

static float from_bits(uint32_t u) { float f; std::memcpy(&f, &u, 4); return f; }
static uint32_t bits(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }
static bool same(float a, float b) { return bits(a) == bits(b) || (std::isnan(a) && std::isnan(b)); }
// the fast path wherever its condition holds, the division elsewhere
static bool agrees(float s, const cgs::StepDivisor &v) {
  if (!same(cgs::div_by(s, v), s / v.d)) return false;
  return !cgs::div_fast_ok(s, v.fast) || same(cgs::div_fast(s, v.d, v.r), s / v.d);
}

int main(int argc, char **argv) {
  const int n_random = argc > 1 ? std::atoi(argv[1]) : 256;
  std::vector<float> divs;
  // adversarial significands: next to 1 and 2, all-ones, powers of two
  for (uint32_t k = 0; k < 48; ++k) {
    divs.push_back(from_bits(0x3f800000u + k));
    divs.push_back(from_bits(0x3fffffffu - k));
  }
  std::mt19937_64 g(210205297);
  for (int i = 0; i < n_random; ++i) divs.push_back(from_bits(0x3f800000u | (uint32_t)(g() & 0x7fffffu)));
  std::vector<long> bad(divs.size(), 0);
  std::vector<std::thread> th;
  const unsigned nt = std::max(1u, std::thread::hardware_concurrency());
  for (unsigned t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      for (size_t i = t; i < divs.size(); i += nt) {
        for (int sd = 0; sd < 2; ++sd) {
          // divisor exponents: [1, 2) and a far scale; negative divisors too
          const float d = (sd ? -std::ldexp(divs[i], 37) : divs[i]);
          const cgs::StepDivisor v = cgs::step_divisor(d);
          for (uint32_t m = 0; m < (1u << 23); ++m) {
            for (int e = 0; e < 2; ++e) {
              const float s = from_bits(((uint32_t)(127 - e) << 23) | m) * (m & 1 ? -1.0f : 1.0f) *
                              (sd ? 0x1p30f : 1.0f);
              if (!agrees(s, v)) ++bad[i];
            }
          }
        }
      }
    });
  for (auto &x : th) x.join();
  long total = 0;
  for (long b : bad) total += b;
  // special operands: zeros, tiny and huge values, infinities, NaN
  const float sp[] = {0.0f, -0.0f, 1e-30f, -3e-38f, 1e-45f, 7e30f, -2e38f, INFINITY, -INFINITY, NAN,
                      0x1p-60f, 0x1p60f, 0x1.fffffep-61f, 0x1.000002p60f, 1.0f, -0.75f};
  for (float d : sp)
    for (float s : sp) {
      const cgs::StepDivisor v = cgs::step_divisor(d);
      if (!agrees(s, v)) {
        ++total;
        std::printf("special mismatch s=%a d=%a\n", s, d);
      }
    }
  // numerators below the fast range with a divisor of at least
  // kWideDivisorMin: 1 + (the sequence's result) must equal 1 + s / d (both
  // 1).  Every 61st float below 2^-60 (subnormals included), both signs.
  {
    std::vector<float> wd;
    for (float d : {cgs::kWideDivisorMin, 0x1.fffffep-34f, 0x1.000002p-34f, 0x1.8p-20f, 1.0f,
                    0x1.fffffep0f, 3.0f, 0x1p40f, 0x1.fffffep59f, 0x1p60f})
      wd.push_back(d);
    for (int i = 0; i < 22; ++i)
      wd.push_back(std::ldexp(from_bits(0x3f800000u | (uint32_t)(g() & 0x7fffffu)),
                              (int)(g() % 94) - 34));
    std::vector<long> badw(nt, 0);
    std::vector<std::thread> tw;
    const uint32_t top = bits(0x1p-60f);
    for (unsigned t = 0; t < nt; ++t)
      tw.emplace_back([&, t] {
        for (size_t i = 0; i < wd.size(); ++i) {
          const cgs::StepDivisor v = cgs::step_divisor(wd[i]);
          for (uint32_t b = 1 + 61 * t; b < top; b += 61 * nt)
            for (int sg = 0; sg < 2; ++sg) {
              const float s = sg ? -from_bits(b) : from_bits(b);
              if (!same(1.0f + cgs::div_fast_core(s, v.d, v.r), 1.0f + s / v.d)) ++badw[t];
            }
        }
      });
    for (auto &x : tw) x.join();
    long nw = 0;
    for (long b : badw) nw += b;
    std::printf("tiny numerators: divisors %zu mismatches %ld\n", wd.size(), nw);
    total += nw;
  }
  std::printf("divisors %zu mismatches %ld\n", divs.size(), total);
  return total != 0;
}
