// Device helpers shared by the libcgs kernels (wave64, gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"
#include "stepdiv.h"

namespace cgs {

constexpr int kWave = 64;

__device__ __forceinline__ uint32_t fastdiv(uint32_t n, FastDiv d) {
  const uint32_t t = __umulhi(d.m, n);
  return (t + ((n - t) >> (d.sh & 0xffu))) >> (d.sh >> 8);
}

// Mixed-radix decode of raw index k (parameter 0 most significant) into
// 4-bit digits: parameters 0..15 in `lo`, 16..31 in `hi`.
__device__ __forceinline__ void decode_packed(uint32_t k, const SpaceDev *__restrict__ sp,
                                              uint64_t &lo, uint64_t &hi) {
  lo = 0;
  hi = 0;
  const int n = sp->n_params;
  for (int j = n - 1; j >= 16; --j) {
    const uint32_t q = fastdiv(k, sp->div[j]);
    hi |= (uint64_t)(k - q * sp->radix[j]) << (4 * (j - 16));
    k = q;
  }
  for (int j = (n < 16 ? n : 16) - 1; j >= 0; --j) {
    const uint32_t q = fastdiv(k, sp->div[j]);
    lo |= (uint64_t)(k - q * sp->radix[j]) << (4 * j);
    k = q;
  }
}

__device__ __forceinline__ uint32_t digit_of(uint64_t lo, uint64_t hi, uint32_t j) {
  const uint64_t w = j < 16 ? (lo >> (4 * j)) : (hi >> (4 * (j - 16)));
  return (uint32_t)w & 15u;
}

__device__ __forceinline__ uint32_t uabs32(int32_t v) {
  return v < 0 ? (uint32_t)(-(int64_t)v) : (uint32_t)v;
}

// AND of all constraints for one configuration.  `table` is the space's value
// table staged in LDS.
__device__ __forceinline__ bool satisfies_all(const SpaceDev *__restrict__ sp,
                                              const int32_t *table, uint64_t lo, uint64_t hi) {
  bool ok = true;
  const int nc = sp->n_cons;
  for (int c = 0; c < nc; ++c) {
    const uint32_t code = sp->cons_code[c];
    const uint32_t kind = code & 0xffu, a = (code >> 8) & 0xffu, b = (code >> 16) & 0xffu,
                   cc = code >> 24;
    const int64_t bound = sp->cons_bound[c];
    const int32_t va = table[a * CGS_MAX_RADIX + digit_of(lo, hi, a)];
    const int32_t vb = table[b * CGS_MAX_RADIX + digit_of(lo, hi, b)];
    const int32_t vc = table[cc * CGS_MAX_RADIX + digit_of(lo, hi, cc)];
    bool r;
    switch (kind) {
    case CGS_DIV: {
      const uint32_t d = uabs32(vb);
      r = d != 0 && (uabs32(va) % d) == 0;
      break;
    }
    case CGS_DIV2: {
      // |v| < 2^20, so |vb * vc| < 2^40; a divisor larger than |va| divides
      // only va == 0.
      const uint64_t d = (uint64_t)uabs32(vb) * (uint64_t)uabs32(vc);
      const uint32_t n = uabs32(va);
      r = d != 0 && (d > n ? n == 0 : (n % (uint32_t)d) == 0);
      break;
    }
    case CGS_PROD_LE: r = (int64_t)va * vb <= bound; break;
    case CGS_PROD3_LE: r = (int64_t)va * vb * vc <= bound; break;
    case CGS_PROD_GE: r = (int64_t)va * vb >= bound; break;
    default: r = va <= vb; break; // CGS_LE
    }
    ok = ok && r;
  }
  return ok;
}

// Order-preserving map float -> uint32 (a < b  <=>  key(a) < key(b) for
// non-NaN values), so min/max reduce with integer atomics.
__device__ __forceinline__ uint32_t float_key(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_float(uint32_t k) {
  const uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __uint_as_float(u);
}

// The constants of one step's normalisation: the divisors of positive
// scores (s_max) and of the others (-s_min) with their reciprocals
// (stepdiv.h), the cut-off and the smallest weight.  1 - s / s_min is
// formed as 1 + s / (-s_min): the same float, since IEEE division and
// rounding to nearest are symmetric under a change of sign.  A divisor that
// no unexplored configuration divides by (s_max <= 0: no positive score;
// s_min >= 0: only zero scores, whose quotient is 0 for any divisor) is
// replaced by 1.
struct StepNorm {
  StepDivisor pos, neg; // s_max and -s_min
  bool fast;            // both divisors in the fast path's range
  bool wide;            // fast, and both divisors >= kWideDivisorMin
  float gamma, w_min;
};
// The reciprocals are made opaque to the optimiser: it would otherwise
// turn the per-lane choice between two reciprocals back into one division
// per configuration.
__device__ __forceinline__ float opaque(float x) {
  asm volatile("" : "+v"(x));
  return x;
}
__device__ __forceinline__ StepNorm step_norm(float s_min, float s_max, float gamma, float w_min) {
  StepNorm nm{step_divisor(s_max > 0.0f ? s_max : 1.0f),
              step_divisor(s_min < 0.0f ? -s_min : 1.0f), false, false, gamma, w_min};
  nm.fast = nm.pos.fast && nm.neg.fast;
  nm.wide = nm.fast && nm.pos.d >= kWideDivisorMin && nm.neg.d >= kWideDivisorMin;
  nm.pos.r = opaque(nm.pos.r);
  nm.neg.r = opaque(nm.neg.r);
  return nm;
}

// Normalised weight of the score-normalisation equation, quantised to
// rint(w * 2^23):
//   s > 0: (1 + s/s_max)^8;  gamma < s <= 0: max(w_min, (1 - s/s_min)^8),
//   1 when s == 0;  s <= gamma: w_min;  explored: 0.
// The eighth power is three squarings.  With gamma <= 0 and w_min <= 1 (the
// session's parameters are checked for both) the cases fold into
//   y = 1 + s / D (D = s_max or -s_min by the sign of s),
//   w = s > gamma ? max(w_min, y^8) : w_min
// (for s > 0, y^8 >= 1 >= w_min): every value is the same float as the
// case-by-case form.  The division is correctly rounded through the step's
// reciprocal (stepdiv.h) wherever the fast path's operand range holds (the
// divisors are checked once per step; |s| <= D for every unexplored
// configuration, so only a non-zero |s| below 2^-60 leaves it) and the IEEE
// division otherwise.  When the step's divisors are both at least
// kWideDivisorMin (nm.wide, kWide = true) no score needs the division: below
// the range only 1 + s / D = 1 matters, which the sequence also gives
// (stepdiv.h), so the per-configuration range check goes too.
template <bool kWide>
__device__ __forceinline__ uint32_t quantized_weight_t(float s, bool explored, const StepNorm &nm) {
  const bool pos = s > 0.0f;
  const float d = pos ? nm.pos.d : nm.neg.d;
  float t;
  if (kWide) {
    t = div_fast_core(s, d, pos ? nm.pos.r : nm.neg.r);
  } else if (nm.fast) {
    t = div_fast_core(s, d, pos ? nm.pos.r : nm.neg.r); // +-0 for s == 0
    const uint32_t ab = __float_as_uint(s) & 0x7fffffffu;
    const bool slow = !explored && ab - 1u < 0x217fffffu; // 0 < |s| < 2^-60
    if (__any(slow)) t = slow ? s / d : t;
  } else {
    t = s == 0.0f ? 0.0f : s / d;
  }
  const float y = 1.0f + t;
  const float y2 = y * y;
  const float y4 = y2 * y2;
  const float y8 = y4 * y4;
  const float w = s > nm.gamma ? fmaxf(nm.w_min, y8) : nm.w_min;
  return explored ? 0u : (uint32_t)rintf(w * 8388608.0f);
}
__device__ __forceinline__ uint32_t quantized_weight(float s, bool explored, const StepNorm &nm) {
  return nm.wide ? quantized_weight_t<true>(s, explored, nm)
                 : quantized_weight_t<false>(s, explored, nm);
}

__device__ __forceinline__ bool explored_bit(const uint32_t *__restrict__ ex, uint32_t l) {
  return (ex[l >> 5] >> (l & 31u)) & 1u;
}

// ------------------------------------------------------------ wave / block
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ uint32_t wave_umin(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, kWave));
  return v;
}
__device__ __forceinline__ uint32_t wave_umax(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, kWave));
  return v;
}

// Inclusive scan across a wave.
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v, uint32_t lane) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint64_t t = __shfl_up(v, o, kWave);
    if (lane >= (uint32_t)o) v += t;
  }
  return v;
}

// Exclusive scan over the whole block (NT threads, NT % 64 == 0); `total`
// receives the block sum.  `scratch` holds NT / 64 entries.  Contains
// barriers: every thread must call it.
template <int NT>
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t *scratch, uint64_t &total) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  constexpr int NW = NT / kWave;
  const uint64_t incl = wave_incl_scan(v, lane);
  __syncthreads();
  if (lane == kWave - 1) scratch[wave] = incl;
  __syncthreads();
  uint64_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint64_t t = scratch[w];
    before += (w < (int)wave) ? t : 0ull;
    all += t;
  }
  total = all;
  return before + incl - v;
}

template <int NT> __device__ __forceinline__ uint64_t block_sum(uint64_t v, uint64_t *scratch) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  constexpr int NW = NT / kWave;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  uint64_t all = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) all += scratch[w];
  return all;
}

} // namespace cgs
