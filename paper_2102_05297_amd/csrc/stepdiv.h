// Correctly rounded float32 division by a divisor that is fixed for a whole
// pass (the score-normalisation equation divides every score by s_max, or
// every non-positive one by s_min, Sect. 3.6).
//
// With r = RN(1/d) computed once by an IEEE division, each quotient costs
// one multiply and two fused multiply-adds instead of the general division
// sequence (operand scaling, reciprocal, five fused multiply-adds, fix-up):
//   q0 = RN(s * r)               within 1.5 ulp of s / d
//   e  = fma(-q0, d, s)          exact: the residual s - q0 d is a float
//   q1 = RN(q0 + e * r)          = RN(s / d)   (Markstein's correction)
// A second correction (e' = fma(-q1, d, s), q2 = fma(e', r, q1)) follows so
// that the result does not rest on q0 being faithful; it changes nothing
// when q1 is already RN(s / d).
//
// Validity: every intermediate must be a normal float.  Both operands are
// therefore confined to 2^-60 <= |x| <= 2^60 (s == 0 also takes the fast
// path and gives +-0 like the division), so |s / d| lies in
// [2^-120, 2^120], |r| in [2^-60, 2^60] and the residuals are at least
// 2^-24 * 2^-1 * |d| * ulp(q) >= 2^-110 in magnitude when non-zero.  Any
// other operand (tiny, huge, zero or non-finite divisor) takes the IEEE
// division, so the result equals s / d for every input.  Checked on the
// host against IEEE division for every numerator significand with several
// hundred divisor significands (tests/test_stepdiv.py), which covers every
// quotient up to scaling by powers of two.
#pragma once

namespace cgs {

struct StepDivisor {
  float d; // the divisor
  float r; // RN(1 / d)
  bool fast; // 2^-60 <= |d| <= 2^60
};

__host__ __device__ __forceinline__ StepDivisor step_divisor(float d) {
  const float ad = d < 0.0f ? -d : d;
  return StepDivisor{d, 1.0f / d, ad >= 0x1p-60f && ad <= 0x1p60f};
}

// The fast path's operand condition (above).
__host__ __device__ __forceinline__ bool div_fast_ok(float s, bool fast) {
  const float as = s < 0.0f ? -s : s;
  return fast && ((as >= 0x1p-60f && as <= 0x1p60f) || s == 0.0f);
}

// The correction sequence above; equal to s / d for non-zero s in the fast
// path's range, and +-0 (the sign of s * r, which may differ from the
// quotient's) for s == 0.
__host__ __device__ __forceinline__ float div_fast_core(float s, float d, float r) {
  const float q0 = s * r;
  const float e0 = fmaf(-q0, d, s);
  const float q1 = fmaf(e0, r, q0);
  const float e1 = fmaf(-q1, d, s);
  return fmaf(e1, r, q1);
}

// A pass whose divisor is at least 2^-34 (and in the fast range) may also
// send numerators below the range, 0 < |s| < 2^-60, through the correction
// sequence when only 1 + s / d is wanted: |s / d| < 2^-26, the sequence's
// result (its intermediates may be subnormal, or flushed) stays below 2^-25
// in magnitude as well, and 1 + t rounds to 1 for either value.  Checked on
// the host for subnormal and tiny numerators (tests/stepdiv_check.cpp).
constexpr float kWideDivisorMin = 0x1p-34f;

// s / d through r = RN(1 / d); equal to the IEEE quotient whenever
// div_fast_ok(s, step_divisor(d).fast).
__host__ __device__ __forceinline__ float div_fast(float s, float d, float r) {
  const float q0 = s * r;
  return s == 0.0f ? q0 : div_fast_core(s, d, r); // +-0 keeps the quotient's sign, as q0 does
}

// The quotient s / v.d for every input (the reference composition; device
// code branches to the division only when some lane of the wave needs it).
__host__ __device__ __forceinline__ float div_by(float s, const StepDivisor &v) {
  return div_fast_ok(s, v.fast) ? div_fast(s, v.d, v.r) : s / v.d;
}

} // namespace cgs
