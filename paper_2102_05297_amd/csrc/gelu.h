// GELU of the perceptron's hidden layers for bf16 activations, evaluated in
// float32 with one exponential and no reciprocal:
//   GELU(z) = z Phi(z) = max(z, 0) - |z| Phi(-|z|),
//   Phi(-x) ~ 2^p(min(x, 9)),
// p a degree-7 polynomial fitted to log2 Phi(-x) on [0, 9] (weighted least
// squares in the Chebyshev basis, reweighted towards the largest errors, then
// expanded in powers of x and rounded to float32).  The tail term is formed
// directly, so negative z lose nothing to cancellation, and for z > 0 the
// subtracted term is at most half of max(z, 0).
//
// Accuracy (tests/gelu_check.cpp, float32 Horner evaluation against a long
// double reference): |p(x) - log2 Phi(-x)| <= 1.1e-4 on [0, 9], so the tail
// term errs by at most 7.7e-5 of itself plus the exponential's rounding,
// about 2^-13.6 relative: far below half a bf16 ulp (2^-9) of the
// activation.  Beyond |z| = 9 the tail uses Phi(-9) = 1.1e-19, so the value
// errs by less than 2 |z| Phi(-9) in absolute terms.
#pragma once

namespace cgs {

constexpr float kGeluTailMax = 9.0f;

// p(x) ~ log2 Phi(-x) for 0 <= x <= 9 (float32 Horner with fused
// multiply-adds).
__host__ __device__ __forceinline__ float gelu_tail_log2(float x) {
  float p = -9.777600098e-07f;
  p = fmaf(p, x, 4.039722626e-05f);
  p = fmaf(p, x, -7.236030069e-04f);
  p = fmaf(p, x, 7.502830587e-03f);
  p = fmaf(p, x, -5.144603923e-02f);
  p = fmaf(p, x, -4.614704549e-01f);
  p = fmaf(p, x, -1.149892092e+00f);
  return fmaf(p, x, -1.000098705e+00f);
}

} // namespace cgs
