// GELU of the perceptron's hidden layers for bf16 activations, evaluated in
// float32 with one exponential and no reciprocal:
//   GELU(z) = z Phi(z) = max(z, 0) - |z| Phi(-|z|),
//   Phi(-x) ~ 2^p(min(x, 6)),
// p a degree-6 polynomial fitted to log2 Phi(-x) on [0, 6] (weighted least
// squares in the Chebyshev basis, reweighted towards the largest errors, then
// expanded in powers of x and rounded to float32: gelu_fit.py).  The tail
// term is formed directly, so negative z lose nothing to cancellation, and
// for z > 0 the subtracted term is at most half of max(z, 0).
//
// Accuracy (tests/gelu_check.cpp, float32 Horner evaluation against a long
// double reference): |p(x) - log2 Phi(-x)| <= 1.15e-4 on [0, 6], so the
// tail term errs by at most 8e-5 of itself plus the exponential's rounding,
// about 2^-13.5 relative: far below half a bf16 ulp (2^-9) of the
// activation.  Beyond |z| = 6 the tail uses Phi(-6) = 9.9e-10, so the value
// errs by less than 2 |z| Phi(-6) in absolute terms.
#pragma once

namespace cgs {

constexpr float kGeluTailMax = 6.0f;

// p(x) ~ log2 Phi(-x) for 0 <= x <= 6 (float32 Horner with fused
// multiply-adds).
__host__ __device__ __forceinline__ float gelu_tail_log2(float x) {
  float p = 2.299025073e-05f;
  p = fmaf(p, x, -6.110958639e-04f);
  p = fmaf(p, x, 7.195475511e-03f);
  p = fmaf(p, x, -5.118479580e-02f);
  p = fmaf(p, x, -4.612732530e-01f);
  p = fmaf(p, x, -1.150172949e+00f);
  return fmaf(p, x, -1.000065088e+00f);
}

} // namespace cgs
