// Perceptron surrogate of the counter model: F -> H -> H -> C with GELU,
// bf16 weights and activations, fp32 accumulation on gfx950 MFMA
// (v_mfma_f32_32x32x16_bf16), fp32 master weights and Adam moments.
//
// Transposed formulation: every layer computes Z^T = W X^T, so weights are
// the MFMA A operand (rows = output features) and activations the B operand
// (columns = 32 configurations per wave).  The accumulator of a 32x32 block
// holds, in lane l and register i, row 8(i/4) + 4(l/32) + (i%4) of column
// l%32.  Registers 8s'..8s'+7 of a block are therefore exactly the B operand
// of one 16-deep K step whose k slots 8(l/32) + j map to rows
// 16s' + 8(j/4) + 4(l/32) + (j%4): the hidden activations never leave
// registers, provided the next layer's weight columns are stored in that
// order.  The packed weight arrays hold each A fragment as 64 lanes x 8 bf16:
//   W1p[r][s][lane][j] = W1[32r + lane%32][16s + 8(lane/32) + j]   (natural)
//   W2p[r][s][lane][j] = W2[32r + lane%32][kperm(s, lane/32, j)]
//   W3p[r][s][lane][j] = W3[32r + lane%32][kperm(s, lane/32, j)]
//   kperm(s, h, j) = 32(s/2) + 16(s%2) + 8(j/4) + 4h + (j%4)
// GELU uses erf from Abramowitz & Stegun 7.1.26 (|error| <= 1.5e-7), far
// below the bf16 rounding of the activations.
#include <algorithm>

#include "device_common.h"

namespace cgs {

namespace {

typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kGemmThreads = 256;

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Phi(z) and phi(z) = exp(-z^2/2) / sqrt(2 pi); erf by A&S 7.1.26.
__device__ __forceinline__ void normal_cdf_pdf(float z, float &cdf, float &pdf) {
  const float x = fabsf(z) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.3275911f * x);
  const float poly =
      t * (0.254829592f +
           t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
  const float e = __expf(-x * x);
  const float erf_abs = 1.0f - poly * e;
  cdf = 0.5f * (1.0f + (z >= 0.0f ? erf_abs : -erf_abs));
  pdf = e * 0.3989422804014327f;
}
// GELU(z) = z Phi(z) = max(z, 0) - |z| Phi(-|z|), where 2 Phi(-|z|) =
// erfc(|z| / sqrt 2) = t P(t) exp(-z^2 / 2) with t = 1 / (1 + p |z| / sqrt 2)
// (A&S 7.1.26; the coefficients below are P's halved).  The tail term is
// formed directly, so negative z lose nothing to cancellation.
__device__ __forceinline__ float gelu(float z) {
  const float az = fabsf(z);
  const float t = __builtin_amdgcn_rcpf(fmaf(az, 0.3275911f * 0.70710678118654752f, 1.0f));
  const float e = __builtin_amdgcn_exp2f(z * z * -0.72134752044448170f); // exp(-z^2 / 2)
  const float poly =
      0.127414796f +
      t * (-0.142248368f + t * (0.7107068705f + t * (-0.7265760135f + t * 0.5307027145f)));
  return fmaf(-(az * e) * t, poly, fmaxf(z, 0.0f));
}
__device__ __forceinline__ float gelu_grad(float z) {
  float c, p;
  normal_cdf_pdf(z, c, p);
  return c + z * p;
}

// ---------------------------------------------------------------- forward
// TRAIN: configurations cfg_raw[batch[i]] (batch may be null: i), writes
// X (bf16 [n][K1]), Z1, Z2 (fp32 [n][H]), H1, H2 (bf16 [n][H]) and the
// unclamped output Y (fp32 [n][Cp]).  Otherwise: the valid configurations
// idx[0..n) and P[c][l] = max(y_c, 0).
//
// H <= 256: layer-1 block r is computed right before layer 2 consumes its
// two K steps, accumulating all H/32 layer-2 blocks at once.
// H = 512: each wave first parks its layer-1 output in a private LDS region
// in fragment order ([r][s'][lane][8] bf16, conflict-free 16-byte reads),
// then accumulates layer 2 in groups of 8 output blocks.
// LDSW: packed weights staged in LDS once per workgroup (H <= 256).
template <int H, int NB3, int S1, bool TRAIN, bool LDSW>
__global__ __launch_bounds__(LDSW ? 512 : 256) void mlp_forward(MlpFwdArgs a) {
  constexpr int NB = H / 32;
  constexpr int S2 = H / 16;
  constexpr int K1 = 16 * S1;
  constexpr bool H1_IN_LDS = H > 256;
  constexpr int G = H1_IN_LDS ? 8 : NB; // layer-2 output blocks per group
  static_assert(!(LDSW && H1_IN_LDS), "weights and hidden activations cannot both use LDS");
  extern __shared__ bf16x8 lds[];
  constexpr int N2 = H * H / 8, N3 = NB3 * 32 * H / 8, N1 = H * K1 / 8;
  if constexpr (LDSW) {
    for (int i = threadIdx.x; i < N2; i += blockDim.x) lds[i] = a.w2p[i];
    for (int i = threadIdx.x; i < N3; i += blockDim.x) lds[N2 + i] = a.w3p[i];
    for (int i = threadIdx.x; i < N1; i += blockDim.x) lds[N2 + N3 + i] = a.w1p[i];
    __syncthreads();
  }
#define W2F(ix) (LDSW ? lds[(ix)] : a.w2p[(ix)])
#define W3F(ix) (LDSW ? lds[N2 + (ix)] : a.w3p[(ix)])
#define W1F(ix) (LDSW ? lds[N2 + N3 + (ix)] : a.w1p[(ix)])
  const int lane = threadIdx.x & 63, hh = lane >> 5, col = lane & 31;
  const uint32_t wave_in_block = threadIdx.x / 64;
  // private hidden-activation region of this wave (H1_IN_LDS): NB * 2 * 64 fragments
  bf16x8 *h1lds = lds + (size_t)wave_in_block * NB * 2 * 64;
  const uint32_t waves_per_block = blockDim.x / 64;
  const uint32_t n_waves = gridDim.x * waves_per_block;
  const uint32_t n_tiles = (a.n + 31) / 32;
  for (uint32_t tile = blockIdx.x * waves_per_block + wave_in_block; tile < n_tiles;
       tile += n_waves) {
    const uint32_t i = tile * 32 + col;
    const bool ok = i < a.n;
    uint32_t raw = 0;
    if (ok) raw = TRAIN ? a.cfg_raw[a.batch ? (uint32_t)a.batch[i] : i] : a.idx[i];
    uint64_t lo = 0, hi = 0;
    if (ok) decode_packed(raw, a.sp, lo, hi);
    bf16x8 xb[S1];
#pragma unroll
    for (int s = 0; s < S1; ++s)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = 16 * s + 8 * hh + j;
        const float f = (ok && k < a.F) ? (float)digit_of(lo, hi, (uint32_t)k) * 0.125f : 0.0f;
        xb[s][j] = (__bf16)f;
        if (TRAIN && ok) a.xout[(size_t)i * K1 + k] = xb[s][j];
      }

    // layer-1 block r -> its two B fragments for layer 2
    auto layer1 = [&](int r, bf16x8 &f0, bf16x8 &f1) {
      f32x16 acc = {};
#pragma unroll
      for (int s = 0; s < S1; ++s) acc = mfma(W1F((r * S1 + s) * 64 + lane), xb[s], acc);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row0 = 32 * r + 8 * q + 4 * hh;
        const float4 bb = *reinterpret_cast<const float4 *>(a.b1 + row0);
        const float z[4] = {acc[4 * q] + bb.x, acc[4 * q + 1] + bb.y, acc[4 * q + 2] + bb.z,
                            acc[4 * q + 3] + bb.w};
        if (TRAIN && ok)
          *reinterpret_cast<float4 *>(a.z1out + (size_t)i * H + row0) =
              make_float4(z[0], z[1], z[2], z[3]);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const __bf16 v = (__bf16)gelu(z[t]);
          if (q < 2) f0[q * 4 + t] = v;
          else f1[(q - 2) * 4 + t] = v;
          if (TRAIN && ok) a.h1out[(size_t)i * H + row0 + t] = v;
        }
      }
    };

    if constexpr (H1_IN_LDS) {
#pragma unroll 2
      for (int r = 0; r < NB; ++r) {
        bf16x8 f0, f1;
        layer1(r, f0, f1);
        h1lds[(r * 2 + 0) * 64 + lane] = f0;
        h1lds[(r * 2 + 1) * 64 + lane] = f1;
      }
    }

    f32x16 accy[NB3];
#pragma unroll
    for (int r3 = 0; r3 < NB3; ++r3) accy[r3] = f32x16{};
#pragma unroll
    for (int g = 0; g < NB / G; ++g) {
      f32x16 acc2[G];
#pragma unroll
      for (int gi = 0; gi < G; ++gi) acc2[gi] = f32x16{};
      // B fragments of layer-2 K steps 2r, 2r+1
      auto hidden = [&](int r, bf16x8 (&f)[2]) {
        if constexpr (H1_IN_LDS) {
          f[0] = h1lds[(r * 2 + 0) * 64 + lane];
          f[1] = h1lds[(r * 2 + 1) * 64 + lane];
        } else {
          layer1(r, f[0], f[1]);
        }
      };
      auto load_w = [&](int r, bf16x8 (&w)[2][G]) {
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
          for (int gi = 0; gi < G; ++gi) w[sp][gi] = W2F(((g * G + gi) * S2 + 2 * r + sp) * 64 + lane);
      };
      auto multiply = [&](const bf16x8 (&w)[2][G], const bf16x8 (&f)[2]) {
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
          for (int gi = 0; gi < G; ++gi) acc2[gi] = mfma(w[sp][gi], f[sp], acc2[gi]);
      };
      if constexpr (LDSW) {
        // LDS fragments: short latency, one K step's fragments at a time
#pragma unroll 1
        for (int r = 0; r < NB; ++r) {
          bf16x8 f[2];
          hidden(r, f);
#pragma unroll
          for (int sp = 0; sp < 2; ++sp) {
            bf16x8 w[G];
#pragma unroll
            for (int gi = 0; gi < G; ++gi) w[gi] = W2F(((g * G + gi) * S2 + 2 * r + sp) * 64 + lane);
#pragma unroll
            for (int gi = 0; gi < G; ++gi) acc2[gi] = mfma(w[gi], f[sp], acc2[gi]);
          }
        }
      } else {
        // global fragments: the next K step's loads overlap this step's MFMAs
        bf16x8 wa[2][G], wb[2][G];
        load_w(0, wa);
#pragma unroll 1
        for (int r = 0; r < NB; r += 2) {
          bf16x8 f[2];
          load_w(r + 1, wb);
          hidden(r, f);
          multiply(wa, f);
          if (r + 2 < NB) load_w(r + 2, wa);
          hidden(r + 1, f);
          multiply(wb, f);
        }
      }
#pragma unroll
      for (int gi = 0; gi < G; ++gi) {
        bf16x8 h2[2];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row0 = 32 * (g * G + gi) + 8 * q + 4 * hh;
          const float4 bb = *reinterpret_cast<const float4 *>(a.b2 + row0);
          const float z[4] = {acc2[gi][4 * q] + bb.x, acc2[gi][4 * q + 1] + bb.y,
                              acc2[gi][4 * q + 2] + bb.z, acc2[gi][4 * q + 3] + bb.w};
          if (TRAIN && ok)
            *reinterpret_cast<float4 *>(a.z2out + (size_t)i * H + row0) =
                make_float4(z[0], z[1], z[2], z[3]);
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const __bf16 v = (__bf16)gelu(z[t]);
            h2[q >> 1][(q & 1) * 4 + t] = v;
            if (TRAIN && ok) a.h2out[(size_t)i * H + row0 + t] = v;
          }
        }
#pragma unroll
        for (int sp = 0; sp < 2; ++sp)
#pragma unroll
          for (int r3 = 0; r3 < NB3; ++r3)
            accy[r3] = mfma(W3F((r3 * S2 + 2 * (g * G + gi) + sp) * 64 + lane), h2[sp], accy[r3]);
      }
    }

    // output
#pragma unroll
    for (int r3 = 0; r3 < NB3; ++r3)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int c = 32 * r3 + 8 * q + 4 * hh + t;
          if (ok && c < a.C) {
            const float y = accy[r3][4 * q + t] + a.b3[c];
            if (TRAIN)
              a.yout[(size_t)i * (32 * NB3) + c] = y;
            else
              a.P[(size_t)c * a.stride + i] = fmaxf(y, 0.0f);
          }
        }
  }
#undef W2F
#undef W3F
#undef W1F
}

// ------------------------------------------------------------- inference
// P[c][l] = max(y_c, 0) over the valid configurations idx[0..n), written for
// throughput.  One workgroup per CU, normally eight waves (two per SIMD); a
// wave carries T tiles of 32 configurations and keeps their hidden
// activations in registers, so one wave's bias + GELU epilogue (VALU) runs
// beside the other wave's MFMAs.
//   resident: W1, W2, W3 and the biases live in LDS for the whole launch
//             (when they fit: H <= 256).
//   stream:   W3, W1 and the biases live in LDS; W2 passes through a double
//             buffer one 32-row block at a time, the next block's global
//             loads overlapping the current block's MFMAs.
// tiles of 32 configurations per wave; waves per workgroup: two per SIMD
// (256 registers each), or one (512) where two output blocks and wide hidden
// layers would not fit
template <int H> constexpr int infer_tiles() { return 1; }
template <int H, int NB3> constexpr int infer_waves() { return NB3 == 2 && H >= 256 ? 4 : 8; }

template <int T, int S1>
__device__ __forceinline__ void infer_features(const MlpFwdArgs &a, uint32_t first, int hh,
                                               int col, bf16x8 (&xb)[T][S1], bool (&ok)[T]) {
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const uint32_t i = first + 32 * t + col;
    ok[t] = i < a.n;
    uint64_t lo = 0, hi = 0;
    if (ok[t]) decode_packed(a.idx[i], a.sp, lo, hi);
#pragma unroll
    for (int s = 0; s < S1; ++s)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = 16 * s + 8 * hh + j;
        const float f = (ok[t] && k < a.F) ? (float)digit_of(lo, hi, (uint32_t)k) * 0.125f : 0.0f;
        xb[t][s][j] = (__bf16)f;
      }
  }
}

// Bias + GELU of one 32x32 accumulator block, as the two bf16 B fragments of
// the next layer's K steps 2r and 2r + 1; `b` points at bias[32 r + 4 hh].
// LOWREG: four values at a time (fewer live temporaries).
template <bool LOWREG = false>
__device__ __forceinline__ void gelu_frags(const f32x16 &acc, const float *b, bf16x8 &f0,
                                           bf16x8 &f1) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 bb = *reinterpret_cast<const float4 *>(b + 8 * q);
    const float z[4] = {acc[4 * q] + bb.x, acc[4 * q + 1] + bb.y, acc[4 * q + 2] + bb.z,
                        acc[4 * q + 3] + bb.w};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const __bf16 v = (__bf16)gelu(z[t]);
      if (q < 2) f0[q * 4 + t] = v;
      else f1[(q - 2) * 4 + t] = v;
    }
    if (LOWREG) __builtin_amdgcn_sched_barrier(0);
  }
}

template <int T, int NB3>
__device__ __forceinline__ void infer_store(const MlpFwdArgs &a, const f32x16 (&accy)[NB3][T],
                                            const float *b3, uint32_t first, int hh, int col,
                                            const bool (&ok)[T]) {
#pragma unroll
  for (int t = 0; t < T; ++t) {
    if (!ok[t]) continue;
    const uint32_t i = first + 32 * t + col;
#pragma unroll
    for (int r3 = 0; r3 < NB3; ++r3)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = 32 * r3 + 8 * q + 4 * hh + u;
          if (c < a.C) a.P[(size_t)c * a.stride + i] = fmaxf(accy[r3][t][4 * q + u] + b3[c], 0.0f);
        }
  }
}

// Stages n 16-byte units from global to LDS with every thread of the block,
// 8 loads per thread in flight before the first LDS store (a plain loop
// waits for every load in turn).
__device__ __forceinline__ void stage_units(bf16x8 *dst, const bf16x8 *src, int n) {
  constexpr int B = 8;
  for (int i0 = threadIdx.x; i0 < n; i0 += B * (int)blockDim.x) {
    bf16x8 v[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int i = i0 + b * (int)blockDim.x;
      v[b] = i < n ? src[i] : bf16x8{};
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int i = i0 + b * (int)blockDim.x;
      if (i < n) dst[i] = v[b];
    }
  }
}

// Biases in LDS: b1[H], b2[H], b3[32 NB3] (zero past C).
__device__ __forceinline__ void stage_biases(float *bias, const MlpFwdArgs &a, int H, int NB3) {
  for (int i = threadIdx.x; i < H; i += blockDim.x) {
    bias[i] = a.b1[i];
    bias[H + i] = a.b2[i];
  }
  for (int i = threadIdx.x; i < 32 * NB3; i += blockDim.x) bias[2 * H + i] = i < a.C ? a.b3[i] : 0.0f;
}

// Layer 1 of the wave's tiles: h1[2r + sp][t] for every block r.
template <int H, int T, int S1>
__device__ __forceinline__ void infer_layer1(const bf16x8 *w1, const float *bias, int lane, int hh,
                                             const bf16x8 (&xb)[T][S1], bf16x8 (&h1)[H / 16][T]) {
#pragma unroll
  for (int r = 0; r < H / 32; ++r) {
    bf16x8 wf[S1];
#pragma unroll
    for (int s = 0; s < S1; ++s) wf[s] = w1[(r * S1 + s) * 64 + lane];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      f32x16 acc = {};
#pragma unroll
      for (int s = 0; s < S1; ++s) acc = mfma(wf[s], xb[t][s], acc);
      gelu_frags(acc, bias + 32 * r + 4 * hh, h1[2 * r][t], h1[2 * r + 1][t]);
    }
    __builtin_amdgcn_sched_barrier(0); // one block's temporaries live at a time
  }
}

// Epilogue of layer-2 block r: bias + GELU, then its two K steps of layer 3.
template <int H, int T, int NB3, bool LOWREG = false>
__device__ __forceinline__ void infer_block_out(const f32x16 (&acc)[T], int r, const bf16x8 *w3,
                                                const float *bias, int lane, int hh,
                                                f32x16 (&accy)[NB3][T]) {
  constexpr int S2 = H / 16;
  bf16x8 w3f[NB3][2];
#pragma unroll
  for (int r3 = 0; r3 < NB3; ++r3)
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) w3f[r3][sp] = w3[(r3 * S2 + 2 * r + sp) * 64 + lane];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    bf16x8 f0, f1;
    gelu_frags<LOWREG>(acc[t], bias + H + 32 * r + 4 * hh, f0, f1);
#pragma unroll
    for (int r3 = 0; r3 < NB3; ++r3) {
      accy[r3][t] = mfma(w3f[r3][0], f0, accy[r3][t]);
      accy[r3][t] = mfma(w3f[r3][1], f1, accy[r3][t]);
    }
  }
}

template <int H, int NB3, int S1, bool RESIDENT, bool W1LDS>
constexpr size_t infer_lds() {
  return (size_t)((RESIDENT ? H * H : 2 * 32 * H) + NB3 * 32 * H + (W1LDS ? H * 16 * S1 : 0)) * 2 +
         (size_t)(2 * H + 32 * NB3) * 4;
}

// RESIDENT: W2 stays in LDS; otherwise its 32-row blocks pass through a
// double buffer.
template <int H, int NB3, int S1, bool RESIDENT, bool W1LDS>
__global__ __launch_bounds__((infer_waves<H, NB3>() * 64))
__attribute__((amdgpu_waves_per_eu((infer_waves<H, NB3>() / 4), (infer_waves<H, NB3>() / 4)))) void
mlp_infer(
    MlpFwdArgs a) {
  constexpr int T = infer_tiles<H>(), NB = H / 32, S2 = H / 16;
  constexpr int NW = infer_waves<H, NB3>(), NT = NW * 64;
  constexpr int NBLK = S2 * 64; // 16-byte units of one 32-row block of W2p
  constexpr int PER = RESIDENT ? 1 : NBLK / NT; // staged units per thread per block
  constexpr int N2 = RESIDENT ? NB * NBLK : 2 * NBLK;
  constexpr int N3 = NB3 * 32 * H / 8, N1 = H * 16 * S1 / 8;
  static_assert(RESIDENT || NBLK % NT == 0, "whole staged units per thread");
  extern __shared__ bf16x8 lds[];
  bf16x8 *w2 = lds, *w3 = lds + N2, *w1l = w3 + N3;
  float *bias = reinterpret_cast<float *>(w1l + (W1LDS ? N1 : 0));
  const bf16x8 *w1 = W1LDS ? w1l : a.w1p;
  if (RESIDENT) stage_units(w2, a.w2p, N2);
  stage_units(w3, a.w3p, N3);
  if (W1LDS) stage_units(w1l, a.w1p, N1);
  stage_biases(bias, a, H, NB3);
  __syncthreads();
  const int lane = threadIdx.x & 63, hh = lane >> 5, col = lane & 31;
  const int tid = threadIdx.x;
  constexpr uint32_t kWgConfigs = 32 * T * NW;
  const uint32_t n_wg = (a.n + kWgConfigs - 1) / kWgConfigs;
  // every wave of the block runs the same iterations (block barriers)
  for (uint32_t wg = blockIdx.x; wg < n_wg; wg += gridDim.x) {
    const uint32_t first = wg * kWgConfigs + (uint32_t)(tid / 64) * 32 * T;
    if (!RESIDENT) {
#pragma unroll
      for (int u = 0; u < PER; ++u) w2[u * NT + tid] = a.w2p[u * NT + tid];
    }
    bf16x8 xb[T][S1];
    bool ok[T];
    infer_features<T, S1>(a, first, hh, col, xb, ok);
    bf16x8 h1[S2][T];
    infer_layer1<H, T, S1>(w1, bias, lane, hh, xb, h1);
    f32x16 accy[NB3][T];
#pragma unroll
    for (int r3 = 0; r3 < NB3; ++r3)
#pragma unroll
      for (int t = 0; t < T; ++t) accy[r3][t] = f32x16{};
    if (!RESIDENT) __syncthreads(); // block 0 in the first buffer
    // with two waves per SIMD the other wave's MFMAs cover this one's epilogue
#pragma unroll 1
    for (int r = 0; r < NB; ++r) {
      const bf16x8 *wr = RESIDENT ? w2 + r * NBLK : w2 + (r & 1) * NBLK;
      const bool more = !RESIDENT && r + 1 < NB;
      bf16x8 st[RESIDENT ? 1 : PER];
      if (more) {
#pragma unroll
        for (int u = 0; u < PER; ++u) st[u] = a.w2p[(size_t)(r + 1) * NBLK + u * NT + tid];
      }
      f32x16 acc[T];
#pragma unroll
      for (int t = 0; t < T; ++t) acc[t] = f32x16{};
#pragma unroll
      for (int ks = 0; ks < S2; ++ks) {
        const bf16x8 wf = wr[ks * 64 + lane];
#pragma unroll
        for (int t = 0; t < T; ++t) acc[t] = mfma(wf, h1[ks][t], acc[t]);
        // at most four fragments in flight ahead of their MFMAs
        if (ks % 4 == 3) __builtin_amdgcn_sched_barrier(0);
      }
      infer_block_out<H, T, NB3, true>(acc, r, w3, bias, lane, hh, accy);
      if (more) {
#pragma unroll
        for (int u = 0; u < PER; ++u) w2[((r + 1) & 1) * NBLK + u * NT + tid] = st[u];
      }
      if (!RESIDENT) __syncthreads();
    }
    infer_store<T, NB3>(a, accy, bias + 2 * H, first, hh, col, ok);
  }
}

// ------------------------------------------------------------------ GEMM
// C[M][N] = sum_k A(m, k) B(k, n), bf16 operands (converted on load), fp32
// accumulation; one 32x32 output tile per workgroup, its K range split over
// the workgroup's waves (kGemmThreads / 64), partial tiles summed in LDS.
// Operands are addressed with arbitrary strides so transposed products need
// no copies.
template <typename T> __device__ __forceinline__ __bf16 to_bf16(T v);
template <> __device__ __forceinline__ __bf16 to_bf16<float>(float v) { return (__bf16)v; }
template <> __device__ __forceinline__ __bf16 to_bf16<__bf16>(__bf16 v) { return v; }

template <typename TA, typename TB, int EPI>
__global__ __launch_bounds__(kGemmThreads) void gemm_bf16(GemmArgs g) {
  constexpr int NW = kGemmThreads / 64;
  __shared__ float part[NW - 1][16][64];
  const TA *A = static_cast<const TA *>(g.A);
  const TB *B = static_cast<const TB *>(g.B);
  const int tiles_n = (g.N + 31) / 32;
  const int m0 = (blockIdx.x / tiles_n) * 32, n0 = (blockIdx.x % tiles_n) * 32;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, hh = lane >> 5, c = lane & 31;
  const int m = m0 + c, n = n0 + c;
  f32x16 acc = {};
  for (int k0 = 16 * w; k0 < g.K; k0 += 16 * NW) {
    bf16x8 af, bf;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + 8 * hh + j;
      af[j] = (m < g.M && k < g.K) ? to_bf16(A[(size_t)m * g.a_sm + (size_t)k * g.a_sk])
                                   : (__bf16)0.0f;
      bf[j] = (n < g.N && k < g.K) ? to_bf16(B[(size_t)k * g.b_sk + (size_t)n * g.b_sn])
                                   : (__bf16)0.0f;
    }
    acc = mfma(af, bf, acc);
  }
  if (w > 0) {
#pragma unroll
    for (int i = 0; i < 16; ++i) part[w - 1][i][lane] = acc[i];
  }
  __syncthreads();
  if (w != 0) return;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
#pragma unroll
    for (int q = 0; q < NW - 1; ++q) acc[i] += part[q][i][lane];
    const int row = m0 + 8 * (i / 4) + 4 * hh + (i % 4), cl = n0 + c;
    if (row >= g.M || cl >= g.N) continue;
    const size_t o = (size_t)row * g.ldc + cl;
    if (EPI == 0) {
      g.Cf[o] = acc[i];
    } else { // dZ = dH * gelu'(Z)
      const float v = acc[i] * gelu_grad(g.Z[o]);
      g.Cf[o] = v;
      g.Cb[o] = (__bf16)v;
    }
  }
}

// ------------------------------------------------------ loss, biases, Adam
// dY = 2 (Y - T) / (n C) in fp32 and bf16, and the mean squared error.
__global__ __launch_bounds__(1024) void mse_grad(const float *__restrict__ Y, int Cp, int C, int n,
                                                 const float *__restrict__ targets,
                                                 const int32_t *__restrict__ batch,
                                                 float *__restrict__ dYf, __bf16 *__restrict__ dYb,
                                                 float *__restrict__ loss_out) {
  __shared__ float red[16];
  const float scale = 2.0f / (float)(n * C);
  float sum = 0.0f;
  for (int e = threadIdx.x; e < n * Cp; e += 1024) {
    const int b = e / Cp, cc = e % Cp;
    float d = 0.0f;
    if (cc < C) {
      const int src = batch ? batch[b] : b;
      d = Y[(size_t)b * Cp + cc] - targets[(size_t)src * C + cc];
      sum += d * d;
    }
    dYf[e] = scale * d;
    dYb[e] = (__bf16)(scale * d);
  }
  sum = wave_sum(sum);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.0f;
    for (int w = 0; w < 16; ++w) t += red[w];
    *loss_out = t / (float)(n * C);
  }
}

// Bias gradients: column sums over the batch.  A workgroup takes 64
// consecutive columns (lane = column, coalesced rows); its 16 waves split the
// rows and their partial sums meet in LDS.
constexpr int kBiasWaves = 16;
__global__ __launch_bounds__(kBiasWaves * 64) void bias_grads(
    const float *__restrict__ dz1, const float *__restrict__ dz2, const float *__restrict__ dyf,
    int n, int H, int C, int Cp, float *__restrict__ gb1, float *__restrict__ gb2,
    float *__restrict__ gb3) {
  __shared__ float part[kBiasWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const float *src = nullptr;
  float *dst = nullptr;
  int ld = 0, col = 0;
  if (c < H) {
    src = dz1, dst = gb1, ld = H, col = c;
  } else if (c < 2 * H) {
    src = dz2, dst = gb2, ld = H, col = c - H;
  } else if (c < 2 * H + C) {
    src = dyf, dst = gb3, ld = Cp, col = c - 2 * H;
  }
  float sum = 0.0f;
  if (src) {
#pragma unroll 4
    for (int b = w; b < n; b += kBiasWaves) sum += src[(size_t)b * ld + col];
  }
  part[w][lane] = sum;
  __syncthreads();
  if (w == 0 && src) {
    float t = 0.0f;
#pragma unroll
    for (int k = 0; k < kBiasWaves; ++k) t += part[k][lane];
    dst[col] = t;
  }
}

// Position of master parameter p in the packed bf16 weight arrays, or -1
// for biases.  which: 1, 2, 3 = W1p, W2p, W3p.
__device__ __forceinline__ long packed_position(const MlpShape &sh, size_t p, int &which) {
  const size_t w1 = (size_t)sh.H * sh.F, b1 = sh.H, w2 = (size_t)sh.H * sh.H, b2 = sh.H;
  const size_t w3 = (size_t)sh.C * sh.H;
  const int S1 = sh.K1 / 16, S2 = sh.H / 16;
  if (p < w1) {
    const int o = (int)(p / sh.F), f = (int)(p % sh.F);
    const int s = f / 16, kk = f % 16, hh = kk / 8, j = kk % 8;
    const int lane = hh * 32 + o % 32;
    which = 1;
    return ((long)((o / 32) * S1 + s) * 64 + lane) * 8 + j;
  }
  p -= w1;
  if (p < b1) return which = 0, -1;
  p -= b1;
  size_t o, k;
  if (p < w2) {
    o = p / sh.H;
    k = p % sh.H;
    which = 2;
  } else {
    p -= w2;
    if (p < b2) return which = 0, -1;
    p -= b2;
    if (p >= w3) return which = 0, -1;
    o = p / sh.H;
    k = p % sh.H;
    which = 3;
  }
  const int r = (int)(k / 32), kk = (int)(k % 32), sp = kk / 16, rem = kk % 16;
  const int hh = (rem % 8) / 4, j = 4 * (rem / 8) + rem % 4;
  const int lane = hh * 32 + (int)(o % 32);
  return ((long)((o / 32) * S2 + 2 * r + sp) * 64 + lane) * 8 + j;
}

__device__ __forceinline__ void pack_one(const MlpShape &sh, size_t p, float v, __bf16 *w1p,
                                         __bf16 *w2p, __bf16 *w3p) {
  int which = 0;
  const long pos = packed_position(sh, p, which);
  if (which == 1) w1p[pos] = (__bf16)v;
  else if (which == 2) w2p[pos] = (__bf16)v;
  else if (which == 3) w3p[pos] = (__bf16)v;
}

__global__ __launch_bounds__(256) void pack_weights(MlpShape sh, const float *__restrict__ theta,
                                                    size_t n, __bf16 *w1p, __bf16 *w2p,
                                                    __bf16 *w3p) {
  const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (p < n) pack_one(sh, p, theta[p], w1p, w2p, w3p);
}

// Adam (Kingma & Ba, Algorithm 1); c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t).
__global__ __launch_bounds__(256) void adam_pack(MlpShape sh, float *__restrict__ theta,
                                                 float *__restrict__ m, float *__restrict__ v,
                                                 const float *__restrict__ grad, size_t n,
                                                 float lr, float b1, float b2, float eps, float c1,
                                                 float c2, __bf16 *w1p, __bf16 *w2p,
                                                 __bf16 *w3p) {
  const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  const float g = grad[p];
  const float mm = b1 * m[p] + (1.0f - b1) * g;
  const float vv = b2 * v[p] + (1.0f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const float th = theta[p] - lr * (mm * c1) / (sqrtf(vv * c2) + eps);
  theta[p] = th;
  pack_one(sh, p, th, w1p, w2p, w3p);
}

template <typename K>
hipError_t launch_infer_kernel(K kernel, size_t lds, uint32_t grid, uint32_t threads,
                               const MlpFwdArgs &a, hipStream_t stream) {
  if (grid == 0) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kernel, dim3(grid), dim3(threads), lds, stream, a);
  return hipGetLastError();
}

constexpr size_t kLdsBytes = 160 * 1024;

template <int H, int NB3, int S1>
hipError_t launch_infer_h(const MlpFwdArgs &a, hipStream_t stream) {
  const uint32_t cu = (uint32_t)std::max(a.n_cu, 1);
  constexpr uint32_t threads = infer_waves<H, NB3>() * 64;
  constexpr uint32_t wg_cfg = 32 * infer_tiles<H>() * infer_waves<H, NB3>();
  const uint32_t grid = std::min<uint32_t>((a.n + wg_cfg - 1) / wg_cfg, cu);
  if constexpr (infer_lds<H, NB3, S1, true, true>() <= kLdsBytes)
    return launch_infer_kernel(mlp_infer<H, NB3, S1, true, true>,
                               infer_lds<H, NB3, S1, true, true>(), grid, threads, a, stream);
  else if constexpr (infer_lds<H, NB3, S1, false, true>() <= kLdsBytes)
    return launch_infer_kernel(mlp_infer<H, NB3, S1, false, true>,
                               infer_lds<H, NB3, S1, false, true>(), grid, threads, a, stream);
  else
    return launch_infer_kernel(mlp_infer<H, NB3, S1, false, false>,
                               infer_lds<H, NB3, S1, false, false>(), grid, threads, a, stream);
}

template <int H> hipError_t launch_infer_nb(const MlpFwdArgs &a, hipStream_t s) {
  const int nb3 = (a.C + 31) / 32, s1 = a.K1 / 16;
  if (nb3 == 1 && s1 == 1) return launch_infer_h<H, 1, 1>(a, s);
  if (nb3 == 1 && s1 == 2) return launch_infer_h<H, 1, 2>(a, s);
  if (nb3 == 2 && s1 == 1) return launch_infer_h<H, 2, 1>(a, s);
  if (nb3 == 2 && s1 == 2) return launch_infer_h<H, 2, 2>(a, s);
  return hipErrorInvalidValue;
}

template <int H, int NB3, int S1, bool TRAIN, bool LDSW>
hipError_t launch_fwd_t(const MlpFwdArgs &a, hipStream_t stream) {
  const uint32_t n_tiles = (a.n + 31) / 32;
  if (n_tiles == 0) return hipSuccess;
  if (LDSW) {
    const size_t lds = (size_t)(H * H + NB3 * 32 * H + H * 16 * S1) * sizeof(__bf16);
    static bool attr_set = false;
    if (!attr_set) {
      hipError_t e = hipFuncSetAttribute(
          reinterpret_cast<const void *>(&mlp_forward<H, NB3, S1, TRAIN, LDSW>),
          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      attr_set = true;
    }
    const uint32_t grid = std::min<uint32_t>((n_tiles + 7) / 8, (uint32_t)a.n_cu);
    hipLaunchKernelGGL((mlp_forward<H, NB3, S1, TRAIN, LDSW>), dim3(grid), dim3(512), lds, stream,
                       a);
  } else {
    // H = 512: each of the 4 waves keeps its layer-1 output in LDS
    const size_t lds = H > 256 ? (size_t)4 * (H / 32) * 2 * 64 * sizeof(bf16x8) : 0;
    if (lds > 64 * 1024) {
      static bool attr_set = false;
      if (!attr_set) {
        hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&mlp_forward<H, NB3, S1, TRAIN, LDSW>),
            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
      }
    }
    const uint32_t grid = std::min<uint32_t>((n_tiles + 3) / 4, (uint32_t)a.n_cu * 8);
    hipLaunchKernelGGL((mlp_forward<H, NB3, S1, TRAIN, LDSW>), dim3(grid), dim3(256), lds, stream,
                       a);
  }
  return hipGetLastError();
}

template <int H, int NB3, int S1>
hipError_t launch_fwd_h(const MlpFwdArgs &a, bool train, hipStream_t stream) {
  if (train) return launch_fwd_t<H, NB3, S1, true, false>(a, stream);
  return launch_infer_h<H, NB3, S1>(a, stream);
}

template <int H> hipError_t launch_fwd_nb(const MlpFwdArgs &a, bool train, hipStream_t s) {
  const int nb3 = (a.C + 31) / 32, s1 = a.K1 / 16;
  if (nb3 == 1 && s1 == 1) return launch_fwd_h<H, 1, 1>(a, train, s);
  if (nb3 == 1 && s1 == 2) return launch_fwd_h<H, 1, 2>(a, train, s);
  if (nb3 == 2 && s1 == 1) return launch_fwd_h<H, 2, 1>(a, train, s);
  if (nb3 == 2 && s1 == 2) return launch_fwd_h<H, 2, 2>(a, train, s);
  return hipErrorInvalidValue;
}

} // namespace

hipError_t launch_mlp_forward(const MlpFwdArgs &a, bool train, hipStream_t stream) {
  switch (a.H) {
  case 64: return launch_fwd_nb<64>(a, train, stream);
  case 128: return launch_fwd_nb<128>(a, train, stream);
  case 256: return launch_fwd_nb<256>(a, train, stream);
  case 512: return launch_fwd_nb<512>(a, train, stream);
  default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gemm(const GemmArgs &g, int a_bf16, int b_bf16, int epi, hipStream_t stream) {
  const int tiles = ((g.M + 31) / 32) * ((g.N + 31) / 32);
  if (tiles == 0) return hipSuccess;
  const dim3 grid(tiles), block(kGemmThreads);
#define GEMM_CASE(TA, TB, E)                                                                   \
  hipLaunchKernelGGL((gemm_bf16<TA, TB, E>), grid, block, 0, stream, g)
  if (a_bf16 && b_bf16 && epi == 0) GEMM_CASE(__bf16, __bf16, 0);
  else if (a_bf16 && !b_bf16 && epi == 1) GEMM_CASE(__bf16, float, 1);
  else if (a_bf16 && !b_bf16 && epi == 0) GEMM_CASE(__bf16, float, 0);
  else if (a_bf16 && b_bf16 && epi == 1) GEMM_CASE(__bf16, __bf16, 1);
  else return hipErrorInvalidValue;
#undef GEMM_CASE
  return hipGetLastError();
}

hipError_t launch_mse_grad(const float *Y, int Cp, int C, int n, const float *targets,
                           const int32_t *batch, float *dYf, __bf16 *dYb, float *loss_out,
                           hipStream_t stream) {
  hipLaunchKernelGGL(mse_grad, dim3(1), dim3(1024), 0, stream, Y, Cp, C, n, targets, batch, dYf,
                     dYb, loss_out);
  return hipGetLastError();
}

hipError_t launch_bias_grads(const float *dz1, const float *dz2, const float *dyf, int n, int H,
                             int C, int Cp, float *gb1, float *gb2, float *gb3,
                             hipStream_t stream) {
  const int total = 2 * H + C;
  hipLaunchKernelGGL(bias_grads, dim3((total + 63) / 64), dim3(kBiasWaves * 64), 0, stream, dz1,
                     dz2, dyf, n, H, C, Cp, gb1, gb2, gb3);
  return hipGetLastError();
}

hipError_t launch_pack_weights(const MlpShape &sh, const float *theta, size_t n, __bf16 *w1p,
                               __bf16 *w2p, __bf16 *w3p, hipStream_t stream) {
  hipLaunchKernelGGL(pack_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, sh,
                     theta, n, w1p, w2p, w3p);
  return hipGetLastError();
}

hipError_t launch_adam_pack(const MlpShape &sh, float *theta, float *m, float *v,
                            const float *grad, size_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2, __bf16 *w1p, __bf16 *w2p, __bf16 *w3p,
                            hipStream_t stream) {
  hipLaunchKernelGGL(adam_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, sh, theta,
                     m, v, grad, n, lr, b1, b2, eps, c1, c2, w1p, w2p, w3p);
  return hipGetLastError();
}

} // namespace cgs
