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
// GELU's tail Phi(-|z|) is the exponential of a polynomial (gelu.h), within
// 2^-13.6 of itself: far below the bf16 rounding of the activations.  The
// training forward forms GELU'(z) from the same tail (within 4e-5 of it).
//
// Training runs a step in two launches (the training-step section below):
// the forward and backward chain per 32 rows of the batch, then the weight
// gradients by 32 x 32 tiles with Adam applied where they are formed.
#include <algorithm>

#include "device_common.h"
#include "gelu.h"
#include "models.h"

namespace cgs {

namespace {

typedef __attribute__((ext_vector_type(16))) float f32x16;


__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// min(|z|, 6) and max(z, 0) for finite z, each one v_med3_f32: written as
// fminf / fmaxf they would first canonicalise z (an accumulator value the
// compiler cannot prove canonical), one more instruction each.
__device__ __forceinline__ float tail_arg(float az) {
  return __builtin_amdgcn_fmed3f(az, 0.0f, kGeluTailMax);
}
__device__ __forceinline__ float relu(float z) {
  return __builtin_amdgcn_fmed3f(z, 0.0f, 3.40282347e38f);
}
// GELU(z) = max(z, 0) - |z| Phi(-|z|) with Phi(-x) = 2^p(min(x, 9)) (gelu.h):
// ten VALU operations and one exponential.
__device__ __forceinline__ float gelu(float z) {
  const float az = fabsf(z);
  const float e = __builtin_amdgcn_exp2f(gelu_tail_log2(tail_arg(az)));
  return fmaf(-az, e, relu(z));
}
// GELU(z) as above and, from the same tail, its derivative
// GELU'(z) = Phi(z) + z phi(z), phi(z) = 2^(-z^2 / (2 ln 2)) / sqrt(2 pi):
// the training forward keeps the derivative for the backward pass.
__device__ __forceinline__ float gelu_with_grad(float z, float &dg) {
  const float az = fabsf(z);
  const float e = __builtin_amdgcn_exp2f(gelu_tail_log2(tail_arg(az)));
  const float cdf = z > 0.0f ? 1.0f - e : e;
  const float pdf =
      0.3989422804014327f * __builtin_amdgcn_exp2f(-0.7213475204444817f * (z * z));
  dg = fmaf(z, pdf, cdf);
  return fmaf(-az, e, relu(z));
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

// The bias of one 32x32 accumulator block in the accumulator's layout (lane
// l, register i: row 8(i/4) + 4(l/32) + i%4); `b` points at
// bias[32 r + 4 hh].  Accumulating onto it adds the bias without a VALU
// operation per value.
__device__ __forceinline__ f32x16 bias_acc(const float *b) {
  f32x16 acc;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 bb = *reinterpret_cast<const float4 *>(b + 8 * q);
    acc[4 * q] = bb.x;
    acc[4 * q + 1] = bb.y;
    acc[4 * q + 2] = bb.z;
    acc[4 * q + 3] = bb.w;
  }
  return acc;
}

// GELU of one 32x32 accumulator block (bias included), as the two bf16 B
// fragments of the next layer's K steps 2r and 2r + 1.  LOWREG: four values
// at a time (fewer live temporaries).
template <bool LOWREG = false>
__device__ __forceinline__ void gelu_frags(const f32x16 &acc, bf16x8 &f0, bf16x8 &f1) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float z[4] = {acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]};
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
                                            uint32_t first, int hh, int col, const bool (&ok)[T]) {
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
          if (c < a.C) a.P[(size_t)c * a.stride + i] = fmaxf(accy[r3][t][4 * q + u], 0.0f);
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
      f32x16 acc = bias_acc(bias + 32 * r + 4 * hh);
#pragma unroll
      for (int s = 0; s < S1; ++s) acc = mfma(wf[s], xb[t][s], acc);
      gelu_frags(acc, h1[2 * r][t], h1[2 * r + 1][t]);
    }
    __builtin_amdgcn_sched_barrier(0); // one block's temporaries live at a time
  }
}

// Epilogue of layer-2 block r (bias included): GELU, then its two K steps
// of layer 3.
template <int H, int T, int NB3, bool LOWREG = false>
__device__ __forceinline__ void infer_block_out(const f32x16 (&acc)[T], int r, const bf16x8 *w3,
                                                int lane, f32x16 (&accy)[NB3][T]) {
  constexpr int S2 = H / 16;
  bf16x8 w3f[NB3][2];
#pragma unroll
  for (int r3 = 0; r3 < NB3; ++r3)
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) w3f[r3][sp] = w3[(r3 * S2 + 2 * r + sp) * 64 + lane];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    bf16x8 f0, f1;
    gelu_frags<LOWREG>(acc[t], f0, f1);
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
      for (int t = 0; t < T; ++t) accy[r3][t] = bias_acc(bias + 2 * H + 32 * r3 + 4 * hh);
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
      for (int t = 0; t < T; ++t) acc[t] = bias_acc(bias + H + 32 * r + 4 * hh);
#pragma unroll
      for (int ks = 0; ks < S2; ++ks) {
        const bf16x8 wf = wr[ks * 64 + lane];
#pragma unroll
        for (int t = 0; t < T; ++t) acc[t] = mfma(wf, h1[ks][t], acc[t]);
        // at most four fragments in flight ahead of their MFMAs
        if (ks % 4 == 3) __builtin_amdgcn_sched_barrier(0);
      }
      infer_block_out<H, T, NB3, true>(acc, r, w3, lane, accy);
      if (more) {
#pragma unroll
        for (int u = 0; u < PER; ++u) w2[((r + 1) & 1) * NBLK + u * NT + tid] = st[u];
      }
      if (!RESIDENT) __syncthreads();
    }
    infer_store<T, NB3>(a, accy, first, hh, col, ok);
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

// The training kernel's B operands in the fragment order of
// v_mfma_f32_16x16x32_bf16: element (row n, k) of a matrix whose K length is
// KD (a multiple of 32) sits at [n / 16][k / 32][16 ((k % 32) / 8) + n % 16]
// [k % 8], so the fragment of output tile n / 16 at K step k / 32 is 64
// lanes x 16 contiguous bytes, one load per wave.
__device__ __forceinline__ size_t frag16_pos(size_t n, size_t k, size_t KD) {
  return (((n >> 4) * (KD >> 5) + (k >> 5)) * 64 + 16 * ((k & 31) >> 3) + (n & 15)) * 8 +
         (k & 7);
}

// Transposed copies for the backward products dH = dZ W: w2t holds W2^T
// (row k, K index o: W2[o][k], K length H), w3t holds W3^T (row k, K index
// c: W3[c][k], K length Cp; c >= C stays zero).
__device__ __forceinline__ void pack_transposed(const MlpShape &sh, size_t p, float v,
                                                __bf16 *w2t, __bf16 *w3t) {
  const size_t H = sh.H, first_w2 = H * sh.F + H, first_w3 = first_w2 + H * H + H;
  if (p >= first_w2 && p < first_w2 + H * H) {
    const size_t q = p - first_w2; // W2[q / H][q % H]
    w2t[frag16_pos(q % H, q / H, H)] = (__bf16)v;
  } else if (p >= first_w3 && p < first_w3 + (size_t)sh.C * H) {
    const size_t q = p - first_w3, Cp = 32 * (((size_t)sh.C + 31) / 32); // W3[q / H][q % H]
    w3t[frag16_pos(q % H, q / H, Cp)] = (__bf16)v;
  }
}

// Copies for the forward products: w1n holds W1 (row o, K index f, K length
// 32: features past F stay zero), w2n holds W2 (K length H), w3n holds W3
// (rows Cp, rows past C stay zero).
__device__ __forceinline__ void pack_natural(const MlpShape &sh, size_t p, float v, __bf16 *w1n,
                                             __bf16 *w2n, __bf16 *w3n) {
  const size_t H = sh.H, F = sh.F, first_w2 = H * F + H, first_w3 = first_w2 + H * H + H;
  if (p < H * F) {
    w1n[frag16_pos(p / F, p % F, 32)] = (__bf16)v;
  } else if (p >= first_w2 && p < first_w2 + H * H) {
    const size_t q = p - first_w2;
    w2n[frag16_pos(q / H, q % H, H)] = (__bf16)v;
  } else if (p >= first_w3 && p < first_w3 + (size_t)sh.C * H) {
    const size_t q = p - first_w3;
    w3n[frag16_pos(q / H, q % H, H)] = (__bf16)v;
  }
}

__device__ __forceinline__ void pack_all(const MlpShape &sh, size_t p, float v, const MlpCopies &cp) {
  pack_one(sh, p, v, cp.w1p, cp.w2p, cp.w3p);
  pack_transposed(sh, p, v, cp.w2t, cp.w3t);
  pack_natural(sh, p, v, cp.w1n, cp.w2n, cp.w3n);
}

__global__ __launch_bounds__(256) void pack_weights(MlpShape sh, const float *__restrict__ theta,
                                                    size_t n, MlpCopies cp) {
  const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  pack_all(sh, p, theta[p], cp);
}

// ------------------------------------------------------------ training step
// One Adam step is two launches.
//  mlp_train_rows: one workgroup per 16 rows of the batch, one wave per
//    16-column output tile of a hidden layer (two for H = 512).
//    Z = A W^T + b on v_mfma_f32_16x16x32_bf16 with the activations as the
//    A operand, read from LDS, and the weights as the B operand, read from
//    bf16 copies in the MFMA's fragment order (frag16_pos: one contiguous
//    1 KB load per wave and K step); the activations pass between layers
//    through LDS.
//    Then the loss terms and dY = scale (Y - T), and the backward chain
//    dZ2 = (dY W3) * gelu'(Z2), dZ1 = (dZ2 W2) * gelu'(Z1) with W3 and W2
//    from their transposed bf16 copies.  Every product of the chain is local
//    to the rows; each wave keeps GELU' of its own tiles in registers from
//    the forward pass.  It stores the operands of the weight gradients
//    transposed (feature-major, the batch contiguous, so the next launch
//    reads them as vector fragments), the column sums of dY, dZ2 and dZ1
//    over its rows, and its sum of squared errors.
//  mlp_grad_tiles: one workgroup per 32 x 32 tile of dW2 = dZ2^T H1,
//    dW1 = dZ1^T X and dW3 = dY^T H2 (the batch as the reduction dimension,
//    split over the waves and added in wave order) and one per 256 biases
//    (block sums in block order; the first also forms the loss); each stores
//    its gradients or applies Adam to its parameters and rewrites their bf16
//    copies.
// Rows past the batch carry X = 0 and dY = 0, so they add nothing.
// Layout of v_mfma_f32_16x16x32_bf16 (checked on the GPU with an in-bounds
// probe): lane l holds A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16]
// for j = 0..7, and D[4 (l / 16) + r][l % 16] for r = 0..3.
constexpr int kGradThreads = 256;

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) __bf16 bf16x4;

__device__ __forceinline__ f32x4 mfma16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 frag_at(const __bf16 *p) {
  return *reinterpret_cast<const bf16x8 *>(p);
}

// One lane's 4 accumulator values (rows 4 kg + r of column col) as bf16:
// into the LDS array (row stride ld; none when lds is null) and transposed
// into dst[col][m0 + 4 kg .. + 3] (row length n_pad), one 8-byte store.
__device__ __forceinline__ void store_act4(const float (&v)[4], __bf16 *lds, int ld, int col,
                                           __bf16 *dst, uint32_t n_pad, uint32_t m0, int kg) {
  bf16x4 b;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    b[r] = (__bf16)v[r];
    if (lds) lds[(4 * kg + r) * ld + col] = b[r];
  }
  *reinterpret_cast<bf16x4 *>(dst + (size_t)col * n_pad + m0 + 4 * kg) = b;
}

// Sum over the 16 rows of a tile column: the lane's 4 values, then the 4
// lane groups; the result is in every lane of the column.
__device__ __forceinline__ float column_sum16(float s) {
  s += __shfl_xor(s, 16);
  s += __shfl_xor(s, 32);
  return s;
}

template <int H> constexpr int train_waves() { return H / 16 < 16 ? H / 16 : 16; }

template <int H, int NB3> struct TrainShape {
  static constexpr int NT = H / 16;                  // 16-column tiles of a hidden layer
  static constexpr int NW = train_waves<H>();        // waves
  static constexpr int TPW = NT / NW;                // tiles per wave
  static constexpr int CP = 32 * NB3, NT3 = CP / 16; // output columns and tiles
  static constexpr int KS = H / 32;                  // K steps of an H-deep product
  // LDS row strides (bf16), padded by 16 bytes so that the 16 rows of a
  // fragment load start in different banks; features padded to 32
  static constexpr int LX = 32 + 8, LH = H + 8, LY = CP + 8;
  static constexpr size_t lds = (size_t)16 * (LX + 2 * LH + LY) * sizeof(__bf16) + 16 * sizeof(float);
};

// Rows of `steps` training steps of n rows each (step s, row r: pair
// batch[s n + r], or pair r without a batch): features digit / 8 as bf16,
// xg[s][n_pad][K1] (zeros past F and for rows n .. n_pad-1), and with
// targets set their targets tg[s][n][C].  One thread per row.
__global__ __launch_bounds__(256) void mlp_gather_rows(const SpaceDev *__restrict__ sp,
                                                       const uint32_t *__restrict__ cfg_raw,
                                                       const int32_t *__restrict__ batch,
                                                       const float *__restrict__ targets,
                                                       uint32_t steps, uint32_t n, uint32_t n_pad,
                                                       int F, int K1, int C, __bf16 *xg,
                                                       float *tg) {
  const uint64_t id = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (id >= (uint64_t)steps * n_pad) return;
  const uint32_t s = (uint32_t)(id / n_pad), r = (uint32_t)(id % n_pad);
  __bf16 *x = xg + id * K1;
  if (r >= n) {
    for (int k = 0; k < K1; ++k) x[k] = (__bf16)0.0f;
    return;
  }
  const uint64_t row = (uint64_t)s * n + r;
  const uint32_t src = batch ? (uint32_t)batch[row] : r;
  uint64_t dlo = 0, dhi = 0;
  decode_packed(cfg_raw[src], sp, dlo, dhi);
  for (int k = 0; k < K1; ++k)
    x[k] = (__bf16)(k < F ? (float)digit_of(dlo, dhi, (uint32_t)k) * 0.125f : 0.0f);
  if (targets)
    for (int c = 0; c < C; ++c) tg[row * C + c] = targets[(size_t)src * C + c];
}

template <int H, int NB3>
__global__ __launch_bounds__(train_waves<H>() * 64) void mlp_train_rows(TrainRowsArgs a) {
  using TS = TrainShape<H, NB3>;
  constexpr int NW = TS::NW, TPW = TS::TPW, CP = TS::CP, NT3 = TS::NT3, KS = TS::KS;
  constexpr int SB = KS < 8 ? KS : 8; // K steps whose weight fragments are loaded together
  constexpr int LX = TS::LX, LH = TS::LH, LY = TS::LY;
  static_assert(NT3 <= NW, "one output tile per wave");
  extern __shared__ __align__(16) unsigned char train_lds[];
  __bf16 *xs = reinterpret_cast<__bf16 *>(train_lds);
  __bf16 *h1s = xs + 16 * LX;
  __bf16 *h2s = h1s + 16 * LH; // H2, then dZ2
  __bf16 *dys = h2s + 16 * LH;
  float *lred = reinterpret_cast<float *>(dys + 16 * LY);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, kg = lane >> 4, r16 = lane & 15;
  const uint32_t blk = blockIdx.x, m0 = 16u * blk;
  const bool train = a.train;

  // the output waves' targets, requested before anything else
  float tv[4];
  if (train && w < NT3) {
    const int col = 16 * w + r16;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t m = m0 + 4 * kg + r;
      tv[r] = (m < a.n && col < a.C) ? a.tin[(size_t)m * a.C + col] : 0.0f;
    }
  }
  // the block's features: 16 gathered rows, padded to 32 with zeros
  if (tid < 64) {
    const int row = tid >> 2, seg = tid & 3;
    const bf16x8 x = 8 * seg < a.K1 ? frag_at(a.xin + (size_t)(m0 + row) * a.K1 + 8 * seg)
                                    : bf16x8{};
    *reinterpret_cast<bf16x8 *>(xs + row * LX + 8 * seg) = x;
  }
  __syncthreads();
  if (tid < 128) { // X^T for dW1: 32 feature rows, zeros past K1
    const int k = tid >> 2, seg = tid & 3;
    bf16x4 b;
#pragma unroll
    for (int e = 0; e < 4; ++e) b[e] = xs[(4 * seg + e) * LX + k];
    *reinterpret_cast<bf16x4 *>(a.xt + (size_t)k * a.n_pad + m0 + 4 * seg) = b;
  }

  f32x4 g1[TPW], g2[TPW]; // GELU'(Z1), GELU'(Z2) of the wave's tiles
  float v[4];
  // acc += the H-deep product of the LDS activations (row stride LH) with
  // output tile t of a weight copy in fragment order (frag16_pos, K length
  // H), SB fragments in flight at a time
  auto tile_frags = [&](const __bf16 *wc, int t, int ks) {
    return wc + ((size_t)t * ks * 64 + lane) * 8;
  };
  auto product = [&](f32x4 acc, const __bf16 *act, const __bf16 *wr) {
#pragma unroll
    for (int s0 = 0; s0 < KS; s0 += SB) {
      bf16x8 bfr[SB];
#pragma unroll
      for (int u = 0; u < SB; ++u) bfr[u] = frag_at(wr + 512 * (s0 + u));
#pragma unroll
      for (int u = 0; u < SB; ++u)
        acc = mfma16(frag_at(act + r16 * LH + 32 * (s0 + u) + 8 * kg), bfr[u], acc);
    }
    return acc;
  };
  // Z1 = X W1^T + b1, H1 = gelu(Z1)
#pragma unroll 1
  for (int q = 0; q < TPW; ++q) {
    const int col = 16 * (w + NW * q) + r16;
    const float bv = a.b1[col];
    f32x4 acc = {bv, bv, bv, bv};
    acc = mfma16(frag_at(xs + r16 * LX + 8 * kg), frag_at(tile_frags(a.w1n, w + NW * q, 1)),
                 acc);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float dg;
      v[r] = gelu_with_grad(acc[r], dg);
      g1[q][r] = dg;
    }
    store_act4(v, h1s, LH, col, a.h1t, a.n_pad, m0, kg);
  }
  __syncthreads();
  // Z2 = H1 W2^T + b2, H2 = gelu(Z2)
#pragma unroll 1
  for (int q = 0; q < TPW; ++q) {
    const int col = 16 * (w + NW * q) + r16;
    const float bv = a.b2[col];
    f32x4 acc = {bv, bv, bv, bv};
    acc = product(acc, h1s, tile_frags(a.w2n, w + NW * q, KS));
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float dg;
      v[r] = gelu_with_grad(acc[r], dg);
      g2[q][r] = dg;
    }
    store_act4(v, h2s, LH, col, a.h2t, a.n_pad, m0, kg);
  }
  __syncthreads();
  // Y = H2 W3^T + b3 on waves 0 .. NT3-1; training: dY, squared errors
  if (w < NT3) {
    const int col = 16 * w + r16;
    const float bv = col < a.C ? a.b3[col] : 0.0f;
    f32x4 acc = {bv, bv, bv, bv};
    acc = product(acc, h2s, tile_frags(a.w3n, w, KS));
    if (!train) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t m = m0 + 4 * kg + r;
        if (m < a.n) a.yout[(size_t)m * CP + col] = acc[r];
      }
    } else {
      float sq = 0.0f, ds = 0.0f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t m = m0 + 4 * kg + r;
        const float d = (m < a.n && col < a.C) ? acc[r] - tv[r] : 0.0f;
        sq += d * d;
        v[r] = a.scale * d;
        ds += v[r];
      }
      store_act4(v, dys, LY, col, a.dyt, a.n_pad, m0, kg);
      ds = column_sum16(ds);
      if (kg == 0) a.bp3[(size_t)blk * CP + col] = ds;
      sq = wave_sum(sq);
      if (lane == 0) lred[w] = sq;
    }
  }
  if (!train) return; // uniform over the workgroup
  __syncthreads();
  if (tid == 0) {
    float t = lred[0];
#pragma unroll
    for (int i = 1; i < NT3; ++i) t += lred[i];
    a.lossp[blk] = t;
  }
  // dZ2 = (dY W3) * gelu'(Z2), into the H2 array
#pragma unroll 1
  for (int q = 0; q < TPW; ++q) {
    const int col = 16 * (w + NW * q) + r16;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8 w3f[CP / 32];
#pragma unroll
    for (int s = 0; s < CP / 32; ++s) w3f[s] = frag_at(tile_frags(a.w3t, w + NW * q, CP / 32) + 512 * s);
#pragma unroll
    for (int s = 0; s < CP / 32; ++s)
      acc = mfma16(frag_at(dys + r16 * LY + 32 * s + 8 * kg), w3f[s], acc);
    float bs = 0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      v[r] = acc[r] * g2[q][r];
      bs += v[r];
    }
    store_act4(v, h2s, LH, col, a.dz2t, a.n_pad, m0, kg);
    bs = column_sum16(bs);
    if (kg == 0) a.bp2[(size_t)blk * H + col] = bs;
  }
  __syncthreads();
  // dZ1 = (dZ2 W2) * gelu'(Z1)
#pragma unroll 1
  for (int q = 0; q < TPW; ++q) {
    const int col = 16 * (w + NW * q) + r16;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    acc = product(acc, h2s, tile_frags(a.w2t, w + NW * q, KS));
    float bs = 0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      v[r] = acc[r] * g1[q][r];
      bs += v[r];
    }
    store_act4(v, nullptr, 0, col, a.dz1t, a.n_pad, m0, kg);
    bs = column_sum16(bs);
    if (kg == 0) a.bp1[(size_t)blk * H + col] = bs;
  }
}

// Gradient g of master parameter p: stored (gradient mode), or one Adam step
// (Kingma & Ba, Algorithm 1; c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t))
// followed by the bf16 copies of the new value.
// The bf16 copies of weight (o, k) of layer `kind` (1: W1[o][k], k < F;
// 2: W2[o][k]; 3: W3[o][k], o < C) in every layout pack_all writes, with the
// row and column known: the same positions, no divisions.
__device__ __forceinline__ void pack_weight(const MlpShape &sh, int kind, int o, int k, float v,
                                            const MlpCopies &cp) {
  const __bf16 b = (__bf16)v;
  const int H = sh.H;
  if (kind == 1) {
    const int S1 = sh.K1 / 16;
    const int lane = 32 * ((k & 15) >> 3) + (o & 31);
    cp.w1p[(((size_t)(o >> 5) * S1 + (k >> 4)) * 64 + lane) * 8 + (k & 7)] = b;
    cp.w1n[frag16_pos(o, k, 32)] = b;
    return;
  }
  const int rem = k & 15;
  const int lane = 32 * ((rem & 7) >> 2) + (o & 31), j = 4 * (rem >> 3) + (rem & 3);
  const size_t pp =
      (((size_t)(o >> 5) * (H / 16) + 2 * (k >> 5) + ((k & 31) >> 4)) * 64 + lane) * 8 + j;
  if (kind == 2) {
    cp.w2p[pp] = b;
    cp.w2t[frag16_pos(k, o, H)] = b;
    cp.w2n[frag16_pos(o, k, H)] = b;
  } else {
    cp.w3p[pp] = b;
    cp.w3t[frag16_pos(k, o, 32 * (((size_t)sh.C + 31) / 32))] = b;
    cp.w3n[frag16_pos(o, k, H)] = b;
  }
}

// Adam on parameter p (or its gradient stored, in gradient mode); a weight
// (kind 1..3 at row o, column k) also rewrites its bf16 copies.
__device__ __forceinline__ void apply_grad(const GradTilesArgs &g, size_t p, float gv, int kind,
                                           int o, int k) {
  if (g.grad) {
    g.grad[p] = gv;
    return;
  }
  const float mm = g.beta1 * g.m[p] + (1.0f - g.beta1) * gv;
  const float vv = g.beta2 * g.v[p] + (1.0f - g.beta2) * gv * gv;
  g.m[p] = mm;
  g.v[p] = vv;
  const float th = g.theta[p] - g.lr * (mm * g.c1) / (sqrtf(vv * g.c2) + g.eps);
  g.theta[p] = th;
  if (kind) pack_weight(g.sh, kind, o, k, th, g.cp);
}

__global__ __launch_bounds__(kGradThreads) void mlp_grad_tiles(GradTilesArgs g) {
  constexpr int NW = kGradThreads / 64;
  __shared__ float part[NW][16][64];
  const int H = g.sh.H, F = g.sh.F, C = g.sh.C, NT = H / 32, NB3 = (C + 31) / 32;
  const size_t off_b1 = (size_t)H * F, off_w2 = off_b1 + H, off_b2 = off_w2 + (size_t)H * H;
  const size_t off_w3 = off_b2 + H, off_b3 = off_w3 + (size_t)C * H;
  const int T2 = NT * NT, T1 = NT, T3 = NB3 * NT;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, hh = lane >> 5, c = lane & 31;
  int j = blockIdx.x;
  if (j >= T2 + T1 + T3) { // biases, one per thread: the row blocks' column sums in block order
    const int Cp = 32 * NB3, nblk = (int)(g.n_pad / 16); // the row kernel's blocks
    const int first = j - (T2 + T1 + T3);
    const int idx = first * kGradThreads + tid;
    if (idx < 2 * H + C) {
      const float *src;
      int ld, col;
      size_t p;
      if (idx < H) {
        src = g.bp1, ld = H, col = idx, p = off_b1 + col;
      } else if (idx < 2 * H) {
        src = g.bp2, ld = H, col = idx - H, p = off_b2 + col;
      } else {
        src = g.bp3, ld = Cp, col = idx - 2 * H, p = off_b3 + col;
      }
      float s = 0.0f;
#pragma unroll 8
      for (int b = 0; b < nblk; ++b) s += src[(size_t)b * ld + col];
      apply_grad(g, p, s, 0, 0, 0); // biases have no bf16 copies
    }
    if (first == 0 && tid == 0 && g.loss_out) {
      float t = 0.0f;
#pragma unroll 8
      for (int b = 0; b < nblk; ++b) t += g.lossp[b];
      *g.loss_out = t / g.loss_div;
    }
    return;
  }
  // tile: rows r0.. of the A operand (dZ^T), rows c0.. of the B operand
  const __bf16 *A, *B;
  int kind, r0, c0;
  if (j < T2) {
    kind = 2, r0 = 32 * (j / NT), c0 = 32 * (j % NT), A = g.dz2t, B = g.h1t;
  } else if ((j -= T2) < T1) {
    kind = 1, r0 = 32 * j, c0 = 0, A = g.dz1t, B = g.xt;
  } else {
    j -= T1;
    kind = 3, r0 = 32 * (j / NT), c0 = 32 * (j % NT), A = g.dyt, B = g.h2t;
  }
  const __bf16 *pa = A + (size_t)(r0 + c) * g.n_pad + 8 * hh;
  const __bf16 *pb = B + (size_t)(c0 + c) * g.n_pad + 8 * hh;
  f32x16 acc = {};
  constexpr int KB = 4; // K steps of a wave whose fragments are loaded together
  for (uint32_t k0 = 16 * w; k0 < g.n_pad; k0 += KB * 16 * NW) {
    bf16x8 fa[KB], fb[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const uint32_t k = k0 + u * 16 * NW;
      fa[u] = k < g.n_pad ? frag_at(pa + k) : bf16x8{};
      fb[u] = k < g.n_pad ? frag_at(pb + k) : bf16x8{};
    }
#pragma unroll
    for (int u = 0; u < KB; ++u) acc = mfma(fa[u], fb[u], acc);
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) part[w][i][lane] = acc[i];
  __syncthreads();
  // wave w finishes rows 8 w + 4 hh + e (registers 4 w + e) of the tile
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int i = 4 * w + e;
    float gv = part[0][i][lane];
#pragma unroll
    for (int q = 1; q < NW; ++q) gv += part[q][i][lane];
    const int row = r0 + 8 * w + 4 * hh + e, col = c0 + c;
    if (kind == 2) apply_grad(g, off_w2 + (size_t)row * H + col, gv, 2, row, col);
    else if (kind == 1 && col < F) apply_grad(g, (size_t)row * F + col, gv, 1, row, col);
    else if (kind == 3 && row < C) apply_grad(g, off_w3 + (size_t)row * H + col, gv, 3, row, col);
  }
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

template <int H, int NB3, int S1>
hipError_t launch_fwd_h(const MlpFwdArgs &a, bool train, hipStream_t stream) {
  // the training forward is part of launch_mlp_train_rows
  if (train) return hipErrorInvalidValue;
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

namespace {

template <int H, int NB3>
hipError_t launch_train_rows_h(const TrainRowsArgs &a, hipStream_t stream) {
  using TS = TrainShape<H, NB3>;
  static_assert(TS::lds <= 64 * 1024, "static launch size");
  hipLaunchKernelGGL((mlp_train_rows<H, NB3>), dim3(a.n_pad / 16), dim3(TS::NW * 64), TS::lds,
                     stream, a);
  return hipGetLastError();
}

template <int H> hipError_t launch_train_rows_nb(const TrainRowsArgs &a, hipStream_t s) {
  const int nb3 = (a.C + 31) / 32;
  if (nb3 == 1) return launch_train_rows_h<H, 1>(a, s);
  if (nb3 == 2) return launch_train_rows_h<H, 2>(a, s);
  return hipErrorInvalidValue;
}

} // namespace

hipError_t launch_mlp_train_rows(const TrainRowsArgs &a, hipStream_t stream) {
  if (a.n == 0) return hipSuccess;
  if (a.n_pad % 32 != 0 || a.n_pad < a.n) return hipErrorInvalidValue;
  switch (a.H) {
  case 64: return launch_train_rows_nb<64>(a, stream);
  case 128: return launch_train_rows_nb<128>(a, stream);
  case 256: return launch_train_rows_nb<256>(a, stream);
  case 512: return launch_train_rows_nb<512>(a, stream);
  default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mlp_gather_rows(const SpaceDev *sp, const uint32_t *cfg_raw,
                                  const int32_t *batch, const float *targets, uint32_t steps,
                                  uint32_t n, uint32_t n_pad, int F, int K1, int C, __bf16 *xg,
                                  float *tg, hipStream_t stream) {
  const uint64_t threads = (uint64_t)steps * n_pad;
  if (threads == 0) return hipSuccess;
  if (n_pad < n || (K1 != 16 && K1 != 32)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(mlp_gather_rows, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0,
                     stream, sp, cfg_raw, batch, targets, steps, n, n_pad, F, K1, C, xg, tg);
  return hipGetLastError();
}

hipError_t launch_mlp_grad_tiles(const GradTilesArgs &g, hipStream_t stream) {
  const int NT = g.sh.H / 32, NB3 = (g.sh.C + 31) / 32;
  if (g.n_pad == 0 || g.n_pad % 32 != 0 || NB3 < 1 || NB3 > 2 || g.sh.K1 > 32)
    return hipErrorInvalidValue;
  const int blocks = NT * NT + NT + NB3 * NT + (2 * g.sh.H + g.sh.C + kGradThreads - 1) / kGradThreads;
  hipLaunchKernelGGL(mlp_grad_tiles, dim3(blocks), dim3(kGradThreads), 0, stream, g);
  return hipGetLastError();
}

hipError_t launch_pack_weights(const MlpShape &sh, const float *theta, size_t n,
                               const MlpCopies &cp, hipStream_t stream) {
  hipLaunchKernelGGL(pack_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, sh,
                     theta, n, cp);
  return hipGetLastError();
}

} // namespace cgs
