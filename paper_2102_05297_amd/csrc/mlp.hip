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
// backward pass's GELU derivative uses erf from Abramowitz & Stegun 7.1.26
// (|error| <= 1.5e-7).
//
// Training runs the forward pass as one GEMM per layer (gemm_bf16 with the
// bias and GELU in its epilogue, 32 x 32 output tiles, so a batch of a few
// hundred configurations still spreads over tens of workgroups) and the
// backward pass with the same GEMM kernel.
#include <algorithm>

#include "device_common.h"
#include "gelu.h"
#include "models.h"

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
// GELU(z) = max(z, 0) - |z| Phi(-|z|) with Phi(-x) = 2^p(min(x, 9)) (gelu.h):
// nine VALU operations and one exponential.
__device__ __forceinline__ float gelu(float z) {
  const float az = fabsf(z);
  const float e = __builtin_amdgcn_exp2f(gelu_tail_log2(fminf(az, kGeluTailMax)));
  return fmaf(-az, e, fmaxf(z, 0.0f));
}
__device__ __forceinline__ float gelu_grad(float z) {
  float c, p;
  normal_cdf_pdf(z, c, p);
  return c + z * p;
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

// ------------------------------------------------------------------ GEMM
// C[M][N] = sum_k A(m, k) B(k, n), bf16 operands (converted on load), fp32
// accumulation; one 32x32 output tile per workgroup, its K range split over
// the workgroup's waves (kGemmThreads / 64), partial tiles summed in LDS.
// Operands are addressed with arbitrary strides so transposed products need
// no copies.
template <typename T> __device__ __forceinline__ __bf16 to_bf16(T v);
template <> __device__ __forceinline__ __bf16 to_bf16<float>(float v) { return (__bf16)v; }
template <> __device__ __forceinline__ __bf16 to_bf16<__bf16>(__bf16 v) { return v; }
// 8 consecutive values (16-byte aligned for bf16, 32-byte for float) as bf16.
__device__ __forceinline__ bf16x8 load_bf16x8(const __bf16 *p) {
  return *reinterpret_cast<const bf16x8 *>(p);
}
__device__ __forceinline__ bf16x8 load_bf16x8(const float *p) {
  const float4 lo = *reinterpret_cast<const float4 *>(p);
  const float4 hi = *reinterpret_cast<const float4 *>(p + 4);
  bf16x8 r;
  r[0] = (__bf16)lo.x;
  r[1] = (__bf16)lo.y;
  r[2] = (__bf16)lo.z;
  r[3] = (__bf16)lo.w;
  r[4] = (__bf16)hi.x;
  r[5] = (__bf16)hi.y;
  r[6] = (__bf16)hi.z;
  r[7] = (__bf16)hi.w;
  return r;
}

// EPI 0: C = A B; 1: dZ = (A B) * gelu'(Z) (fp32 and bf16); 2: Z = A B + bias
// (fp32) and H = gelu(Z) (bf16); 3: Y = A B + bias (fp32); 4: as 3, plus the
// training loss terms of LossArgs (dY and one sum of squared errors per
// tile).  bias[N] for 2, 3, 4.
// Output tile `tile` (row-major over 32 x 32 tiles) by one workgroup of
// kGemmThreads; shared by the plain launch and the grouped backward launch.
// The first layer's A operand straight from the configurations: row m is
// configuration cfg_raw[batch[m]] (cfg_raw[m] without a batch), column k its
// parameter k's digit / 8 (0 past F); the workgroups of the first column of
// output tiles also store the rows as bf16 into xout[m][K1] for the
// backward pass.
struct FeatArgs {
  const SpaceDev *sp;
  const uint32_t *cfg_raw;
  const int32_t *batch;
  int F, K1;
  __bf16 *xout;
};

template <typename TA, typename TB, int EPI, bool FEAT = false>
__device__ __forceinline__ void gemm_tile(const GemmArgs &g, const float *bias, const LossArgs &la,
                                          int tile, const FeatArgs &fa = FeatArgs{}) {
  constexpr int NW = kGemmThreads / 64;
  __shared__ float part[NW - 1][16][64];
  const TA *A = static_cast<const TA *>(g.A);
  const TB *B = static_cast<const TB *>(g.B);
  const int tiles_n = (g.N + 31) / 32;
  const int m0 = (tile / tiles_n) * 32, n0 = (tile % tiles_n) * 32;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, hh = lane >> 5, c = lane & 31;
  const int m = m0 + c, n = n0 + c;
  f32x16 acc = {};
  // unit stride along K (and 8-element aligned rows): a fragment's 8 values
  // are one contiguous, 16-byte aligned run, loaded as vectors
  const bool a_vec =
      g.a_sk == 1 && g.a_sm % 8 == 0 && (reinterpret_cast<uintptr_t>(A) & 15u) == 0;
  const bool b_vec =
      g.b_sk == 1 && g.b_sn % 8 == 0 && (reinterpret_cast<uintptr_t>(B) & 15u) == 0;
  uint64_t dlo = 0, dhi = 0; // FEAT: the digits of row m's configuration
  if (FEAT && m < g.M && 16 * w < g.K) {
    const uint32_t src = fa.batch ? (uint32_t)fa.batch[m] : (uint32_t)m;
    decode_packed(fa.cfg_raw[src], fa.sp, dlo, dhi);
  }
  for (int k0 = 16 * w; k0 < g.K; k0 += 16 * NW) {
    bf16x8 af, bf;
    const int kf = k0 + 8 * hh; // first k of this lane's fragment
    const bool full = kf + 8 <= g.K;
    if (FEAT) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = kf + j;
        af[j] = (__bf16)((m < g.M && k < fa.F) ? (float)digit_of(dlo, dhi, (uint32_t)k) * 0.125f
                                               : 0.0f);
      }
      if (n0 == 0 && m < g.M && kf < fa.K1)
        *reinterpret_cast<bf16x8 *>(fa.xout + (size_t)m * fa.K1 + kf) = af;
    } else if (a_vec && full && m < g.M) {
      af = load_bf16x8(A + (size_t)m * g.a_sm + kf);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = kf + j;
        af[j] = (m < g.M && k < g.K) ? to_bf16(A[(size_t)m * g.a_sm + (size_t)k * g.a_sk])
                                     : (__bf16)0.0f;
      }
    }
    if (b_vec && full && n < g.N) {
      bf = load_bf16x8(B + (size_t)n * g.b_sn + kf);
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = kf + j;
        bf[j] = (n < g.N && k < g.K) ? to_bf16(B[(size_t)k * g.b_sk + (size_t)n * g.b_sn])
                                     : (__bf16)0.0f;
      }
    }
    acc = mfma(af, bf, acc);
  }
  if (w > 0) {
#pragma unroll
    for (int i = 0; i < 16; ++i) part[w - 1][i][lane] = acc[i];
  }
  __syncthreads();
  if (w != 0) return;
  float sq = 0.0f; // EPI 4: this lane's squared errors
  float tv[16];    // EPI 4: the targets of this lane's 16 outputs
  if (EPI == 4) {
    // every target load issued before the first dY store (the stores could
    // alias them); rows and columns past the end read row 0, column 0
    int src[16];
    const int cl = n0 + c < g.N ? n0 + c : 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = m0 + 8 * (i / 4) + 4 * hh + (i % 4);
      const int r = row < g.M ? row : 0;
      src[i] = la.batch ? la.batch[r] : r;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) tv[i] = la.targets[(size_t)src[i] * g.N + cl];
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
#pragma unroll
    for (int q = 0; q < NW - 1; ++q) acc[i] += part[q][i][lane];
    const int row = m0 + 8 * (i / 4) + 4 * hh + (i % 4), cl = n0 + c;
    if (row >= g.M || cl >= g.N) continue;
    const size_t o = (size_t)row * g.ldc + cl;
    if (EPI == 0) {
      g.Cf[o] = acc[i];
    } else if (EPI == 1) { // dZ = dH * gelu'(Z)
      const float v = acc[i] * gelu_grad(g.Z[o]);
      g.Cf[o] = v;
      g.Cb[o] = (__bf16)v;
    } else if (EPI == 2) { // Z = W x + b, H = gelu(Z)
      const float v = acc[i] + bias[cl];
      g.Cf[o] = v;
      g.Cb[o] = (__bf16)gelu(v);
    } else if (EPI == 3) { // Y = W h + b
      g.Cf[o] = acc[i] + bias[cl];
    } else { // Y, then d = Y - T and dY = scale * d
      const float y = acc[i] + bias[cl];
      g.Cf[o] = y;
      const float d = y - tv[i];
      sq += d * d;
      la.dyf[o] = la.scale * d;
      la.dyb[o] = (__bf16)(la.scale * d);
    }
  }
  if (EPI == 4) {
    sq = wave_sum(sq);
    if (lane == 0) la.partial[tile] = sq;
  }
}

template <typename TA, typename TB, int EPI>
__global__ __launch_bounds__(kGemmThreads) void gemm_bf16(GemmArgs g, const float *bias,
                                                          LossArgs la) {
  gemm_tile<TA, TB, EPI>(g, bias, la, blockIdx.x);
}

// The first hidden layer with its inputs decoded in the operand load
// (FeatArgs): Z1 = X W1^T + b1, H1 = gelu(Z1), X stored on the side.
__global__ __launch_bounds__(kGemmThreads) void gemm_layer1(GemmArgs g, const float *bias,
                                                            FeatArgs fa) {
  gemm_tile<__bf16, float, 2, true>(g, bias, LossArgs{}, blockIdx.x, fa);
}

// Column sums of src[nrows][ld] over columns [64 b, 64 b + 64) of ncols by
// one workgroup: lanes take columns (coalesced rows), the waves split the
// rows and meet in LDS, added in wave order.  Block 0 also forms the loss
// from the per-tile partials, in tile order.
__device__ __forceinline__ void colsum_block(const ColSumJob &cs, int b) {
  constexpr int NW = kGemmThreads / 64;
  __shared__ float part[NW][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (b == 0 && threadIdx.x == 0 && cs.loss_out) {
    float t = 0.0f;
    for (int k = 0; k < cs.n_partial; ++k) t += cs.partial[k];
    *cs.loss_out = t / cs.loss_div;
  }
  const int col = b * 64 + lane;
  float sum = 0.0f;
  if (col < cs.ncols) {
#pragma unroll 4
    for (int r = w; r < cs.nrows; r += NW) sum += cs.src[(size_t)r * cs.ld + col];
  }
  part[w][lane] = sum;
  __syncthreads();
  if (w == 0 && col < cs.ncols) {
    float t = 0.0f;
#pragma unroll
    for (int k = 0; k < NW; ++k) t += part[k][lane];
    cs.dst[col] = t;
  }
}

__device__ __forceinline__ int gemm_tiles(const GemmArgs &g) {
  return g.M > 0 && g.N > 0 ? ((g.M + 31) / 32) * ((g.N + 31) / 32) : 0;
}

// One level of the backward pass in one launch: two independent bf16 x bf16
// products (epilogue 0: plain, 1: times gelu'(Z)) and one set of bias
// gradients, each workgroup working on one of them.
__global__ __launch_bounds__(kGemmThreads) void gemm_bwd_group(GemmArgs g0, int epi0, GemmArgs g1,
                                                               int epi1, ColSumJob cs) {
  int b = blockIdx.x;
  const int t0 = gemm_tiles(g0), t1 = gemm_tiles(g1);
  if (b < t0) {
    if (epi0) gemm_tile<__bf16, __bf16, 1>(g0, nullptr, LossArgs{}, b);
    else gemm_tile<__bf16, __bf16, 0>(g0, nullptr, LossArgs{}, b);
    return;
  }
  b -= t0;
  if (b < t1) {
    if (epi1) gemm_tile<__bf16, __bf16, 1>(g1, nullptr, LossArgs{}, b);
    else gemm_tile<__bf16, __bf16, 0>(g1, nullptr, LossArgs{}, b);
    return;
  }
  colsum_block(cs, b - t1);
}

// ------------------------------------------------------ loss, biases, Adam
// (dY and the squared errors come from the output layer's GEMM epilogue.)

// Bias gradients: column sums over the batch.  A workgroup takes 64
// consecutive columns (lane = column, coalesced rows); its 16 waves split the
// rows and their partial sums meet in LDS.
constexpr int kBiasWaves = 16;
__global__ __launch_bounds__(kBiasWaves * 64) void bias_grads(
    const float *__restrict__ dz1, const float *__restrict__ dz2, const float *__restrict__ dyf,
    int n, int H, int C, int Cp, float *__restrict__ gb1, float *__restrict__ gb2,
    float *__restrict__ gb3, const float *__restrict__ partial, int n_partial,
    float *__restrict__ loss_out) {
  __shared__ float part[kBiasWaves][64];
  if (blockIdx.x == 0 && threadIdx.x == 0) { // the loss, tile partials in order
    float t = 0.0f;
    for (int k = 0; k < n_partial; ++k) t += partial[k];
    *loss_out = t / (float)(n * C);
  }
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

// Transposed bf16 copies of W2 and W3, K-contiguous for the backward
// products dH = dZ W (so their weight fragments are vector loads):
// w2t[k][o] = W2[o][k] (row length H), w3t[k][c] = W3[c][k] (row length Cp,
// the padding never read).
__device__ __forceinline__ void pack_transposed(const MlpShape &sh, size_t p, float v,
                                                __bf16 *w2t, __bf16 *w3t) {
  const size_t H = sh.H, first_w2 = H * sh.F + H, first_w3 = first_w2 + H * H + H;
  if (p >= first_w2 && p < first_w2 + H * H) {
    const size_t q = p - first_w2;
    w2t[(q % H) * H + q / H] = (__bf16)v;
  } else if (p >= first_w3 && p < first_w3 + (size_t)sh.C * H) {
    const size_t q = p - first_w3, Cp = 32 * (((size_t)sh.C + 31) / 32);
    w3t[(q % H) * Cp + q / H] = (__bf16)v;
  }
}

__global__ __launch_bounds__(256) void pack_weights(MlpShape sh, const float *__restrict__ theta,
                                                    size_t n, __bf16 *w1p, __bf16 *w2p,
                                                    __bf16 *w3p, __bf16 *w2t, __bf16 *w3t) {
  const size_t p = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  const float th = theta[p];
  pack_one(sh, p, th, w1p, w2p, w3p);
  pack_transposed(sh, p, th, w2t, w3t);
}

// Adam (Kingma & Ba, Algorithm 1); c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t).
__global__ __launch_bounds__(256) void adam_pack(MlpShape sh, float *__restrict__ theta,
                                                 float *__restrict__ m, float *__restrict__ v,
                                                 const float *__restrict__ grad, size_t n,
                                                 float lr, float b1, float b2, float eps, float c1,
                                                 float c2, __bf16 *w1p, __bf16 *w2p,
                                                 __bf16 *w3p, __bf16 *w2t, __bf16 *w3t) {
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
  pack_transposed(sh, p, th, w2t, w3t);
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
  // the training forward is launch_mlp_train_forward (one GEMM per layer)
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

hipError_t launch_mlp_train_forward(const MlpFwdArgs &a, const float *w1, const float *w2,
                                   const float *w3, const LossArgs *loss, hipStream_t stream) {
  if (a.n == 0) return hipSuccess;
  const int Cp = 32 * ((a.C + 31) / 32);
  auto gemm = [&](const GemmArgs &g, const float *bias, int epi) {
    const dim3 grid(((g.M + 31) / 32) * ((g.N + 31) / 32)), block(kGemmThreads);
    if (epi == 2)
      hipLaunchKernelGGL((gemm_bf16<__bf16, float, 2>), grid, block, 0, stream, g, bias,
                         LossArgs{});
    else if (loss == nullptr)
      hipLaunchKernelGGL((gemm_bf16<__bf16, float, 3>), grid, block, 0, stream, g, bias,
                         LossArgs{});
    else
      hipLaunchKernelGGL((gemm_bf16<__bf16, float, 4>), grid, block, 0, stream, g, bias, *loss);
  };
  // Z1 = X W1^T + b1, H1 = gelu(Z1); Z2 = H1 W2^T + b2, H2 = gelu(Z2); Y = H2 W3^T + b3
  const int n = (int)a.n;
  {
    // layer 1 decodes its inputs (the digits of the batch's configurations)
    // in the operand load and stores them as X for the backward pass
    const GemmArgs g1{n, a.H, a.F, nullptr, a.K1, 1, w1, 1, a.F, a.z1out, a.h1out, nullptr, a.H};
    const dim3 grid(((g1.M + 31) / 32) * ((g1.N + 31) / 32)), block(kGemmThreads);
    hipLaunchKernelGGL(gemm_layer1, grid, block, 0, stream, g1, a.b1,
                       FeatArgs{a.sp, a.cfg_raw, a.batch, a.F, a.K1, a.xout});
  }
  gemm(GemmArgs{n, a.H, a.H, a.h1out, a.H, 1, w2, 1, a.H, a.z2out, a.h2out, nullptr, a.H}, a.b2,
       2);
  gemm(GemmArgs{n, a.C, a.H, a.h2out, a.H, 1, w3, 1, a.H, a.yout, nullptr, nullptr, Cp}, a.b3, 3);
  return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs &g, int a_bf16, int b_bf16, int epi, hipStream_t stream) {
  const int tiles = ((g.M + 31) / 32) * ((g.N + 31) / 32);
  if (tiles == 0) return hipSuccess;
  const dim3 grid(tiles), block(kGemmThreads);
#define GEMM_CASE(TA, TB, E)                                                                   \
  hipLaunchKernelGGL((gemm_bf16<TA, TB, E>), grid, block, 0, stream, g, nullptr, LossArgs{})
  if (a_bf16 && b_bf16 && epi == 0) GEMM_CASE(__bf16, __bf16, 0);
  else if (a_bf16 && !b_bf16 && epi == 1) GEMM_CASE(__bf16, float, 1);
  else if (a_bf16 && !b_bf16 && epi == 0) GEMM_CASE(__bf16, float, 0);
  else if (a_bf16 && b_bf16 && epi == 1) GEMM_CASE(__bf16, __bf16, 1);
  else return hipErrorInvalidValue;
#undef GEMM_CASE
  return hipGetLastError();
}

hipError_t launch_bwd_group(const GemmArgs &g0, int epi0, const GemmArgs &g1, int epi1,
                            const ColSumJob &cs, hipStream_t stream) {
  auto tiles = [](const GemmArgs &g) {
    return g.M > 0 && g.N > 0 ? ((g.M + 31) / 32) * ((g.N + 31) / 32) : 0;
  };
  const int blocks = tiles(g0) + tiles(g1) + (cs.ncols + 63) / 64;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(gemm_bwd_group, dim3(blocks), dim3(kGemmThreads), 0, stream, g0, epi0, g1,
                     epi1, cs);
  return hipGetLastError();
}

hipError_t launch_bias_grads(const float *dz1, const float *dz2, const float *dyf, int n, int H,
                             int C, int Cp, float *gb1, float *gb2, float *gb3,
                             const float *partial, int n_partial, float *loss_out,
                             hipStream_t stream) {
  const int total = 2 * H + C;
  hipLaunchKernelGGL(bias_grads, dim3((total + 63) / 64), dim3(kBiasWaves * 64), 0, stream, dz1,
                     dz2, dyf, n, H, C, Cp, gb1, gb2, gb3, partial, n_partial, loss_out);
  return hipGetLastError();
}

hipError_t launch_pack_weights(const MlpShape &sh, const float *theta, size_t n, __bf16 *w1p,
                               __bf16 *w2p, __bf16 *w3p, __bf16 *w2t, __bf16 *w3t,
                               hipStream_t stream) {
  hipLaunchKernelGGL(pack_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, sh,
                     theta, n, w1p, w2p, w3p, w2t, w3t);
  return hipGetLastError();
}

hipError_t launch_adam_pack(const MlpShape &sh, float *theta, float *m, float *v,
                            const float *grad, size_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2, __bf16 *w1p, __bf16 *w2p, __bf16 *w3p,
                            __bf16 *w2t, __bf16 *w3t, hipStream_t stream) {
  hipLaunchKernelGGL(adam_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, sh, theta,
                     m, v, grad, n, lr, b1, b2, eps, c1, c2, w1p, w2p, w3p, w2t, w3t);
  return hipGetLastError();
}

} // namespace cgs
