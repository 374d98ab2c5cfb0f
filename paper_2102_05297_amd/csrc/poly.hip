// Least-squares polynomial counter models per binary subspace (Sect. 3.4.1).
//
// The binary parameters' digits select a subspace; within it every counter is
// a polynomial in the non-binary parameters: products of their features over
// all parameter sets up to the chosen order (main effects and interactions),
// plus squares.  Feature x_j = (2 v - v_max - v_min) / (v_max - v_min).
//
// Fit: F[i][t] (float64) for every measured point and basis term, with the
// point's counters appended as columns T..T+C-1; per subspace the Gram matrix
// of those columns gives F^T F and F^T Y; a ridge 1e-9 trace / T is added and
// one workgroup per subspace factors it (Cholesky, packed lower triangle in
// LDS) and solves for every counter.  Evaluation: one thread per valid
// configuration, float32, coefficients of a group of subspaces in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "device_common.h"
#include "models.h"

namespace cgs {

namespace {

constexpr int kPolyThreads = 256;
constexpr int kGB = 32;        // Gram block edge
constexpr int kGramChunk = 128; // points staged per round of the Gram kernel
constexpr int kEvalThreads = 1024; // one workgroup per CU holds the coefficients
constexpr double kRidge = 1e-9;

__device__ __forceinline__ uint32_t term_count(uint32_t d) { return d & 7u; }
__device__ __forceinline__ uint32_t term_var(uint32_t d, uint32_t i) {
  return (d >> (3 + 5 * i)) & 31u;
}

__device__ __forceinline__ uint32_t subspace_of(const PolyDev *pd, uint64_t lo, uint64_t hi) {
  uint32_t s = 0;
  for (int i = 0; i < pd->B; ++i) s |= digit_of(lo, hi, pd->bin_params[i]) << i;
  return s;
}

// Exclusive prefix sums of in[0..n) in one workgroup.
__global__ __launch_bounds__(1024) void poly_excl_scan(const uint64_t *__restrict__ in,
                                                       uint64_t *__restrict__ out, uint32_t n) {
  __shared__ uint64_t scratch[16];
  const uint32_t t = threadIdx.x, per = (n + 1023) / 1024;
  const uint32_t a = min(n, t * per), b = min(n, a + per);
  uint64_t mine = 0;
  for (uint32_t i = a; i < b; ++i) mine += in[i];
  uint64_t tot;
  uint64_t run = block_excl_scan<1024>(mine, scratch, tot);
  for (uint32_t i = a; i < b; ++i) {
    const uint64_t v = in[i];
    out[i] = run;
    run += v;
  }
}

// ---------------------------------------------------------------- design
__device__ __forceinline__ bool in_design(const SpaceDev *sp, const uint32_t *allowed,
                                          uint32_t raw) {
  uint64_t lo, hi;
  decode_packed(raw, sp, lo, hi);
  bool ok = true;
  for (int j = 0; j < sp->n_params; ++j) ok = ok && ((allowed[j] >> digit_of(lo, hi, j)) & 1u);
  return ok;
}

__global__ __launch_bounds__(kPolyThreads) void poly_design_count(
    const SpaceDev *__restrict__ sp, const uint32_t *__restrict__ idx, uint32_t nv,
    const uint32_t *__restrict__ allowed, uint64_t *__restrict__ cnt) {
  __shared__ uint64_t scratch[kPolyThreads / 64];
  for (uint32_t tile = blockIdx.x; (uint64_t)tile * kPolyThreads < nv; tile += gridDim.x) {
    const uint32_t l = tile * kPolyThreads + threadIdx.x;
    const uint64_t f = (l < nv && in_design(sp, allowed, idx[l])) ? 1ull : 0ull;
    const uint64_t s = block_sum<kPolyThreads>(f, scratch);
    if (threadIdx.x == 0) cnt[tile] = s;
  }
}

__global__ __launch_bounds__(kPolyThreads) void poly_design_write(
    const SpaceDev *__restrict__ sp, const uint32_t *__restrict__ idx, uint32_t nv,
    const uint32_t *__restrict__ allowed, const uint64_t *__restrict__ off,
    uint32_t *__restrict__ out) {
  __shared__ uint64_t scratch[kPolyThreads / 64];
  for (uint32_t tile = blockIdx.x; (uint64_t)tile * kPolyThreads < nv; tile += gridDim.x) {
    const uint32_t l = tile * kPolyThreads + threadIdx.x;
    const bool f = l < nv && in_design(sp, allowed, idx[l]);
    uint64_t tot;
    const uint64_t r = block_excl_scan<kPolyThreads>(f ? 1ull : 0ull, scratch, tot);
    if (f) out[off[tile] + r] = l;
  }
}

// ---------------------------------------------------------------- fit
// F[i][t]: basis term t of point i for t < T, its counter t - T for t >= T;
// sub[i]: its subspace.  err bit 0: a point outside the valid list, bit 1: a
// non-finite target.
__global__ __launch_bounds__(kPolyThreads) void poly_features(
    const PolyDev *__restrict__ pd, const SpaceDev *__restrict__ sp,
    const uint32_t *__restrict__ idx, uint32_t nv, const uint32_t *__restrict__ pts,
    const float *__restrict__ Y, uint32_t n, double *__restrict__ F, uint32_t *__restrict__ sub,
    uint32_t *__restrict__ err) {
  const uint32_t T = pd->T, C = pd->C, Ta = T + C;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (uint64_t)n * Ta;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t i = (uint32_t)(e / Ta), t = (uint32_t)(e - (uint64_t)i * Ta);
    const uint32_t p = pts[i];
    uint64_t lo = 0, hi = 0;
    if (p < nv) decode_packed(idx[p], sp, lo, hi);
    else if (t == 0) atomicOr(err, 1u);
    double v;
    if (t < T) {
      const uint32_t d = pd->terms[t];
      v = 1.0;
      for (uint32_t q = 0; q < term_count(d); ++q) {
        const uint32_t j = term_var(d, q);
        v *= pd->xv64[j * CGS_MAX_RADIX + digit_of(lo, hi, j)];
      }
    } else {
      const float y = Y[(uint64_t)i * C + (t - T)];
      if (!isfinite(y)) atomicOr(err, 2u);
      v = isfinite(y) ? (double)y : 0.0;
    }
    F[e] = v;
    if (t == 0) sub[i] = subspace_of(pd, lo, hi);
  }
}

// Gram matrix [F | Y]^T [F | Y] of one subspace's points, one 32 x 32 block
// of it per workgroup: blockIdx.x = subspace, blockIdx.y = block pair
// (a-block <= b-block), blockIdx.z = part: part q of gridDim.z sums the q-th
// contiguous share of list[off[s] .. off[s + 1]) (the subspace's points in
// input order) into G + q * S * Ta^2; poly_gram_sum adds the parts in order,
// so the sums are the same on every run.  The rows of a chunk of points are
// staged in LDS with all loads in flight.
__global__ __launch_bounds__(kPolyThreads) void poly_gram(const PolyDev *__restrict__ pd,
                                                          const double *__restrict__ F,
                                                          const uint32_t *__restrict__ list,
                                                          const uint32_t *__restrict__ off,
                                                          const uint32_t *__restrict__ pairs,
                                                          double *__restrict__ G) {
  extern __shared__ double gl[]; // fa[kGramChunk][kGB + 1], fb[kGramChunk][kGB + 1]
  double(*fa)[kGB + 1] = reinterpret_cast<double(*)[kGB + 1]>(gl);
  double(*fb)[kGB + 1] = reinterpret_cast<double(*)[kGB + 1]>(gl + kGramChunk * (kGB + 1));
  const uint32_t T = pd->T, Ta = T + pd->C, s = blockIdx.x;
  const uint32_t pr = pairs[blockIdx.y];
  const uint32_t a0 = (pr & 0xffffu) * kGB, b0 = (pr >> 16) * kGB;
  const uint32_t t = threadIdx.x;
  const uint32_t ra = (t / (kGB / 2)) * 2, cb = (t % (kGB / 2)) * 2; // 2 x 2 outputs
  const uint32_t q0 = off[s], len = off[s + 1] - q0;
  const uint32_t p0 = q0 + (uint32_t)((uint64_t)len * blockIdx.z / gridDim.z);
  const uint32_t p1 = q0 + (uint32_t)((uint64_t)len * (blockIdx.z + 1) / gridDim.z);
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  constexpr int kB = 8;
  for (uint32_t base = p0; base < p1; base += kGramChunk) {
    const uint32_t m = min((uint32_t)kGramChunk, p1 - base);
    __syncthreads();
    for (uint32_t e0 = t; e0 < m * kGB; e0 += kB * kPolyThreads) {
      double va[kB], vb[kB];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const uint32_t e = min(e0 + u * kPolyThreads, m * kGB - 1);
        const uint32_t p = e / kGB, c = e % kGB;
        const double *row = F + (uint64_t)list[base + p] * Ta;
        va[u] = a0 + c < Ta ? row[a0 + c] : 0.0;
        vb[u] = b0 + c < Ta ? row[b0 + c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const uint32_t e = e0 + u * kPolyThreads;
        if (e < m * kGB) {
          fa[e / kGB][e % kGB] = va[u];
          fb[e / kGB][e % kGB] = vb[u];
        }
      }
    }
    __syncthreads();
    for (uint32_t p = 0; p < m; ++p) {
      const double x0 = fa[p][ra], x1 = fa[p][ra + 1], y0 = fb[p][cb], y1 = fb[p][cb + 1];
      acc[0][0] += x0 * y0;
      acc[0][1] += x0 * y1;
      acc[1][0] += x1 * y0;
      acc[1][1] += x1 * y1;
    }
  }
  double *Gs = G + ((uint64_t)blockIdx.z * gridDim.x + s) * Ta * Ta;
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) {
      const uint32_t a = a0 + ra + u, b = b0 + cb + v;
      if (a < Ta && b < Ta) {
        Gs[(uint64_t)a * Ta + b] = acc[u][v];
        Gs[(uint64_t)b * Ta + a] = acc[u][v];
      }
    }
}

// G[e] = sum of the parts' entries e, parts in order (Gp: [parts][S Ta^2]).
__global__ __launch_bounds__(256) void poly_gram_sum(const double *__restrict__ Gp,
                                                     uint64_t total, uint32_t parts,
                                                     double *__restrict__ G) {
  for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * 256) {
    double x = Gp[e];
    for (uint32_t q = 1; q < parts; ++q) x += Gp[(uint64_t)q * total + e];
    G[e] = x;
  }
}

__device__ __forceinline__ uint32_t pk(uint32_t i, uint32_t j) { return i * (i + 1) / 2 + j; }

// One workgroup per subspace: (G + lam I) beta = R by Cholesky in LDS
// (packed lower triangle), then the two triangular solves for CC counters at
// a time, each elimination step spread over (row, counter) pairs.
__global__ __launch_bounds__(kPolyThreads) void poly_solve(const PolyDev *__restrict__ pd,
                                                           const double *__restrict__ G,
                                                           uint32_t CC,
                                                           double *__restrict__ beta64,
                                                           float *__restrict__ beta32,
                                                           uint32_t *__restrict__ err) {
  extern __shared__ double L[]; // packed lower triangle, then z[T][CC]
  __shared__ double s_lam;
  const uint32_t T = pd->T, C = pd->C, Ta = T + C, s = blockIdx.x, t = threadIdx.x;
  const uint32_t tx = t % 16, ty = t / 16;
  const double *Gs = G + (uint64_t)s * Ta * Ta;
  double *z = L + (uint64_t)T * (T + 1) / 2;
  double *b64 = beta64 + (uint64_t)s * T * C;
  float *b32 = beta32 + (uint64_t)s * T * C;
  if (Gs[0] == 0.0) { // no point in this subspace (the constant column sums to n_s)
    for (uint32_t e = t; e < T * C; e += kPolyThreads) {
      b64[e] = 0.0;
      b32[e] = 0.0f;
    }
    return;
  }
  // G's lower triangle into L by the whole workgroup, 8 loads per thread in
  // flight (one thread per row would wait for up to T loads in turn)
  constexpr int kB = 8;
  const uint32_t nt = T * T;
  for (uint32_t e0 = t; e0 < nt; e0 += kB * kPolyThreads) {
    double v[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const uint32_t e = min(e0 + u * kPolyThreads, nt - 1);
      v[u] = Gs[(uint64_t)(e / T) * Ta + e % T];
    }
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const uint32_t e = e0 + u * kPolyThreads, i = e / T, j = e % T;
      if (e < nt && j <= i) L[pk(i, j)] = v[u];
    }
  }
  __syncthreads();
  if (t == 0) { // the trace in index order
    double tr = 0.0;
    for (uint32_t i = 0; i < T; ++i) tr += L[pk(i, i)];
    s_lam = kRidge * tr / (double)T;
  }
  __syncthreads();
  for (uint32_t i = t; i < T; i += kPolyThreads) L[pk(i, i)] += s_lam;
  // right-looking Cholesky, column by column; the trailing update is tiled
  // 16 x 16 over (row, column) pairs of the remaining lower triangle
  for (uint32_t j = 0; j < T; ++j) {
    __syncthreads();
    if (t == 0) {
      double d = L[pk(j, j)];
      if (!(d > 0.0)) {
        atomicOr(err, 4u);
        d = s_lam;
      }
      L[pk(j, j)] = sqrt(d);
    }
    __syncthreads();
    const double djj = L[pk(j, j)];
    for (uint32_t i = j + 1 + t; i < T; i += kPolyThreads) L[pk(i, j)] /= djj;
    __syncthreads();
    for (uint32_t i = j + 1 + ty; i < T; i += 16) {
      const double lij = L[pk(i, j)];
      for (uint32_t k = j + 1 + tx; k <= i; k += 16) L[pk(i, k)] -= lij * L[pk(k, j)];
    }
  }
  // L z = R, then L^T beta = z, CC counters at a time
  for (uint32_t c0 = 0; c0 < C; c0 += CC) {
    const uint32_t cc = min(CC, C - c0);
    __syncthreads();
    for (uint32_t e0 = t; e0 < T * cc; e0 += kB * kPolyThreads) {
      double v[kB];
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const uint32_t e = min(e0 + u * kPolyThreads, T * cc - 1);
        v[u] = Gs[(uint64_t)(e / cc) * Ta + T + c0 + e % cc];
      }
#pragma unroll
      for (int u = 0; u < kB; ++u) {
        const uint32_t e = e0 + u * kPolyThreads;
        if (e < T * cc) z[(e / cc) * CC + e % cc] = v[u];
      }
    }
    for (uint32_t i = 0; i < T; ++i) {
      __syncthreads();
      if (t < cc) z[i * CC + t] /= L[pk(i, i)];
      __syncthreads();
      for (uint32_t e = t; e < (T - 1 - i) * cc; e += kPolyThreads) {
        const uint32_t k = i + 1 + e / cc, c = e % cc;
        z[k * CC + c] -= L[pk(k, i)] * z[i * CC + c];
      }
    }
    for (uint32_t i = T; i-- > 0;) {
      __syncthreads();
      if (t < cc) z[i * CC + t] /= L[pk(i, i)];
      __syncthreads();
      for (uint32_t e = t; e < i * cc; e += kPolyThreads) {
        const uint32_t k = e / cc, c = e % cc;
        z[k * CC + c] -= L[pk(i, k)] * z[i * CC + c];
      }
    }
    __syncthreads();
    for (uint32_t e = t; e < T * cc; e += kPolyThreads) {
      const uint32_t i = e / cc, c = e % cc;
      const double v = z[i * CC + c];
      b64[(uint64_t)i * C + c0 + c] = v;
      b32[(uint64_t)i * C + c0 + c] = (float)v;
    }
  }
}

// ---------------------------------------------------------------- evaluate
// P[c][l] for the valid configurations whose subspace lies in this
// workgroup's group of SG subspaces (group blockIdx.x / per_group, part
// blockIdx.x % per_group of the valid list): coefficients of the group,
// padded with zeros to CB counters so every multiply-add runs unguarded on
// vector loads, feature table and term descriptors staged in LDS.
template <int CB>
__global__ __launch_bounds__(kEvalThreads) void poly_eval(const PolyDev *__restrict__ pd,
                                                          const SpaceDev *__restrict__ sp,
                                                          const uint32_t *__restrict__ idx,
                                                          uint32_t nv,
                                                          const float *__restrict__ beta32,
                                                          uint32_t SG, uint32_t per_group,
                                                          float *__restrict__ P, uint64_t stride) {
  extern __shared__ float lds[]; // [SG][T][CB] coefficients
  __shared__ float xv[CGS_MAX_PARAMS * CGS_MAX_RADIX];
  __shared__ uint32_t terms[kPolyMaxTerms];
  const uint32_t T = pd->T, C = pd->C, S = pd->S, t = threadIdx.x;
  const uint32_t group = blockIdx.x / per_group, part = blockIdx.x % per_group;
  const uint32_t g0 = group * SG, g1 = min(S, g0 + SG);
  // 16 coefficient loads per thread in flight before the first LDS store (a
  // plain loop waits for every load in turn)
  constexpr int kB = 16;
  const uint32_t n_co = (g1 - g0) * T * CB;
  for (uint32_t e0 = t; e0 < n_co; e0 += kB * kEvalThreads) {
    float v[kB];
#pragma unroll
    for (int b = 0; b < kB; ++b) {
      const uint32_t e = e0 + b * kEvalThreads;
      const uint32_t c = e % CB, st = e / CB; // st = (s - g0) * T + term
      v[b] = (e < n_co && c < C) ? beta32[((uint64_t)g0 * T + st) * C + c] : 0.0f;
    }
#pragma unroll
    for (int b = 0; b < kB; ++b) {
      const uint32_t e = e0 + b * kEvalThreads;
      if (e < n_co) lds[e] = v[b];
    }
  }
  for (uint32_t e = t; e < CGS_MAX_PARAMS * CGS_MAX_RADIX; e += kEvalThreads) xv[e] = pd->xv32[e];
  for (uint32_t e = t; e < T; e += kEvalThreads) terms[e] = pd->terms[e];
  __syncthreads();
  // product of the features of term d for the configuration with digits lo, hi
  auto feature = [&](uint32_t d, uint64_t lo, uint64_t hi) {
    float f = 1.0f;
    for (uint32_t q = 0; q < term_count(d); ++q) {
      const uint32_t j = term_var(d, q);
      f *= xv[j * CGS_MAX_RADIX + digit_of(lo, hi, j)];
    }
    return f;
  };
  auto one = [&](uint32_t l, uint64_t lo, uint64_t hi, uint32_t s) {
    const float *bs = lds + (uint64_t)(s - g0) * T * CB;
    float acc[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[c] = 0.0f;
    for (uint32_t k = 0; k < T; ++k) {
      const float f = feature(terms[k], lo, hi);
      const float4 *bk = reinterpret_cast<const float4 *>(bs + k * CB);
#pragma unroll
      for (int c4 = 0; c4 < CB / 4; ++c4) {
        const float4 b = bk[c4];
        acc[4 * c4] += f * b.x;
        acc[4 * c4 + 1] += f * b.y;
        acc[4 * c4 + 2] += f * b.z;
        acc[4 * c4 + 3] += f * b.w;
      }
    }
#pragma unroll
    for (int c = 0; c < CB; ++c)
      if ((uint32_t)c < C) P[(uint64_t)c * stride + l] = fmaxf(acc[c], 0.0f); // counters >= 0
  };
  if constexpr (CB > 32) { // two accumulator sets would not fit in registers
    for (uint32_t l = part * kEvalThreads + t; l < nv; l += per_group * kEvalThreads) {
      uint64_t lo, hi;
      decode_packed(idx[l], sp, lo, hi);
      const uint32_t s = subspace_of(pd, lo, hi);
      if (s >= g0 && s < g1) one(l, lo, hi, s);
    }
    return;
  }
  // two consecutive configurations per thread: when they share a subspace
  // (consecutive ones mostly do) each coefficient read from LDS serves both
  for (uint32_t l0 = 2 * (part * kEvalThreads + t); l0 < nv;
       l0 += 2 * per_group * kEvalThreads) {
    const uint32_t l1 = l0 + 1;
    uint64_t lo0, hi0, lo1 = 0, hi1 = 0;
    decode_packed(idx[l0], sp, lo0, hi0);
    const uint32_t s0 = subspace_of(pd, lo0, hi0);
    uint32_t s1 = ~0u;
    if (l1 < nv) {
      decode_packed(idx[l1], sp, lo1, hi1);
      s1 = subspace_of(pd, lo1, hi1);
    }
    const bool in0 = s0 >= g0 && s0 < g1, in1 = s1 >= g0 && s1 < g1;
    if (in0 && in1 && s0 == s1) {
      const float *bs = lds + (uint64_t)(s0 - g0) * T * CB;
      float a0[CB], a1[CB];
#pragma unroll
      for (int c = 0; c < CB; ++c) a0[c] = a1[c] = 0.0f;
      for (uint32_t k = 0; k < T; ++k) {
        const uint32_t d = terms[k];
        const float f0 = feature(d, lo0, hi0), f1 = feature(d, lo1, hi1);
        const float4 *bk = reinterpret_cast<const float4 *>(bs + k * CB);
#pragma unroll
        for (int c4 = 0; c4 < CB / 4; ++c4) {
          const float4 b = bk[c4];
          a0[4 * c4] += f0 * b.x;
          a0[4 * c4 + 1] += f0 * b.y;
          a0[4 * c4 + 2] += f0 * b.z;
          a0[4 * c4 + 3] += f0 * b.w;
          a1[4 * c4] += f1 * b.x;
          a1[4 * c4 + 1] += f1 * b.y;
          a1[4 * c4 + 2] += f1 * b.z;
          a1[4 * c4 + 3] += f1 * b.w;
        }
      }
#pragma unroll
      for (int c = 0; c < CB; ++c)
        if ((uint32_t)c < C)
          *reinterpret_cast<float2 *>(P + (uint64_t)c * stride + l0) =
              make_float2(fmaxf(a0[c], 0.0f), fmaxf(a1[c], 0.0f)); // counters >= 0
    } else {
      if (in0) one(l0, lo0, hi0, s0);
      if (in1) one(l1, lo1, hi1, s1);
    }
  }
}

template <typename K> hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

constexpr size_t kEvalLds = 144 * 1024;
constexpr size_t kSolveLds = 156 * 1024;

} // namespace

// LDS of the solve: the packed factor, then as many counters' right-hand
// sides as fit in the rest of 160 KB (at least one).
uint32_t poly_solve_cc(int T, int C) {
  const size_t tri = (size_t)T * (T + 1) / 2 * 8;
  const size_t room = tri < kSolveLds ? kSolveLds - tri : 0;
  return (uint32_t)std::max<size_t>(1, std::min<size_t>(C, room / ((size_t)T * 8)));
}
size_t poly_solve_lds(int T, int C) {
  return ((size_t)T * (T + 1) / 2 + (size_t)T * poly_solve_cc(T, C)) * 8;
}

hipError_t launch_poly_design(const SpaceDev *d_space, const uint32_t *d_idx, uint32_t nv,
                              const uint32_t *d_allowed, uint64_t *d_tile_cnt,
                              uint64_t *d_tile_off, uint32_t *d_out, hipStream_t stream) {
  const uint32_t tiles = (nv + kPolyThreads - 1) / kPolyThreads;
  const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(tiles, 4096));
  poly_design_count<<<grid, kPolyThreads, 0, stream>>>(d_space, d_idx, nv, d_allowed, d_tile_cnt);
  poly_excl_scan<<<1, 1024, 0, stream>>>(d_tile_cnt, d_tile_off, tiles);
  poly_design_write<<<grid, kPolyThreads, 0, stream>>>(d_space, d_idx, nv, d_allowed, d_tile_off,
                                                      d_out);
  return hipGetLastError();
}

uint32_t poly_gram_parts(int S, uint32_t n_pairs) {
  const uint64_t wgs = (uint64_t)S * n_pairs;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(8, 1024 / std::max<uint64_t>(wgs, 1)));
}

hipError_t launch_poly_fit(const PolyDev *d_pd, int T, int C, int S, const SpaceDev *d_space,
                           const uint32_t *d_idx, uint32_t nv, const uint32_t *d_pts,
                           const float *d_Y, uint32_t n, double *d_F, uint32_t *d_sub,
                           const uint32_t *d_list, const uint32_t *d_off,
                           const uint32_t *d_pairs, uint32_t n_pairs, double *d_G, double *d_Gp,
                           double *d_beta64, float *d_beta32, uint32_t *d_err,
                           hipStream_t stream) {
  const uint64_t fe = (uint64_t)n * (T + C);
  const uint32_t gf = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(8192, (fe + 255) / 256));
  poly_features<<<gf, kPolyThreads, 0, stream>>>(d_pd, d_space, d_idx, nv, d_pts, d_Y, n, d_F,
                                                 d_sub, d_err);
  const size_t gram_lds = (size_t)2 * kGramChunk * (kGB + 1) * sizeof(double);
  hipError_t e = allow_lds(poly_gram, gram_lds);
  if (e != hipSuccess) return e;
  // few (subspace, block pair) workgroups: each subspace's points in parts
  const uint32_t parts = d_Gp ? poly_gram_parts(S, n_pairs) : 1u;
  poly_gram<<<dim3(S, n_pairs, parts), kPolyThreads, gram_lds, stream>>>(
      d_pd, d_F, d_list, d_off, d_pairs, parts > 1 ? d_Gp : d_G);
  if (parts > 1) {
    const uint64_t total = (uint64_t)S * (T + C) * (T + C);
    const uint32_t g = (uint32_t)std::min<uint64_t>(4096, (total + 255) / 256);
    poly_gram_sum<<<g, 256, 0, stream>>>(d_Gp, total, parts, d_G);
  }
  const size_t lds = poly_solve_lds(T, C);
  e = allow_lds(poly_solve, lds);
  if (e != hipSuccess) return e;
  poly_solve<<<S, kPolyThreads, lds, stream>>>(d_pd, d_G, poly_solve_cc(T, C), d_beta64,
                                               d_beta32, d_err);
  return hipGetLastError();
}

hipError_t launch_poly_eval(const PolyDev *d_pd, int T, int C, int S, const SpaceDev *d_space,
                            const uint32_t *d_idx, uint32_t nv, const float *d_beta32, float *d_P,
                            uint64_t stride, hipStream_t stream) {
  const int CB = C <= 8 ? 8 : C <= 16 ? 16 : C <= 24 ? 24 : C <= 32 ? 32 : C <= 48 ? 48 : 64;
  const size_t per = (size_t)T * CB * 4;
  const uint32_t SG = (uint32_t)std::max<size_t>(1, std::min<size_t>(S, kEvalLds / per));
  const uint32_t groups = (S + SG - 1) / SG;
  const size_t lds = SG * per;
  const uint32_t grid = std::max<uint32_t>(
      1, std::min<uint32_t>(1024, (nv + kEvalThreads - 1) / kEvalThreads));
  hipError_t e = hipSuccess;
#define CGS_POLY_EVAL(CBV)                                                                      \
  do {                                                                                          \
    e = allow_lds(poly_eval<CBV>, lds);                                                         \
    if (e == hipSuccess)                                                                        \
      poly_eval<CBV><<<grid * groups, kEvalThreads, lds, stream>>>(                             \
          d_pd, d_space, d_idx, nv, d_beta32, SG, grid, d_P, stride);                           \
  } while (0)
  switch (CB) {
  case 8: CGS_POLY_EVAL(8); break;
  case 16: CGS_POLY_EVAL(16); break;
  case 24: CGS_POLY_EVAL(24); break;
  case 32: CGS_POLY_EVAL(32); break;
  case 48: CGS_POLY_EVAL(48); break;
  default: CGS_POLY_EVAL(64); break;
  }
#undef CGS_POLY_EVAL
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

} // namespace cgs
