// Regression-forest evaluation over every valid configuration (Sect. 3.4.2:
// internal nodes test a tuning parameter, leaves hold predicted counters).
//
// One thread per valid configuration, 256 per workgroup.  Each thread decodes
// its raw index once into packed 4-bit digits.  Trees are processed one at a
// time: the workgroup stages tree t's internal nodes (uint16: feature |
// threshold << 8) in LDS, every thread walks depth D levels out of LDS and
// parks its leaf id in LDS.  Then each thread gathers its T leaf vectors
// (float4 loads from the L2-resident leaf array), sums them in ascending t
// starting from tree 0, divides once by T, and writes the counters
// structure-of-arrays: P[c][l], so a row of P is contiguous over
// configurations and the sweep reads it coalesced.
#include <algorithm>

#include "device_common.h"
#include "models.h"

namespace cgs {

namespace {

constexpr int kForestThreads = 256;
constexpr int kForestBatch = 16; // loads in flight per thread (node staging, leaf gathers)

__global__ __launch_bounds__(kForestThreads) void forest_eval(
    const SpaceDev *__restrict__ sp, const uint32_t *__restrict__ idx, uint32_t first,
    uint32_t count, const uint16_t *__restrict__ nodes, const float *__restrict__ leaves,
    int n_trees, int depth, int n_counters, float *__restrict__ P, uint64_t stride,
    uint16_t *__restrict__ leaf_out) {
  extern __shared__ uint16_t smem[];
  const uint32_t n_int = (1u << depth) - 1u;
  const uint32_t n_int_pad = (n_int + 8u) & ~7u; // keep the leaf-id area 16-byte aligned
  uint16_t *lnodes = smem;
  uint16_t *lleaf = smem + n_int_pad; // [T][256]

  const uint32_t i = blockIdx.x * kForestThreads + threadIdx.x;
  const bool active = i < count;
  const uint32_t l = first + i;
  uint64_t lo = 0, hi = 0;
  if (active) decode_packed(idx[l], sp, lo, hi);

  for (int t = 0; t < n_trees; ++t) {
    __syncthreads();
    const uint16_t *tn = nodes + (size_t)t * n_int;
    // the tree's nodes, kForestBatch loads per thread issued before the
    // first LDS store (a plain loop waits for every load in turn)
    for (uint32_t j0 = threadIdx.x; j0 < n_int; j0 += kForestBatch * kForestThreads) {
      uint16_t v[kForestBatch];
#pragma unroll
      for (int b = 0; b < kForestBatch; ++b) {
        const uint32_t j = j0 + b * kForestThreads;
        v[b] = j < n_int ? tn[j] : (uint16_t)0;
      }
#pragma unroll
      for (int b = 0; b < kForestBatch; ++b) {
        const uint32_t j = j0 + b * kForestThreads;
        if (j < n_int) lnodes[j] = v[b];
      }
    }
    __syncthreads();
    uint32_t node = 0;
    for (int lev = 0; lev < depth; ++lev) {
      const uint32_t nd = lnodes[node];
      const uint32_t dig = digit_of(lo, hi, nd & 0xffu);
      node = 2u * node + 1u + (dig > (nd >> 8) ? 1u : 0u);
    }
    const uint32_t leaf = node - n_int;
    lleaf[t * kForestThreads + threadIdx.x] = (uint16_t)leaf;
    if (leaf_out != nullptr && active) leaf_out[(size_t)t * count + i] = (uint16_t)leaf;
  }
  if (!active) return;

  const uint32_t n_leaf = 1u << depth;
  const float t_div = (float)n_trees;
  if ((n_counters & 3) == 0) {
    // leaf vectors of kForestBatch / 2 trees in flight at once; the sums
    // still run in ascending tree order from tree 0
    constexpr int TB = kForestBatch / 2;
    for (int c = 0; c < n_counters; c += 4) {
      float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      for (int t0 = 0; t0 < n_trees; t0 += TB) {
        float4 v[TB];
#pragma unroll
        for (int u = 0; u < TB; ++u) {
          const int t = min(t0 + u, n_trees - 1);
          const uint32_t lf = lleaf[t * kForestThreads + threadIdx.x];
          v[u] = *reinterpret_cast<const float4 *>(leaves + ((size_t)t * n_leaf + lf) * n_counters +
                                                   c);
        }
#pragma unroll
        for (int u = 0; u < TB; ++u) {
          if (t0 + u >= n_trees) break;
          if (t0 + u == 0) {
            acc = v[0];
          } else {
            acc.x = acc.x + v[u].x;
            acc.y = acc.y + v[u].y;
            acc.z = acc.z + v[u].z;
            acc.w = acc.w + v[u].w;
          }
        }
      }
      P[(size_t)(c + 0) * stride + l] = acc.x / t_div;
      P[(size_t)(c + 1) * stride + l] = acc.y / t_div;
      P[(size_t)(c + 2) * stride + l] = acc.z / t_div;
      P[(size_t)(c + 3) * stride + l] = acc.w / t_div;
    }
  } else {
    for (int c = 0; c < n_counters; ++c) {
      float acc = leaves[(size_t)lleaf[threadIdx.x] * n_counters + c];
      for (int t = 1; t < n_trees; ++t) {
        const uint32_t lf = lleaf[t * kForestThreads + threadIdx.x];
        acc = acc + leaves[((size_t)t * n_leaf + lf) * n_counters + c];
      }
      P[(size_t)c * stride + l] = acc / t_div;
    }
  }
}

// Resident variant, for forests whose nodes fit in LDS together (T (2^D - 1)
// uint16 <= kResidentLds, T <= kResidentTrees): each workgroup stages every
// tree once and then runs grid-stride over tiles of configurations, so the
// node tables cross L2 once per workgroup instead of once per 256
// configurations, and there is no barrier per tree.  A thread walks its
// configuration through all trees level by level (the T independent LDS
// reads of a level are in flight together), keeps the leaf ids in registers
// and gathers and sums the leaf vectors exactly as forest_eval does
// (ascending t from tree 0, one division by T).
constexpr int kResidentThreads = 1024;
constexpr int kResidentTrees = 16;
constexpr size_t kResidentLds = 160 * 1024 - 1024;

template <int TM>
__global__ __launch_bounds__(kResidentThreads) void forest_eval_resident(
    const SpaceDev *__restrict__ sp, const uint32_t *__restrict__ idx, uint32_t first,
    uint32_t count, const uint16_t *__restrict__ nodes, const float *__restrict__ leaves,
    int n_trees, int depth, int n_counters, float *__restrict__ P, uint64_t stride,
    uint16_t *__restrict__ leaf_out) {
  extern __shared__ uint16_t lnodes[]; // [T][2^D - 1]
  const uint32_t n_int = (1u << depth) - 1u;
  const uint32_t total = (uint32_t)n_trees * n_int;
  for (uint32_t j0 = threadIdx.x; j0 < total; j0 += kForestBatch * kResidentThreads) {
    uint16_t v[kForestBatch];
#pragma unroll
    for (int b = 0; b < kForestBatch; ++b) {
      const uint32_t j = j0 + b * kResidentThreads;
      v[b] = j < total ? nodes[j] : (uint16_t)0;
    }
#pragma unroll
    for (int b = 0; b < kForestBatch; ++b) {
      const uint32_t j = j0 + b * kResidentThreads;
      if (j < total) lnodes[j] = v[b];
    }
  }
  __syncthreads();
  const uint32_t n_leaf = 1u << depth;
  // x / T; for T a power of two, x * (1 / T) is the same float (exact scaling)
  const float t_div = (float)n_trees;
  const bool pow2 = (n_trees & (n_trees - 1)) == 0;
  const float t_inv = 1.0f / t_div;
  const uint32_t n_tiles = (count + kResidentThreads - 1) / kResidentThreads;
  for (uint32_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const uint32_t i = tile * kResidentThreads + threadIdx.x;
    if (i >= count) break; // the last tile; no barrier follows
    const uint32_t l = first + i;
    uint64_t lo, hi;
    decode_packed(idx[l], sp, lo, hi);
    // walks of up to 8 trees interleaved level by level; leaf ids two per
    // register
    constexpr int TW = TM < 8 ? TM : 8;
    uint32_t leafp[(TM + 1) / 2];
#pragma unroll
    for (int t0 = 0; t0 < TM; t0 += TW) {
      uint32_t nw[TW];
#pragma unroll
      for (int u = 0; u < TW; ++u) nw[u] = 0;
      for (int lev = 0; lev < depth; ++lev) {
#pragma unroll
        for (int u = 0; u < TW; ++u) {
          if (t0 + u < n_trees) {
            const uint32_t nd = lnodes[(t0 + u) * n_int + nw[u]];
            nw[u] = 2u * nw[u] + 1u + (digit_of(lo, hi, nd & 0xffu) > (nd >> 8) ? 1u : 0u);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < TW; u += 2)
        leafp[(t0 + u) / 2] = (nw[u] - n_int) | (u + 1 < TW ? (nw[u + 1] - n_int) << 16 : 0u);
    }
    auto leaf_of = [&](int t) { return (leafp[t >> 1] >> (16 * (t & 1))) & 0xffffu; };
    if (leaf_out != nullptr) {
#pragma unroll
      for (int t = 0; t < TM; ++t)
        if (t < n_trees) leaf_out[(size_t)t * count + i] = (uint16_t)leaf_of(t);
    }
    auto store = [&](int c, float acc) {
      P[(size_t)c * stride + l] = pow2 ? acc * t_inv : acc / t_div;
    };
    if ((n_counters & 3) == 0) {
      // leaf vectors of up to 8 trees in flight (more would spill at 1024
      // threads); the sum runs in ascending t from tree 0
      constexpr int TB = TM < 8 ? TM : 8;
      for (int c = 0; c < n_counters; c += 4) {
        float4 acc;
#pragma unroll
        for (int t0 = 0; t0 < TM; t0 += TB) {
          float4 v[TB];
#pragma unroll
          for (int u = 0; u < TB; ++u)
            if (t0 + u < n_trees)
              v[u] = *reinterpret_cast<const float4 *>(
                  leaves + ((size_t)(t0 + u) * n_leaf + leaf_of(t0 + u)) * n_counters + c);
          if (t0 == 0) acc = v[0];
#pragma unroll
          for (int u = (t0 == 0 ? 1 : 0); u < TB; ++u) {
            if (t0 + u < n_trees) {
              acc.x = acc.x + v[u].x;
              acc.y = acc.y + v[u].y;
              acc.z = acc.z + v[u].z;
              acc.w = acc.w + v[u].w;
            }
          }
        }
        store(c, acc.x);
        store(c + 1, acc.y);
        store(c + 2, acc.z);
        store(c + 3, acc.w);
      }
    } else {
      for (int c = 0; c < n_counters; ++c) {
        float acc = leaves[(size_t)leaf_of(0) * n_counters + c];
#pragma unroll
        for (int t = 1; t < TM; ++t)
          if (t < n_trees) acc = acc + leaves[((size_t)t * n_leaf + leaf_of(t)) * n_counters + c];
        store(c, acc);
      }
    }
  }
}

// Partial sums of squared prediction differences over sampled valid
// configurations: one double per workgroup.  DENSE_A: Pa holds the sampled
// configurations' predictions in sample order (column i for sample i).
template <bool DENSE_A>
__global__ __launch_bounds__(256) void sq_diff(const float *__restrict__ Pa,
                                               const float *__restrict__ Pb, uint64_t stride_a,
                                               uint64_t stride_b, int n_counters,
                                               const uint32_t *__restrict__ sample, uint32_t n,
                                               double *__restrict__ partial) {
  __shared__ double red[4];
  double acc = 0.0;
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const uint32_t l = sample[i];
    for (int c = 0; c < n_counters; ++c) {
      const double d = (double)Pa[(size_t)c * stride_a + (DENSE_A ? i : l)] -
                       (double)Pb[(size_t)c * stride_b + l];
      acc += d * d;
    }
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Predictions of listed valid configurations: out[i][c] = P[c][idx[i]].
__global__ __launch_bounds__(256) void gather_rows(const float *__restrict__ P, uint64_t stride,
                                                   int n_counters,
                                                   const uint32_t *__restrict__ idx, uint32_t n,
                                                   float *__restrict__ out) {
  const uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (uint64_t)n * n_counters) return;
  const uint32_t i = (uint32_t)(e / n_counters);
  const int c = (int)(e % n_counters);
  out[e] = P[(size_t)c * stride + idx[i]];
}

} // namespace

hipError_t launch_gather_rows(const float *P, uint64_t stride, int n_counters,
                              const uint32_t *d_idx, uint32_t n, float *d_out,
                              hipStream_t stream) {
  const uint64_t total = (uint64_t)n * n_counters;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, P,
                     stride, n_counters, d_idx, n, d_out);
  return hipGetLastError();
}

hipError_t launch_sq_diff(const float *Pa, const float *Pb, uint64_t stride_a, uint64_t stride_b,
                          int n_counters, const uint32_t *sample, uint32_t n, double *partial,
                          uint32_t grid, hipStream_t stream) {
  hipLaunchKernelGGL(sq_diff<false>, dim3(grid), dim3(256), 0, stream, Pa, Pb, stride_a, stride_b,
                     n_counters, sample, n, partial);
  return hipGetLastError();
}

hipError_t launch_sq_diff_dense(const float *Pa, const float *Pb, uint64_t stride_a,
                                uint64_t stride_b, int n_counters, const uint32_t *sample,
                                uint32_t n, double *partial, uint32_t grid, hipStream_t stream) {
  hipLaunchKernelGGL(sq_diff<true>, dim3(grid), dim3(256), 0, stream, Pa, Pb, stride_a, stride_b,
                     n_counters, sample, n, partial);
  return hipGetLastError();
}

// Evaluates valid configurations [first, first + count).  With d_leaf_out
// set, also writes leaf ids [T][count] and skips nothing else.
hipError_t launch_forest_eval(const SpaceDev *d_space, const uint32_t *d_idx, uint32_t n_valid,
                              const uint16_t *d_nodes, const float *d_leaves, int n_trees,
                              int depth, int n_counters, float *d_P, uint64_t stride,
                              uint16_t *d_leaf_out, uint32_t leaf_first, uint32_t leaf_count,
                              hipStream_t stream) {
  const uint32_t first = d_leaf_out ? leaf_first : 0u;
  const uint32_t count = d_leaf_out ? leaf_count : n_valid;
  if (count == 0) return hipSuccess;
  const uint32_t n_int = (1u << depth) - 1u;
  const size_t res_lds = (size_t)n_trees * n_int * sizeof(uint16_t);
  const bool resident = n_trees <= kResidentTrees && res_lds <= kResidentLds;
  if (resident) {
    // as many workgroups as fit on the device at once (LDS-bound), at most
    // one per tile
    int dev = 0, n_cu = 256;
    if (hipGetDevice(&dev) == hipSuccess)
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    const uint32_t per_cu = (uint32_t)std::max<size_t>(1, std::min<size_t>(2, kResidentLds / std::max<size_t>(res_lds, 1)));
    const uint32_t tiles = (count + kResidentThreads - 1) / kResidentThreads;
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(tiles, (uint32_t)n_cu * per_cu));
#define CGS_FOREST_RES(TMV)                                                                     \
  do {                                                                                          \
    if (res_lds > 65536) {                                                                      \
      const hipError_t e = hipFuncSetAttribute(                                                 \
          reinterpret_cast<const void *>(forest_eval_resident<TMV>),                            \
          hipFuncAttributeMaxDynamicSharedMemorySize, (int)res_lds);                            \
      if (e != hipSuccess) return e;                                                            \
    }                                                                                           \
    hipLaunchKernelGGL(forest_eval_resident<TMV>, dim3(grid), dim3(kResidentThreads), res_lds,  \
                       stream, d_space, d_idx, first, count, d_nodes, d_leaves, n_trees, depth, \
                       n_counters, d_P, stride, d_leaf_out);                                    \
  } while (0)
    if (n_trees <= 1) CGS_FOREST_RES(1);
    else if (n_trees <= 2) CGS_FOREST_RES(2);
    else if (n_trees <= 4) CGS_FOREST_RES(4);
    else if (n_trees <= 8) CGS_FOREST_RES(8);
    else CGS_FOREST_RES(16);
#undef CGS_FOREST_RES
    return hipGetLastError();
  }
  const uint32_t n_int_pad = (n_int + 8u) & ~7u;
  const size_t lds = (size_t)(n_int_pad + (uint32_t)n_trees * kForestThreads) * sizeof(uint16_t);
  const uint32_t grid = (count + kForestThreads - 1) / kForestThreads;
  hipLaunchKernelGGL(forest_eval, dim3(grid), dim3(kForestThreads), lds, stream, d_space, d_idx,
                     first, count, d_nodes, d_leaves, n_trees, depth, n_counters, d_P, stride,
                     d_leaf_out);
  return hipGetLastError();
}

// Predictions given per configuration, src[l][C], into the model layout
// P[c][stride].
__global__ void rows_to_columns(const float *__restrict__ src, uint32_t n, int C,
                                float *__restrict__ P, uint64_t stride) {
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (uint64_t)n * C;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t l = e / C, c = e - l * C;
    P[c * stride + l] = src[e];
  }
}

hipError_t launch_rows_to_columns(const float *d_src, uint32_t n, int C, float *d_P,
                                  uint64_t stride, hipStream_t stream) {
  const uint64_t total = (uint64_t)n * C;
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(8192, (total + 255) / 256));
  rows_to_columns<<<grid, 256, 0, stream>>>(d_src, n, C, d_P, stride);
  return hipGetLastError();
}

} // namespace cgs
