// The per-step sweep of Alg. 1: score every unexplored configuration
// (Sect. 3.6, score equation), normalise and quantise the scores
// (score-normalisation equation), and draw the next configuration by an
// exact integer inverse-CDF search (Sect. 3.7).
//
// Data layout (all over valid indices l):
//   P[c][stride]   model predictions, float32, one contiguous row per counter
//   explored       bitmask, bit l % 32 of word l / 32
//   s[stride]      float32 scores of the current step
//   bsum[n_blocks] uint64 sums of the quantised weights of each block of
//                  2^block_log2 configurations
//   acc[2][64]     per-step min / max / count accumulators, two sets used by
//                  alternate steps (the step using one set clears the other)
//
// Kernels per step (two launches up to the first draw):
//   score_pass    4 configurations per thread, float4 loads of up to 8
//                 counter rows issued before any arithmetic; float32 with
//                 every operation rounded (this file is built without
//                 contraction): t = (x - a) / (a + x); s = s + dpc * t,
//                 counters ascending; the profiled configuration counts as
//                 explored.  Per-workgroup min / max of s over unexplored
//                 configurations go to one of 64 accumulator slots with
//                 order-preserving uint32 atomics.
//   weight_draw   one workgroup per block: q = rint(w * 2^23) and the block
//                 sum.  The last workgroup to finish (device-scope counter)
//                 performs the first draw of the step and marks the
//                 profiled configuration explored.
//   draw          further draws of the same step: one workgroup.
// A draw: Q = sum of block sums, r = mulhi64(U, Q), scan of the block sums
// to the block holding r, recompute that block's q and scan it to l with
// prefix_l <= r < prefix_l + q_l; mark l explored and subtract q_l from its
// block sum (Alg. 1 zeroes S_l before the next draw of the iteration).
#include "device_common.h"

namespace cgs {

namespace {

constexpr int kScoreThreads = 256;
constexpr int kWeightThreads = 256;
constexpr int kDrawThreads = 1024;
constexpr int kRowsInFlight = 8;

__device__ __forceinline__ StepAccSums reduce_slots(const StepAcc *__restrict__ slots) {
  StepAccSums r{0xffffffffu, 0u, 0u};
  for (int i = 0; i < kAccSlots; ++i) {
    r.min_key = min(r.min_key, slots[i].min_key);
    r.max_key = max(r.max_key, slots[i].max_key);
    r.n_unexplored += slots[i].n_unexplored;
  }
  return r;
}

__global__ __launch_bounds__(kScoreThreads) void score_pass(
    const float *__restrict__ P, uint64_t stride, uint32_t profile, ActiveCounters act,
    const uint32_t *__restrict__ explored, uint32_t n_valid, float *__restrict__ s_out,
    StepAcc *__restrict__ acc) {
  __shared__ uint32_t red[3][kScoreThreads / kWave];
  const uint32_t g = blockIdx.x * kScoreThreads + threadIdx.x; // group of 4 configs
  const uint32_t l0 = 4u * g;
  float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
  uint32_t ex4 = 0xfu;
  if (l0 < n_valid) {
    const uint32_t word = explored[l0 >> 5];
    ex4 = (word >> (l0 & 31u)) & 0xfu;
    // configurations past the end and the profiled one count as explored
    const uint32_t tail = n_valid - l0;
    if (tail < 4u) ex4 |= (0xfu << tail) & 0xfu;
    if (profile - l0 < 4u) ex4 |= 1u << (profile - l0);
    const float *__restrict__ col = P + l0;
    const int n = profile < n_valid ? act.n : 0;
    for (int j0 = 0; j0 < n; j0 += kRowsInFlight) {
      float4 x[kRowsInFlight];
      float av[kRowsInFlight];
#pragma unroll
      for (int u = 0; u < kRowsInFlight; ++u) {
        if (j0 + u < n) {
          const size_t row = (size_t)act.ctr[j0 + u] * stride;
          x[u] = *reinterpret_cast<const float4 *>(col + row);
          av[u] = P[row + profile];
        }
      }
#pragma unroll
      for (int u = 0; u < kRowsInFlight; ++u) {
        if (j0 + u < n && av[u] != 0.0f) { // a_p == 0: counter not in PC_used
          const float ap = av[u];
          const float d = act.delta[j0 + u];
          {
            const float t = (x[u].x - ap) / (ap + x[u].x);
            s0 = (x[u].x != 0.0f) ? s0 + d * t : s0;
          }
          {
            const float t = (x[u].y - ap) / (ap + x[u].y);
            s1 = (x[u].y != 0.0f) ? s1 + d * t : s1;
          }
          {
            const float t = (x[u].z - ap) / (ap + x[u].z);
            s2 = (x[u].z != 0.0f) ? s2 + d * t : s2;
          }
          {
            const float t = (x[u].w - ap) / (ap + x[u].w);
            s3 = (x[u].w != 0.0f) ? s3 + d * t : s3;
          }
        }
      }
    }
    *reinterpret_cast<float4 *>(s_out + l0) = make_float4(s0, s1, s2, s3);
  }
  uint32_t kmin = 0xffffffffu, kmax = 0u, cnt = 0u;
  const float sv[4] = {s0, s1, s2, s3};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (!((ex4 >> e) & 1u)) {
      const uint32_t k = float_key(sv[e]);
      kmin = min(kmin, k);
      kmax = max(kmax, k);
      ++cnt;
    }
  }
  kmin = wave_umin(kmin);
  kmax = wave_umax(kmax);
  cnt = wave_sum(cnt);
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = kmin;
    red[1][wave] = kmax;
    red[2][wave] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kScoreThreads / kWave; ++w) {
      kmin = min(kmin, red[0][w]);
      kmax = max(kmax, red[1][w]);
      cnt += red[2][w];
    }
    if (cnt != 0u) {
      StepAcc *slot = acc + (blockIdx.x & (kAccSlots - 1));
      atomicMin(&slot->min_key, kmin);
      atomicMax(&slot->max_key, kmax);
      atomicAdd(&slot->n_unexplored, cnt);
    }
  }
}

// Quantised weight of valid index l (0 past the end, for explored
// configurations and for the profiled one).
struct ScoreWeights {
  const float *s;
  uint32_t *explored;
  uint32_t n;
  uint32_t profile;
  float s_min, s_max, gamma, w_min;
  __device__ uint32_t operator()(uint32_t l) const {
    if (l >= n) return 0u;
    return quantized_weight(s[l], explored_bit(explored, l) || l == profile, s_min, s_max, gamma,
                            w_min);
  }
  __device__ void remove(uint32_t l) const { atomicOr(&explored[l >> 5], 1u << (l & 31u)); }
};
struct ArrayWeights {
  uint32_t *q;
  uint32_t n;
  __device__ uint32_t operator()(uint32_t l) const { return l < n ? q[l] : 0u; }
  __device__ void remove(uint32_t l) const { q[l] = 0u; }
};

// Block sums are read with device-coherent loads: in the fused kernel they
// were written by other workgroups of the same launch.
__device__ __forceinline__ uint64_t load_coherent(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int NT, typename W>
__device__ void draw_body(const W &wsrc, int block_log2, uint64_t *__restrict__ bsum,
                          uint32_t n_blocks, uint64_t u64, const uint32_t *__restrict__ idx,
                          DrawResult *__restrict__ res) {
  __shared__ uint64_t scratch[NT / kWave];
  __shared__ uint64_t found_block, found_rem;
  __shared__ int found;
  const uint32_t tid = threadIdx.x;

  // Q = sum of block sums
  uint64_t part = 0;
  for (uint32_t b = tid; b < n_blocks; b += NT) part += load_coherent(bsum + b);
  const uint64_t Q = block_sum<NT>(part, scratch);
  if (Q == 0) {
    if (tid == 0) {
      res->valid = kNoPick;
      res->raw = kNoPick;
      res->total = 0;
      res->r = 0;
    }
    return;
  }
  const uint64_t r = __umul64hi(u64, Q);
  if (tid == 0) {
    // overwritten by the thread that finds the pick; stays "no pick" only if
    // the block sums disagree with the weights (reported as an error)
    res->valid = kNoPick;
    res->raw = kNoPick;
    res->total = Q;
    res->r = r;
    found = 0;
    found_block = 0;
    found_rem = 0;
  }

  // block b with prefix_b <= r < prefix_b + bsum[b]
  uint64_t running = 0;
  for (uint32_t base = 0; base < n_blocks; base += NT) {
    const uint32_t b = base + tid;
    const uint64_t v = b < n_blocks ? load_coherent(bsum + b) : 0ull;
    uint64_t chunk;
    const uint64_t excl = running + block_excl_scan<NT>(v, scratch, chunk);
    if (v != 0 && excl <= r && r < excl + v) {
      found_block = b;
      found_rem = r - excl;
      found = 1;
    }
    running += chunk;
    __syncthreads();
    if (found) break;
  }
  if (!found) return;
  const uint32_t blk = (uint32_t)found_block;
  const uint64_t rem = found_rem;

  // configuration inside the block: thread tid owns a contiguous run
  const uint32_t B = 1u << block_log2;
  const uint32_t per = B / NT;
  const uint32_t first = (blk << block_log2) + tid * per;
  uint64_t mine = 0;
  for (uint32_t e = 0; e < per; ++e) mine += wsrc(first + e);
  uint64_t blk_total;
  uint64_t pre = block_excl_scan<NT>(mine, scratch, blk_total);
  if (mine != 0 && pre <= rem && rem < pre + mine) {
    for (uint32_t e = 0; e < per; ++e) {
      const uint32_t q = wsrc(first + e);
      if (rem < pre + q) {
        const uint32_t l = first + e;
        wsrc.remove(l);
        bsum[blk] = load_coherent(bsum + blk) - q;
        res->valid = l;
        res->raw = idx ? idx[l] : l;
        break;
      }
      pre += q;
    }
  }
}

// One workgroup per block of 2^block_log2 configurations.
__global__ __launch_bounds__(kWeightThreads) void weight_draw(
    const float *__restrict__ s, uint32_t *__restrict__ explored, uint32_t n_valid,
    uint32_t profile, const StepAcc *__restrict__ acc, StepAcc *__restrict__ acc_next,
    float gamma, float w_min, int block_log2, uint64_t *__restrict__ bsum, uint32_t n_blocks,
    uint32_t *__restrict__ done, int do_draw, uint64_t u64, const uint32_t *__restrict__ idx,
    DrawResult *__restrict__ res) {
  __shared__ uint64_t scratch[kWeightThreads / kWave];
  __shared__ int is_last;
  const StepAccSums a = reduce_slots(acc);
  const float s_min = key_float(a.min_key), s_max = key_float(a.max_key);
  if (blockIdx.x == 0 && threadIdx.x < kAccSlots) {
    // clear the accumulators of the next step
    acc_next[threadIdx.x].min_key = 0xffffffffu;
    acc_next[threadIdx.x].max_key = 0u;
    acc_next[threadIdx.x].n_unexplored = 0u;
  }
  const uint32_t base = blockIdx.x << block_log2;
  const uint32_t end = min(n_valid, base + (1u << block_log2));
  uint64_t sum = 0;
  // 4096 configurations per round: 4 float4 of scores per thread, loaded first
  for (uint32_t r0 = base; r0 < end; r0 += 16u * kWeightThreads) {
    float4 sv[4];
    uint32_t ex[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t l0 = r0 + 4u * (threadIdx.x + k * kWeightThreads);
      if (l0 < end) {
        sv[k] = *reinterpret_cast<const float4 *>(s + l0);
        ex[k] = explored[l0 >> 5];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t l0 = r0 + 4u * (threadIdx.x + k * kWeightThreads);
      if (l0 < end) {
        uint32_t ex4 = (ex[k] >> (l0 & 31u)) & 0xfu;
        if (profile - l0 < 4u) ex4 |= 1u << (profile - l0);
        const float ss[4] = {sv[k].x, sv[k].y, sv[k].z, sv[k].w};
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (l0 + e < end)
            sum += quantized_weight(ss[e], (ex4 >> e) & 1u, s_min, s_max, gamma, w_min);
      }
    }
  }
  const uint64_t total = block_sum<kWeightThreads>(sum, scratch);
  if (threadIdx.x == 0) {
    __hip_atomic_store(bsum + blockIdx.x, total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t prev =
        __hip_atomic_fetch_add(done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    is_last = prev == n_blocks - 1;
  }
  __syncthreads();
  if (!is_last) return;
  // last workgroup: every block sum of this launch is visible
  __atomic_thread_fence(__ATOMIC_ACQUIRE);
  if (do_draw) {
    ScoreWeights w{s, explored, n_valid, profile, s_min, s_max, gamma, w_min};
    draw_body<kWeightThreads>(w, block_log2, bsum, n_blocks, u64, idx, res);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (profile < n_valid) atomicOr(&explored[profile >> 5], 1u << (profile & 31u));
    *done = 0u;
  }
}

__global__ __launch_bounds__(kDrawThreads) void draw_scores(
    const float *__restrict__ s, uint32_t *__restrict__ explored, uint32_t n_valid,
    const StepAcc *__restrict__ acc, float gamma, float w_min, int block_log2,
    uint64_t *__restrict__ bsum, uint32_t n_blocks, uint64_t u64,
    const uint32_t *__restrict__ idx, DrawResult *__restrict__ res) {
  const StepAccSums a = reduce_slots(acc);
  ScoreWeights w{s, explored, n_valid, kNoProfile, key_float(a.min_key), key_float(a.max_key),
                 gamma, w_min};
  draw_body<kDrawThreads>(w, block_log2, bsum, n_blocks, u64, idx, res);
}

__global__ __launch_bounds__(kDrawThreads) void draw_array(uint32_t *__restrict__ q, uint32_t n,
                                                           int block_log2,
                                                           uint64_t *__restrict__ bsum,
                                                           uint32_t n_blocks, uint64_t u64,
                                                           DrawResult *__restrict__ res) {
  ArrayWeights w{q, n};
  draw_body<kDrawThreads>(w, block_log2, bsum, n_blocks, u64, nullptr, res);
}

__global__ __launch_bounds__(kWeightThreads) void array_block_sums(const uint32_t *__restrict__ q,
                                                                   uint32_t n, int block_log2,
                                                                   uint64_t *__restrict__ bsum) {
  __shared__ uint64_t scratch[kWeightThreads / kWave];
  const uint32_t B = 1u << block_log2;
  const uint32_t base = blockIdx.x << block_log2;
  uint64_t sum = 0;
  for (uint32_t off = threadIdx.x; off < B; off += kWeightThreads) {
    const uint32_t l = base + off;
    if (l < n) sum += q[l];
  }
  const uint64_t total = block_sum<kWeightThreads>(sum, scratch);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(256) void copy_weights(const float *__restrict__ s,
                                                    uint32_t *__restrict__ explored,
                                                    uint32_t n_valid,
                                                    const StepAcc *__restrict__ acc, float gamma,
                                                    float w_min, uint32_t first, uint32_t count,
                                                    uint32_t *__restrict__ q) {
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const StepAccSums a = reduce_slots(acc);
  ScoreWeights w{s, explored, n_valid, kNoProfile, key_float(a.min_key), key_float(a.max_key),
                 gamma, w_min};
  q[i] = w(first + i);
}

__global__ __launch_bounds__(64) void reset_acc(StepAcc *__restrict__ acc, int n) {
  for (int i = threadIdx.x; i < n; i += 64) {
    acc[i].min_key = 0xffffffffu;
    acc[i].max_key = 0u;
    acc[i].n_unexplored = 0u;
    acc[i].pad = 0u;
  }
}

} // namespace

hipError_t launch_reset_acc(StepAcc *d_acc, int n, hipStream_t stream) {
  hipLaunchKernelGGL(reset_acc, dim3(1), dim3(64), 0, stream, d_acc, n);
  return hipGetLastError();
}

hipError_t launch_score_pass(const float *d_P, uint64_t stride, uint32_t profile,
                             const ActiveCounters &act, const uint32_t *d_explored,
                             uint32_t n_valid, float *d_s, StepAcc *d_acc, hipStream_t stream) {
  const uint32_t groups = (n_valid + 3u) / 4u;
  const uint32_t grid = (groups + kScoreThreads - 1) / kScoreThreads;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(score_pass, dim3(grid), dim3(kScoreThreads), 0, stream, d_P, stride, profile,
                     act, d_explored, n_valid, d_s, d_acc);
  return hipGetLastError();
}

hipError_t launch_weight_draw(const float *d_s, uint32_t *d_explored, uint32_t n_valid,
                              uint32_t profile, const StepAcc *d_acc, StepAcc *d_acc_next,
                              float gamma, float w_min, int block_log2, uint64_t *d_bsum,
                              uint32_t n_blocks, uint32_t *d_done, bool do_draw, uint64_t u64,
                              const uint32_t *d_idx, DrawResult *d_res, hipStream_t stream) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(weight_draw, dim3(n_blocks), dim3(kWeightThreads), 0, stream, d_s, d_explored,
                     n_valid, profile, d_acc, d_acc_next, gamma, w_min, block_log2, d_bsum,
                     n_blocks, d_done, do_draw ? 1 : 0, u64, d_idx, d_res);
  return hipGetLastError();
}

hipError_t launch_draw(const float *d_s, uint32_t *d_explored, uint32_t n_valid,
                       const StepAcc *d_acc, float gamma, float w_min, int block_log2,
                       uint64_t *d_bsum, uint32_t n_blocks, uint64_t u64, const uint32_t *d_idx,
                       DrawResult *d_res, hipStream_t stream) {
  hipLaunchKernelGGL(draw_scores, dim3(1), dim3(kDrawThreads), 0, stream, d_s, d_explored, n_valid,
                     d_acc, gamma, w_min, block_log2, d_bsum, n_blocks, u64, d_idx, d_res);
  return hipGetLastError();
}

hipError_t launch_copy_weights(const float *d_s, uint32_t *d_explored, uint32_t n_valid,
                               const StepAcc *d_acc, float gamma, float w_min, uint32_t first,
                               uint32_t count, uint32_t *d_q, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_weights, dim3((count + 255) / 256), dim3(256), 0, stream, d_s,
                     d_explored, n_valid, d_acc, gamma, w_min, first, count, d_q);
  return hipGetLastError();
}

hipError_t launch_array_block_sums(const uint32_t *d_q, uint32_t n, int block_log2,
                                   uint64_t *d_bsum, hipStream_t stream) {
  const uint32_t n_blocks = (uint32_t)(((uint64_t)n + (1u << block_log2) - 1) >> block_log2);
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(array_block_sums, dim3(n_blocks), dim3(kWeightThreads), 0, stream, d_q, n,
                     block_log2, d_bsum);
  return hipGetLastError();
}

hipError_t launch_array_draw(uint32_t *d_q, uint32_t n, int block_log2, uint64_t *d_bsum,
                             uint32_t n_blocks, uint64_t u64, DrawResult *d_res,
                             hipStream_t stream) {
  hipLaunchKernelGGL(draw_array, dim3(1), dim3(kDrawThreads), 0, stream, d_q, n, block_log2,
                     d_bsum, n_blocks, u64, d_res);
  return hipGetLastError();
}

} // namespace cgs
