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
// Kernels per step (three launches up to the first draw):
//   score_pass    4 configurations per thread, float4 loads of up to 8
//                 counter rows issued before any arithmetic; float32 with
//                 every operation rounded (this file is built without
//                 contraction): t = (x - a) / (a + x); s = s + dpc * t,
//                 counters ascending; the profiled configuration counts as
//                 explored.  Per-workgroup min / max of s over unexplored
//                 configurations go to one of 64 accumulator slots with
//                 order-preserving uint32 atomics.
//   weight_pass   one workgroup per block: q = rint(w * 2^23) and the block
//                 sum (plain stores; the kernel boundary publishes them to
//                 every XCD, which a device-scope handoff inside one launch
//                 would pay for with an L2 write-back per workgroup)
//   draw          one workgroup per draw; the step's first draw also marks the
//                 profiled configuration explored.
// A draw: one scan of the block sums gives Q and the block holding
// r = mulhi64(U, Q); recompute that block's q and scan it to l with
// prefix_l <= r < prefix_l + q_l; mark l explored and subtract q_l from its
// block sum (Alg. 1 zeroes S_l before the next draw of the iteration).  The
// result goes to pinned host memory, closed by a sequence number that the
// host polls.  Every phase issues all of its loads before the first use, so
// a draw costs about four dependent memory round trips.
#include <algorithm>
#include <type_traits>

#include "device_common.h"

namespace cgs {

namespace {

constexpr int kScoreThreads = 256;
constexpr int kWeightThreads = 256;
constexpr int kDrawThreads = 1024;
constexpr int kRowsInFlight = 8;
constexpr uint32_t kScoreGrid = 2048; // 8 workgroups of 256 threads per CU

// Combines the kAccSlots accumulator slots: wave 0 loads one slot per lane
// and reduces across the wave; the result is broadcast through LDS.  Every
// thread of the block must call it (it contains a barrier).
__device__ __forceinline__ StepAccSums reduce_slots(const StepAcc *__restrict__ slots) {
  static_assert(kAccSlots == kWave, "one slot per lane");
  __shared__ StepAccSums shared_sums;
  if (threadIdx.x < kWave) {
    const StepAcc a = slots[threadIdx.x];
    const uint32_t mn = wave_umin(a.min_key), mx = wave_umax(a.max_key);
    const uint32_t n = wave_sum(a.n_unexplored);
    if (threadIdx.x == 0) shared_sums = StepAccSums{mn, mx, n};
  }
  __syncthreads();
  return shared_sums;
}

// Scores the 4 configurations of this thread in `tile` (4 * kScoreThreads
// configurations per tile) and folds the unexplored ones into the running
// min / max keys and count.  Counters ctr[0..n) with changes delta[].
template <int RIF = kRowsInFlight>
__device__ __forceinline__ void score_tile(const float *__restrict__ P, uint64_t stride,
                                           uint32_t profile, int n, const uint32_t *ctr,
                                           const float *delta,
                                           const uint32_t *__restrict__ explored,
                                           uint32_t n_valid, float *__restrict__ s_out,
                                           uint32_t tile, uint32_t &kmin, uint32_t &kmax,
                                           uint32_t &cnt) {
  const uint32_t l0 = 4u * (tile * kScoreThreads + threadIdx.x);
  if (l0 >= n_valid) return;
  float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
  const uint32_t word = explored[l0 >> 5];
  uint32_t ex4 = (word >> (l0 & 31u)) & 0xfu;
  // configurations past the end and the profiled one count as explored
  const uint32_t tail = n_valid - l0;
  if (tail < 4u) ex4 |= (0xfu << tail) & 0xfu;
  if (profile - l0 < 4u) ex4 |= 1u << (profile - l0);
  const float *__restrict__ col = P + l0;
  for (int j0 = 0; j0 < n; j0 += RIF) {
    float4 x[RIF];
    float av[RIF];
#pragma unroll
    for (int u = 0; u < RIF; ++u) {
      if (j0 + u < n) {
        const size_t row = (size_t)ctr[j0 + u] * stride;
        x[u] = *reinterpret_cast<const float4 *>(col + row);
        av[u] = P[row + profile];
      }
    }
#pragma unroll
    for (int u = 0; u < RIF; ++u) {
      if (j0 + u < n && av[u] != 0.0f) { // a_p == 0: counter not in PC_used
        const float ap = av[u];
        const float d = delta[j0 + u];
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
}

// Block-wide reduction of the min / max keys and count; thread 0 adds them
// to accumulator slot `slot` (skipped when nothing was unexplored).
__device__ __forceinline__ void flush_acc(uint32_t kmin, uint32_t kmax, uint32_t cnt,
                                          StepAcc *slot) {
  __shared__ uint32_t red[3][kScoreThreads / kWave];
  kmin = wave_umin(kmin);
  kmax = wave_umax(kmax);
  cnt = wave_sum(cnt);
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  __syncthreads();
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
      atomicMin(&slot->min_key, kmin);
      atomicMax(&slot->max_key, kmax);
      atomicAdd(&slot->n_unexplored, cnt);
    }
  }
}

// Scores 4 configurations per thread over tiles of 4 * kScoreThreads
// configurations, grid-stride, so few workgroups update the accumulators.
// With prof_dev, the profiled configuration is read from device memory
// (written there by the previous step's draw) instead of `profile`.
__global__ __launch_bounds__(kScoreThreads) void score_pass(
    const float *__restrict__ P, uint64_t stride, uint32_t profile,
    const uint32_t *__restrict__ prof_dev, ActiveCounters act,
    const uint32_t *__restrict__ explored, uint32_t n_valid, float *__restrict__ s_out,
    StepAcc *__restrict__ acc) {
  if (prof_dev) profile = *prof_dev;
  uint32_t kmin = 0xffffffffu, kmax = 0u, cnt = 0u;
  const int n = profile < n_valid ? act.n : 0;
  const uint32_t n_tiles = (n_valid + 4u * kScoreThreads - 1) / (4u * kScoreThreads);
  for (uint32_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x)
    score_tile(P, stride, profile, n, act.ctr, act.delta, explored, n_valid, s_out, tile, kmin,
               kmax, cnt);
  flush_acc(kmin, kmax, cnt, acc + (blockIdx.x & (kAccSlots - 1)));
}

// Folds the accumulator slot each lane of wave 0 loaded into the step's
// min / max / count and leaves them in `out` (LDS).  No barrier: the caller
// publishes `out` with its next one.
__device__ __forceinline__ void reduce_slot_values(const StepAcc &slot, StepAccSums *out) {
  if (threadIdx.x < kWave) {
    const uint32_t mn = wave_umin(slot.min_key), mx = wave_umax(slot.max_key);
    const uint32_t n = wave_sum(slot.n_unexplored);
    if (threadIdx.x == 0) *out = StepAccSums{mn, mx, n};
  }
}

// Quantised weight of valid index l (0 past the end, for explored
// configurations and for the profiled one).  The step's s_min / s_max come
// from its accumulator slots in three stages, so a draw can overlap their
// load with its first loads: stage_load (every thread), stage_reduce (after
// the caller's own loads), then a barrier, then stage_read.
struct ScoreWeights {
  const float *s;
  uint32_t *explored;
  uint32_t n;
  uint32_t profile;
  const StepAcc *acc;
  float gamma, w_min;
  StepNorm nm{};
  StepAcc slot{};
  __device__ void stage_load() {
    if (threadIdx.x < kWave) slot = acc[threadIdx.x];
  }
  __device__ void stage_reduce(StepAccSums *sh) const { reduce_slot_values(slot, sh); }
  __device__ void stage_read(const StepAccSums *sh) {
    nm = step_norm(key_float(sh->min_key), key_float(sh->max_key), gamma, w_min);
  }
  __device__ uint32_t operator()(uint32_t l) const {
    if (l >= n) return 0u;
    return quantized_weight(s[l], explored_bit(explored, l) || l == profile, nm);
  }
  // Weights of l = first .. first + cnt - 1 (cnt <= K) into q[], 0 beyond;
  // every load is issued before the first is used.
  template <int K> __device__ void run(uint32_t first, uint32_t cnt, uint32_t (&q)[K]) const {
    float sv[K];
    uint32_t ew[K];
#pragma unroll
    for (int e = 0; e < K; ++e) {
      const uint32_t l = first + e;
      const bool in = (uint32_t)e < cnt && l < n;
      sv[e] = in ? s[l] : 0.0f;
      ew[e] = in ? explored[l >> 5] : 0xffffffffu;
    }
#pragma unroll
    for (int e = 0; e < K; ++e) {
      const uint32_t l = first + e;
      const bool ex = ((ew[e] >> (l & 31u)) & 1u) || l == profile;
      q[e] = quantized_weight(sv[e], ex, nm);
    }
  }
  __device__ void remove(uint32_t l) const { atomicOr(&explored[l >> 5], 1u << (l & 31u)); }
  __device__ uint64_t valid_of(uint32_t l) const { return l; }
  __device__ uint64_t raw_of(uint32_t l, const uint32_t *idx) const { return idx ? idx[l] : l; }
};
struct ArrayWeights {
  uint32_t *q;
  uint32_t n;
  __device__ void stage_load() {}
  __device__ void stage_reduce(StepAccSums *) const {}
  __device__ void stage_read(const StepAccSums *) {}
  __device__ uint32_t operator()(uint32_t l) const { return l < n ? q[l] : 0u; }
  template <int K> __device__ void run(uint32_t first, uint32_t cnt, uint32_t (&out)[K]) const {
#pragma unroll
    for (int e = 0; e < K; ++e) {
      const uint32_t l = first + e;
      out[e] = ((uint32_t)e < cnt && l < n) ? q[l] : 0u;
    }
  }
  __device__ void remove(uint32_t l) const { q[l] = 0u; }
  __device__ uint64_t valid_of(uint32_t l) const { return l; }
  __device__ uint64_t raw_of(uint32_t l, const uint32_t *idx) const { return idx ? idx[l] : l; }
};
// Quantised weights of a restricted step's candidates (position l in
// candidate order): drawing candidate l removes it and marks its
// configuration nb[l] explored.
struct NbWeights {
  uint32_t *q;
  const uint32_t *nb;
  uint32_t *explored;
  uint32_t n;
  __device__ void stage_load() {}
  __device__ void stage_reduce(StepAccSums *) const {}
  __device__ void stage_read(const StepAccSums *) {}
  __device__ uint32_t operator()(uint32_t l) const { return l < n ? q[l] : 0u; }
  template <int K> __device__ void run(uint32_t first, uint32_t cnt, uint32_t (&out)[K]) const {
#pragma unroll
    for (int e = 0; e < K; ++e) {
      const uint32_t l = first + e;
      out[e] = ((uint32_t)e < cnt && l < n) ? q[l] : 0u;
    }
  }
  __device__ void remove(uint32_t l) const {
    q[l] = 0u;
    atomicOr(&explored[nb[l] >> 5], 1u << (nb[l] & 31u));
  }
  __device__ uint64_t valid_of(uint32_t l) const { return nb[l]; }
  __device__ uint64_t raw_of(uint32_t l, const uint32_t *idx) const { return idx[nb[l]]; }
};

// The draw result lives in mapped, coherent pinned host memory.  The thread
// that settles a draw stores its fields with system-scope stores and then
// `seq` with a system-scope release, so a host that sees `seq` sees the
// fields (the host polls `seq` instead of waiting for the stream).
__device__ __forceinline__ void put(uint64_t *field, uint64_t v) {
  __hip_atomic_store(field, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void publish(DrawResult *res, uint64_t valid, uint64_t raw,
                                        uint64_t total, uint64_t r, uint64_t seq) {
  put(&res->valid, valid);
  put(&res->raw, raw);
  put(&res->total, total);
  put(&res->r, r);
  __hip_atomic_store(&res->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

constexpr uint32_t kNoLane = 0xffffffffu;
constexpr uint32_t kKeepWeights = 8; // weights per thread kept in registers

// One draw by one workgroup of NT threads.
//  1. Thread t owns the contiguous run of block sums [t * per, t * per + per);
//     one exclusive scan over the run totals gives Q and, for the thread
//     whose run holds r, the block b with prefix_b <= r < prefix_b + bsum_b.
//  2. Every thread takes 2^block_log2 / NT consecutive configurations of
//     block b; a second scan finds l with prefix_l <= r' < prefix_l + q_l.
// The winner removes l, subtracts q_l from bsum_b and publishes the result.
template <int NT, typename W>
__device__ void draw_body(W &wsrc, int block_log2, uint64_t *__restrict__ bsum,
                          uint32_t n_blocks, uint64_t u64, const uint32_t *__restrict__ idx,
                          DrawResult *__restrict__ res, uint64_t seq,
                          uint32_t *__restrict__ prof_out = nullptr) {
  __shared__ uint64_t scratch[NT / kWave];
  __shared__ StepAccSums sums;
  __shared__ uint32_t found_block;
  __shared__ uint64_t found_rem;
  __shared__ int picked;
  const uint32_t tid = threadIdx.x;

  wsrc.stage_load();
  const uint32_t per = (n_blocks + NT - 1) / NT;
  const uint32_t b0 = tid * per;
  const uint32_t b1 = min(n_blocks, b0 + per);
  constexpr uint32_t kChunk = 4; // block sums loaded per round trip
  uint64_t mine = 0;
  for (uint32_t c = b0; c < b1; c += kChunk) {
    uint64_t v[kChunk];
#pragma unroll
    for (uint32_t k = 0; k < kChunk; ++k) v[k] = c + k < b1 ? bsum[c + k] : 0ull;
#pragma unroll
    for (uint32_t k = 0; k < kChunk; ++k) mine += v[k];
  }
  wsrc.stage_reduce(&sums);
  if (tid == 0) picked = 0;
  uint64_t Q;
  const uint64_t pre = block_excl_scan<NT>(mine, scratch, Q); // barriers publish sums
  wsrc.stage_read(&sums);
  if (Q == 0) {
    if (tid == 0) {
      if (prof_out) *prof_out = kNoProfile;
      publish(res, kNoPick, kNoPick, 0, 0, seq);
    }
    return;
  }
  const uint64_t r = __umul64hi(u64, Q);
  if (mine != 0 && pre <= r && r < pre + mine) {
    uint64_t run = pre;
    bool hit = false;
    for (uint32_t c = b0; c < b1 && !hit; c += kChunk) {
      uint64_t v[kChunk];
#pragma unroll
      for (uint32_t k = 0; k < kChunk; ++k) v[k] = c + k < b1 ? bsum[c + k] : 0ull;
#pragma unroll
      for (uint32_t k = 0; k < kChunk; ++k) {
        if (!hit && r < run + v[k]) {
          found_block = c + k;
          found_rem = r - run;
          hit = true;
        }
        run += v[k];
      }
    }
  }
  __syncthreads();
  const uint32_t blk = found_block;
  const uint64_t rem = found_rem;

  // 2^block_log2 / NT >= 4 consecutive configurations per thread, weighed in
  // chunks of kKeepWeights (the first chunk stays in registers)
  const uint32_t per2 = (1u << block_log2) / NT;
  const uint32_t first = (blk << block_log2) + tid * per2;
  uint32_t qk[kKeepWeights];
  wsrc.run(first, min(per2, kKeepWeights), qk);
  uint64_t mine2 = 0;
#pragma unroll
  for (uint32_t e = 0; e < kKeepWeights; ++e) mine2 += qk[e];
  for (uint32_t c = kKeepWeights; c < per2; c += kKeepWeights) {
    uint32_t t[kKeepWeights];
    wsrc.run(first + c, min(per2 - c, kKeepWeights), t);
#pragma unroll
    for (uint32_t e = 0; e < kKeepWeights; ++e) mine2 += t[e];
  }
  uint64_t blk_total;
  const uint64_t pre2 = block_excl_scan<NT>(mine2, scratch, blk_total);
  if (mine2 != 0 && pre2 <= rem && rem < pre2 + mine2) {
    uint32_t l = kNoLane, ql = 0;
    uint64_t run = pre2;
#pragma unroll
    for (uint32_t e = 0; e < kKeepWeights; ++e) {
      if (l == kNoLane && rem < run + qk[e]) {
        l = first + e;
        ql = qk[e];
      }
      run += qk[e];
    }
    for (uint32_t c = kKeepWeights; l == kNoLane && c < per2; c += kKeepWeights) {
      uint32_t t[kKeepWeights];
      wsrc.run(first + c, min(per2 - c, kKeepWeights), t);
#pragma unroll
      for (uint32_t e = 0; e < kKeepWeights; ++e) {
        if (l == kNoLane && rem < run + t[e]) {
          l = first + e + c;
          ql = t[e];
        }
        run += t[e];
      }
    }
    if (l != kNoLane) {
      wsrc.remove(l);
      bsum[blk] -= ql;
      picked = 1;
      if (prof_out) *prof_out = (uint32_t)wsrc.valid_of(l);
      publish(res, wsrc.valid_of(l), wsrc.raw_of(l, idx), Q, r, seq);
    }
  }
  __syncthreads();
  // no pick although Q > 0: the block sums disagree with the weights
  if (tid == 0 && !picked) {
    if (prof_out) *prof_out = kNoProfile;
    publish(res, kNoPick, kNoPick, Q, r, seq);
  }
}

// Sum of the quantised weights of block `blk` (2^block_log2 configurations),
// returned to every thread.  The step's accumulator slots and the block's
// first 4096 scores are loaded together; s_min / s_max are known once both
// have arrived.
__device__ __forceinline__ uint64_t weight_block_sum(const float *__restrict__ s,
                                                     const uint32_t *__restrict__ explored,
                                                     uint32_t n_valid, uint32_t profile,
                                                     const StepAcc *__restrict__ acc, float gamma,
                                                     float w_min, int block_log2, uint32_t blk) {
  __shared__ uint64_t scratch[kWeightThreads / kWave];
  __shared__ StepAccSums sums;
  constexpr uint32_t kRound = 16u * kWeightThreads; // 4 float4 per thread
  const uint32_t base = blk << block_log2;
  const uint32_t end = min(n_valid, base + (1u << block_log2));
  StepAcc slot{};
  if (threadIdx.x < kWave) slot = acc[threadIdx.x];
  float4 sv[4];
  uint32_t ex[4];
  auto load_round = [&](uint32_t r0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t l0 = r0 + 4u * (threadIdx.x + k * kWeightThreads);
      if (l0 < end) {
        sv[k] = *reinterpret_cast<const float4 *>(s + l0);
        ex[k] = explored[l0 >> 5];
      } else { // past the block: weight 0, like explored configurations
        sv[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        ex[k] = 0xffffffffu;
      }
    }
  };
  load_round(base);
  reduce_slot_values(slot, &sums);
  __syncthreads();
  const StepNorm nm = step_norm(key_float(sums.min_key), key_float(sums.max_key), gamma, w_min);
  // the choice of division path is made once per block, outside the loop
  auto weigh = [&](auto wide) {
    uint64_t sum = 0;
    for (uint32_t r0 = base;;) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        // no per-configuration branches: positions past the end (and the
        // profiled configuration) count as explored and weigh 0
        const uint32_t l0 = r0 + 4u * (threadIdx.x + k * kWeightThreads);
        uint32_t ex4 = (ex[k] >> (l0 & 31u)) & 0xfu;
        const uint32_t tail = end - l0;
        if (tail < 4u) ex4 |= (0xfu << tail) & 0xfu;
        if (profile - l0 < 4u) ex4 |= 1u << (profile - l0);
        const float ss[4] = {sv[k].x, sv[k].y, sv[k].z, sv[k].w};
#pragma unroll
        for (int e = 0; e < 4; ++e)
          sum += quantized_weight_t<decltype(wide)::value>(ss[e], (ex4 >> e) & 1u, nm);
      }
      r0 += kRound;
      if (r0 >= end) break;
      load_round(r0);
    }
    return sum;
  };
  const uint64_t sum = nm.wide ? weigh(std::true_type{}) : weigh(std::false_type{});
  return block_sum<kWeightThreads>(sum, scratch); // its barriers also retire `sums`
}

__device__ __forceinline__ void clear_acc(StepAcc *acc_next) {
  if (threadIdx.x < kAccSlots) {
    acc_next[threadIdx.x].min_key = 0xffffffffu;
    acc_next[threadIdx.x].max_key = 0u;
    acc_next[threadIdx.x].n_unexplored = 0u;
  }
}

// One workgroup per block of 2^block_log2 configurations: block sums of q.
__global__ __launch_bounds__(kWeightThreads) void weight_pass(
    const float *__restrict__ s, const uint32_t *__restrict__ explored, uint32_t n_valid,
    uint32_t profile, const uint32_t *__restrict__ prof_dev, const StepAcc *__restrict__ acc,
    StepAcc *__restrict__ acc_next, float gamma, float w_min, int block_log2,
    uint64_t *__restrict__ bsum) {
  if (prof_dev) profile = *prof_dev;
  if (blockIdx.x == 0) clear_acc(acc_next); // the next step's accumulators
  const uint64_t total = weight_block_sum(s, explored, n_valid, profile, acc, gamma, w_min,
                                          block_log2, blockIdx.x);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// One draw.  `profile` (or kNoProfile; read from prof_dev when given) is
// excluded and, when `mark_profile`, marked explored once the draw is done.
// With prof_out, the pick's valid index (kNoProfile when there is none) is
// also stored there for the next step.
__global__ __launch_bounds__(kDrawThreads) void draw_scores(
    const float *__restrict__ s, uint32_t *__restrict__ explored, uint32_t n_valid,
    uint32_t profile, const uint32_t *__restrict__ prof_dev, int mark_profile,
    const StepAcc *__restrict__ acc, float gamma, float w_min, int block_log2,
    uint64_t *__restrict__ bsum, uint32_t n_blocks, uint64_t u64,
    const uint32_t *__restrict__ idx, DrawResult *__restrict__ res, uint64_t seq,
    uint32_t *__restrict__ prof_out) {
  if (prof_dev) profile = *prof_dev;
  ScoreWeights w{s, explored, n_valid, profile, acc, gamma, w_min};
  draw_body<kDrawThreads>(w, block_log2, bsum, n_blocks, u64, idx, res, seq, prof_out);
  __syncthreads();
  if (threadIdx.x == 0 && mark_profile && profile < n_valid)
    atomicOr(&explored[profile >> 5], 1u << (profile & 31u));
}

// Further draws of one step (after its first), made one after another by
// one workgroup, each removing its pick before the next exactly as separate
// launches of draw_scores would: draw i uses u64[i] and publishes into
// res[i] under sequence number seq0 + i.
__global__ __launch_bounds__(kDrawThreads) void draw_many(
    const float *__restrict__ s, uint32_t *__restrict__ explored, uint32_t n_valid,
    const StepAcc *__restrict__ acc, float gamma, float w_min, int block_log2,
    uint64_t *__restrict__ bsum, uint32_t n_blocks, DrawSeries series,
    const uint32_t *__restrict__ idx, DrawResult *__restrict__ res, uint64_t seq0) {
  for (int i = 0; i < series.n; ++i) {
    ScoreWeights w{s, explored, n_valid, kNoProfile, acc, gamma, w_min};
    draw_body<kDrawThreads>(w, block_log2, bsum, n_blocks, series.u64[i], idx, res + i,
                            seq0 + (uint64_t)i);
    __syncthreads(); // the pick's removal is seen by the next draw
  }
}

// ------------------------------------------------------------ batched
// Score tiles of every session, grid-stride over the concatenated tile list;
// a workgroup flushes its accumulators whenever the session changes.
// RIF: counter rows in flight per thread; WPE: waves per SIMD the compiler
// plans registers for (the autotuner's variants).
template <int RIF, int WPE>
__global__ __launch_bounds__(kScoreThreads)
__attribute__((amdgpu_waves_per_eu(WPE, 8))) void batch_score(const BatchSess *__restrict__ sess,
                                                              const BatchStep *__restrict__ step,
                                                              const uint16_t *__restrict__ tile_sess,
                                                              uint32_t total_tiles) {
  uint32_t kmin = 0xffffffffu, kmax = 0u, cnt = 0u;
  uint32_t cur = 0xffffffffu;
  for (uint32_t t = blockIdx.x; t < total_tiles; t += gridDim.x) {
    const uint32_t si = tile_sess[t];
    if (si != cur) {
      if (cur != 0xffffffffu)
        flush_acc(kmin, kmax, cnt,
                  sess[cur].acc + step[cur].parity * kAccSlots + (blockIdx.x & (kAccSlots - 1)));
      kmin = 0xffffffffu;
      kmax = 0u;
      cnt = 0u;
      cur = si;
    }
    const BatchSess &d = sess[si];
    const BatchStep &st = step[si];
    const int n = st.profile < d.n_valid ? st.n_act : 0;
    score_tile<RIF>(d.P, d.stride, st.profile, n, st.ctr, st.delta, d.explored, d.n_valid, d.s,
               t - d.tile0, kmin, kmax, cnt);
  }
  if (cur != 0xffffffffu)
    flush_acc(kmin, kmax, cnt,
              sess[cur].acc + step[cur].parity * kAccSlots + (blockIdx.x & (kAccSlots - 1)));
}

// Weight blocks of every session, grid-stride over the concatenated block list.
__global__ __launch_bounds__(kWeightThreads) void batch_weight(
    const BatchSess *__restrict__ sess, const BatchStep *__restrict__ step,
    const uint16_t *__restrict__ blk_sess, uint32_t total_blocks) {
  for (uint32_t b = blockIdx.x; b < total_blocks; b += gridDim.x) {
    const uint32_t si = blk_sess[b];
    const BatchSess &d = sess[si];
    const BatchStep &st = step[si];
    const uint32_t lb = b - d.blk0;
    if (lb == 0) clear_acc(d.acc + (st.parity ^ 1) * kAccSlots);
    const uint64_t total =
        weight_block_sum(d.s, d.explored, d.n_valid, st.profile, d.acc + st.parity * kAccSlots,
                         d.gamma, d.w_min, d.block_log2, lb);
    if (threadIdx.x == 0) d.bsum[lb] = total;
  }
}

// One workgroup per session: its draw, then its profile is marked explored.
__global__ __launch_bounds__(kDrawThreads) void batch_draw(const BatchSess *__restrict__ sess,
                                                           const BatchStep *__restrict__ step) {
  const BatchSess &d = sess[blockIdx.x];
  const BatchStep &st = step[blockIdx.x];
  if (!st.draw) return;
  ScoreWeights w{d.s, d.explored, d.n_valid, st.profile, d.acc + st.parity * kAccSlots, d.gamma,
                 d.w_min};
  draw_body<kDrawThreads>(w, d.block_log2, d.bsum, d.n_blocks, st.u64, d.idx, d.res, st.seq);
  __syncthreads();
  if (threadIdx.x == 0 && st.profile < d.n_valid)
    atomicOr(&d.explored[st.profile >> 5], 1u << (st.profile & 31u));
}

// ------------------------------------------------------------ neighbourhood
// The restricted step scores only candidates near the profiled configuration:
// one thread per candidate (before filtering) unranks it, keeps it if it is
// valid and unexplored, and scores it with the float32 chain of the full
// pass; one workgroup then compacts the kept candidates in candidate order,
// quantises their weights over the kept set and forms the block sums.
constexpr int kNbThreads = 256;
constexpr uint32_t kNbMaxSubsets = 32 + 32 * 31 / 2 + 32 * 31 * 30 / 6; // radius <= 3

__global__ __launch_bounds__(kNbThreads) void nb_score(
    NbStep st, const uint32_t *__restrict__ sub_off, const uint32_t *__restrict__ sub_code,
    const uint32_t *__restrict__ mask, const uint32_t *__restrict__ rank,
    const uint32_t *__restrict__ explored, const float *__restrict__ P, uint64_t stride,
    uint32_t *__restrict__ tmp_idx, float *__restrict__ tmp_s, StepAcc *__restrict__ acc) {
  __shared__ uint32_t off_lds[kNbMaxSubsets + 1];
  __shared__ float a_lds[CGS_MAX_COUNTERS];
  for (uint32_t i = threadIdx.x; i <= st.n_subsets; i += kNbThreads) off_lds[i] = sub_off[i];
  if (threadIdx.x < (uint32_t)st.act.n)
    a_lds[threadIdx.x] = P[(size_t)st.act.ctr[threadIdx.x] * stride + st.profile];
  __syncthreads();
  uint32_t kmin = 0xffffffffu, kmax = 0u, cnt = 0u;
  const uint32_t f = blockIdx.x * kNbThreads + threadIdx.x;
  if (f < st.total) {
    // subset holding candidate f: the last one whose first candidate <= f
    uint32_t lo = 0, hi = st.n_subsets;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (off_lds[mid] <= f) lo = mid;
      else hi = mid;
    }
    const uint32_t code = sub_code[lo];
    uint32_t u = f - off_lds[lo];
    int64_t raw = st.profile_raw;
    // new digits of the changed parameters, the last one fastest; the
    // profile's own digit is skipped
    for (int k = (int)(code >> 24) - 1; k >= 0; --k) {
      const uint32_t j = (code >> (8 * k)) & 0xffu;
      const uint32_t alt = st.radix[j] - 1u;
      const uint32_t a = u % alt;
      u /= alt;
      const uint32_t pd = st.pdig[j];
      const uint32_t v = a < pd ? a : a + 1u;
      raw += ((int64_t)v - (int64_t)pd) * (int64_t)st.stride[j];
    }
    const uint32_t rw = (uint32_t)raw;
    const uint32_t word = mask[rw >> 5], rk = rank[rw >> 5];
    bool keep = (word >> (rw & 31u)) & 1u;
    uint32_t l = 0;
    if (keep) {
      l = rk + (uint32_t)__popc(word & ((1u << (rw & 31u)) - 1u));
      keep = !((explored[l >> 5] >> (l & 31u)) & 1u);
    }
    float s = 0.0f;
    if (keep) {
      for (int j0 = 0; j0 < st.act.n; j0 += kRowsInFlight) {
        float x[kRowsInFlight];
#pragma unroll
        for (int u2 = 0; u2 < kRowsInFlight; ++u2)
          if (j0 + u2 < st.act.n) x[u2] = P[(size_t)st.act.ctr[j0 + u2] * stride + l];
#pragma unroll
        for (int u2 = 0; u2 < kRowsInFlight; ++u2) {
          if (j0 + u2 < st.act.n && a_lds[j0 + u2] != 0.0f) {
            const float ap = a_lds[j0 + u2];
            const float t = (x[u2] - ap) / (ap + x[u2]);
            s = (x[u2] != 0.0f) ? s + st.act.delta[j0 + u2] * t : s;
          }
        }
      }
      const uint32_t k = float_key(s);
      kmin = k;
      kmax = k;
      cnt = 1;
    }
    tmp_idx[f] = keep ? l : 0xffffffffu;
    tmp_s[f] = s;
  }
  flush_acc(kmin, kmax, cnt, acc + (blockIdx.x & (kAccSlots - 1)));
}

constexpr int kNbFinishThreads = 1024;

__global__ __launch_bounds__(kNbFinishThreads) void nb_finish(
    uint32_t total, const uint32_t *__restrict__ tmp_idx, const float *__restrict__ tmp_s,
    StepAcc *__restrict__ acc, float gamma, float w_min, uint32_t *__restrict__ nb_idx,
    float *__restrict__ nb_s, uint32_t *__restrict__ nb_q, uint64_t *__restrict__ nb_bsum,
    NbStats *__restrict__ stats) {
  constexpr uint32_t kChunk = 8;
  __shared__ uint64_t scratch[kNbFinishThreads / kWave];
  __shared__ StepAccSums sums;
  __shared__ unsigned long long bsum_lds[kNbBlocks];
  const uint32_t tid = threadIdx.x;
  StepAcc slot{};
  if (tid < kWave) slot = acc[tid];
  if (tid < kNbBlocks) bsum_lds[tid] = 0ull;
  const uint32_t per = (total + kNbFinishThreads - 1) / kNbFinishThreads;
  const uint32_t f0 = min(total, tid * per), f1 = min(total, f0 + per);
  uint32_t kept = 0;
  for (uint32_t f = f0; f < f1; f += kChunk) {
    uint32_t v[kChunk];
#pragma unroll
    for (uint32_t k = 0; k < kChunk; ++k) v[k] = f + k < f1 ? tmp_idx[f + k] : 0xffffffffu;
#pragma unroll
    for (uint32_t k = 0; k < kChunk; ++k) kept += v[k] != 0xffffffffu;
  }
  reduce_slot_values(slot, &sums);
  uint64_t count;
  uint64_t pos = block_excl_scan<kNbFinishThreads>(kept, scratch, count); // barriers publish sums
  const StepNorm nm = step_norm(key_float(sums.min_key), key_float(sums.max_key), gamma, w_min);
  for (uint32_t f = f0; f < f1; f += kChunk) {
    uint32_t v[kChunk];
    float sv[kChunk];
#pragma unroll
    for (uint32_t k = 0; k < kChunk; ++k) {
      v[k] = f + k < f1 ? tmp_idx[f + k] : 0xffffffffu;
      sv[k] = f + k < f1 ? tmp_s[f + k] : 0.0f;
    }
#pragma unroll
    for (uint32_t k = 0; k < kChunk; ++k) {
      if (v[k] == 0xffffffffu) continue;
      const uint32_t q = quantized_weight(sv[k], false, nm);
      nb_idx[pos] = v[k];
      nb_s[pos] = sv[k];
      nb_q[pos] = q;
      atomicAdd(&bsum_lds[pos >> kNbBlockLog2], (unsigned long long)q);
      ++pos;
    }
  }
  __syncthreads();
  if (tid < kNbBlocks) nb_bsum[tid] = bsum_lds[tid];
  if (tid == 0) {
    uint64_t q_total = 0;
    for (uint32_t b = 0; b < kNbBlocks; ++b) q_total += bsum_lds[b];
    stats->count = (uint32_t)count;
    stats->total = q_total;
    stats->min_key = sums.min_key;
    stats->max_key = sums.max_key;
  }
  clear_acc(acc); // every slot was read before the scan's barriers
}

__global__ __launch_bounds__(kDrawThreads) void nb_draw(
    uint32_t *__restrict__ q, const uint32_t *__restrict__ nb, const NbStats *__restrict__ stats,
    uint64_t *__restrict__ bsum, uint32_t *__restrict__ explored, uint32_t profile,
    int mark_profile, uint32_t n_valid, uint64_t u64, const uint32_t *__restrict__ idx,
    DrawResult *__restrict__ res, uint64_t seq) {
  NbWeights w{q, nb, explored, stats->count};
  draw_body<kDrawThreads>(w, kNbBlockLog2, bsum, kNbBlocks, u64, idx, res, seq);
  __syncthreads();
  if (threadIdx.x == 0 && mark_profile && profile < n_valid)
    atomicOr(&explored[profile >> 5], 1u << (profile & 31u));
}

// Marks the profiled configuration explored (a step read without a draw).
__global__ __launch_bounds__(64) void mark_one(uint32_t *__restrict__ explored, uint32_t l,
                                               uint32_t n_valid) {
  if (threadIdx.x == 0 && l < n_valid) atomicOr(&explored[l >> 5], 1u << (l & 31u));
}

__global__ __launch_bounds__(kDrawThreads) void draw_array(uint32_t *__restrict__ q, uint32_t n,
                                                           int block_log2,
                                                           uint64_t *__restrict__ bsum,
                                                           uint32_t n_blocks, uint64_t u64,
                                                           DrawResult *__restrict__ res) {
  ArrayWeights w{q, n};
  draw_body<kDrawThreads>(w, block_log2, bsum, n_blocks, u64, nullptr, res, 1);
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
  const StepAccSums a = reduce_slots(acc);
  const uint32_t i = blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  ScoreWeights w{s, explored, n_valid, kNoProfile, acc, gamma, w_min};
  w.nm = step_norm(key_float(a.min_key), key_float(a.max_key), gamma, w_min);
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
                             uint32_t n_valid, float *d_s, StepAcc *d_acc, hipStream_t stream,
                             const uint32_t *d_prof) {
  const uint32_t n_tiles = (n_valid + 4u * kScoreThreads - 1) / (4u * kScoreThreads);
  const uint32_t grid = std::min<uint32_t>(n_tiles, kScoreGrid);
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(score_pass, dim3(grid), dim3(kScoreThreads), 0, stream, d_P, stride, profile,
                     d_prof, act, d_explored, n_valid, d_s, d_acc);
  return hipGetLastError();
}

hipError_t launch_weight_pass(const float *d_s, const uint32_t *d_explored, uint32_t n_valid,
                              uint32_t profile, const StepAcc *d_acc, StepAcc *d_acc_next,
                              float gamma, float w_min, int block_log2, uint64_t *d_bsum,
                              uint32_t n_blocks, hipStream_t stream, const uint32_t *d_prof) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(weight_pass, dim3(n_blocks), dim3(kWeightThreads), 0, stream, d_s, d_explored,
                     n_valid, profile, d_prof, d_acc, d_acc_next, gamma, w_min, block_log2,
                     d_bsum);
  return hipGetLastError();
}

hipError_t launch_draw(const float *d_s, uint32_t *d_explored, uint32_t n_valid, uint32_t profile,
                       bool mark_profile, const StepAcc *d_acc, float gamma, float w_min,
                       int block_log2, uint64_t *d_bsum, uint32_t n_blocks, uint64_t u64,
                       const uint32_t *d_idx, DrawResult *d_res, uint64_t seq,
                       hipStream_t stream, const uint32_t *d_prof, uint32_t *d_prof_out) {
  hipLaunchKernelGGL(draw_scores, dim3(1), dim3(kDrawThreads), 0, stream, d_s, d_explored, n_valid,
                     profile, d_prof, mark_profile ? 1 : 0, d_acc, gamma, w_min, block_log2,
                     d_bsum, n_blocks, u64, d_idx, d_res, seq, d_prof_out);
  return hipGetLastError();
}

hipError_t launch_draw_many(const float *d_s, uint32_t *d_explored, uint32_t n_valid,
                            const StepAcc *d_acc, float gamma, float w_min, int block_log2,
                            uint64_t *d_bsum, uint32_t n_blocks, const DrawSeries &series,
                            const uint32_t *d_idx, DrawResult *d_res, uint64_t seq0,
                            hipStream_t stream) {
  if (series.n < 1 || series.n > kMaxDrawSeries) return hipErrorInvalidValue;
  hipLaunchKernelGGL(draw_many, dim3(1), dim3(kDrawThreads), 0, stream, d_s, d_explored, n_valid,
                     d_acc, gamma, w_min, block_log2, d_bsum, n_blocks, series, d_idx, d_res,
                     seq0);
  return hipGetLastError();
}

hipError_t launch_batch_score(const BatchSess *d_sess, const BatchStep *d_step,
                              const uint16_t *d_tile_sess, uint32_t total_tiles, uint32_t grid,
                              int variant, hipStream_t stream) {
  if (total_tiles == 0 || grid == 0) return hipSuccess;
#define CGS_BATCH_SCORE(RIF, WPE)                                                               \
  hipLaunchKernelGGL((batch_score<RIF, WPE>), dim3(grid), dim3(kScoreThreads), 0, stream,      \
                     d_sess, d_step, d_tile_sess, total_tiles)
  switch (variant) {
  case 1: CGS_BATCH_SCORE(4, 4); break;
  case 2: CGS_BATCH_SCORE(16, 2); break;
  case 3: CGS_BATCH_SCORE(8, 4); break;
  case 4: CGS_BATCH_SCORE(4, 8); break;
  default: CGS_BATCH_SCORE(8, 1); break; // the unconstrained kernel
  }
#undef CGS_BATCH_SCORE
  return hipGetLastError();
}

hipError_t launch_batch_weight(const BatchSess *d_sess, const BatchStep *d_step,
                               const uint16_t *d_blk_sess, uint32_t total_blocks, uint32_t grid,
                               hipStream_t stream) {
  if (total_blocks == 0 || grid == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_weight, dim3(grid), dim3(kWeightThreads), 0, stream, d_sess, d_step,
                     d_blk_sess, total_blocks);
  return hipGetLastError();
}

hipError_t launch_batch_draw(const BatchSess *d_sess, const BatchStep *d_step, uint32_t n_sess,
                             hipStream_t stream) {
  if (n_sess == 0) return hipSuccess;
  hipLaunchKernelGGL(batch_draw, dim3(n_sess), dim3(kDrawThreads), 0, stream, d_sess, d_step);
  return hipGetLastError();
}

hipError_t launch_mark_one(uint32_t *d_explored, uint32_t l, uint32_t n_valid,
                           hipStream_t stream) {
  hipLaunchKernelGGL(mark_one, dim3(1), dim3(64), 0, stream, d_explored, l, n_valid);
  return hipGetLastError();
}

hipError_t launch_nb_score(const NbStep &st, const uint32_t *d_sub_off, const uint32_t *d_sub_code,
                           const uint32_t *d_mask, const uint32_t *d_rank,
                           const uint32_t *d_explored, const float *d_P, uint64_t stride,
                           uint32_t *d_tmp_idx, float *d_tmp_s, StepAcc *d_nb_acc,
                           hipStream_t stream) {
  if (st.total == 0 || st.total > kNbMaxCandidates || st.n_subsets > kNbMaxSubsets)
    return hipErrorInvalidValue;
  const uint32_t grid = (st.total + kNbThreads - 1) / kNbThreads;
  hipLaunchKernelGGL(nb_score, dim3(grid), dim3(kNbThreads), 0, stream, st, d_sub_off, d_sub_code,
                     d_mask, d_rank, d_explored, d_P, stride, d_tmp_idx, d_tmp_s, d_nb_acc);
  return hipGetLastError();
}

hipError_t launch_nb_finish(uint32_t total, const uint32_t *d_tmp_idx, const float *d_tmp_s,
                            StepAcc *d_nb_acc, float gamma, float w_min, uint32_t *d_nb_idx,
                            float *d_nb_s, uint32_t *d_nb_q, uint64_t *d_nb_bsum,
                            NbStats *d_stats, hipStream_t stream) {
  if (total > kNbMaxCandidates) return hipErrorInvalidValue;
  hipLaunchKernelGGL(nb_finish, dim3(1), dim3(kNbFinishThreads), 0, stream, total, d_tmp_idx,
                     d_tmp_s, d_nb_acc, gamma, w_min, d_nb_idx, d_nb_s, d_nb_q, d_nb_bsum,
                     d_stats);
  return hipGetLastError();
}

hipError_t launch_nb_draw(uint32_t *d_nb_q, const uint32_t *d_nb_idx, const NbStats *d_stats,
                          uint64_t *d_nb_bsum, uint32_t *d_explored, uint32_t profile,
                          int mark_profile, uint32_t n_valid, uint64_t u64, const uint32_t *d_idx,
                          DrawResult *d_res, uint64_t seq, hipStream_t stream) {
  hipLaunchKernelGGL(nb_draw, dim3(1), dim3(kDrawThreads), 0, stream, d_nb_q, d_nb_idx, d_stats,
                     d_nb_bsum, d_explored, profile, mark_profile, n_valid, u64, d_idx, d_res, seq);
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
