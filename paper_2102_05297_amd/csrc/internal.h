// Internal types shared by the host runtime and the kernels of libcgs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cgs.h"

namespace cgs {

// Division by a run-time invariant 32-bit divisor d, exact for every 32-bit
// dividend: Granlund & Montgomery, "Division by invariant integers using
// multiplication" (PLDI 1994), Fig. 4.1.  With l = ceil(log2 d),
// m = floor(2^32 (2^l - d) / d) + 1, sh1 = min(l, 1), sh2 = max(l - 1, 0):
//   t = mulhi(m, n);  q = (t + ((n - t) >> sh1)) >> sh2.
struct FastDiv {
  uint32_t m;
  uint32_t sh; // sh1 | sh2 << 8
};

// Space description, resident in device memory (one per space).
// Parameter j's value for digit d is table[j * CGS_MAX_RADIX + d].
struct SpaceDev {
  int32_t n_params;
  int32_t n_cons;
  uint32_t n_raw;
  uint32_t n_words; // ceil(n_raw / 32)
  uint32_t radix[CGS_MAX_PARAMS];
  FastDiv div[CGS_MAX_PARAMS];
  uint32_t cons_code[CGS_MAX_CONSTRAINTS]; // kind | a << 8 | b << 16 | c << 24
  int64_t cons_bound[CGS_MAX_CONSTRAINTS];
  int32_t table[CGS_MAX_PARAMS * CGS_MAX_RADIX];
};

// Counters that enter one step's score: Table positions with dpc != 0,
// ascending.  Passed by value to the score kernel.
struct ActiveCounters {
  int32_t n;
  int32_t pad;
  uint32_t ctr[CGS_MAX_COUNTERS];
  float delta[CGS_MAX_COUNTERS];
};

// Per-step accumulators written by the kernels (device memory): one of
// kAccSlots slots per score workgroup, combined by the readers.
struct StepAcc {
  uint32_t min_key;    // order-preserving key of s_min over unexplored
  uint32_t max_key;    // ... of s_max
  uint32_t n_unexplored;
  uint32_t pad;
};
struct StepAccSums {
  uint32_t min_key, max_key, n_unexplored;
};
constexpr int kAccSlots = 64;

// Result of one draw (device memory, copied to pinned host memory).
struct DrawResult {
  uint64_t valid;  // picked valid index, or ~0 when the total weight is 0
  uint64_t raw;    // its raw index
  uint64_t total;  // Q at this draw
  uint64_t r;      // floor(U * Q / 2^64)
  uint64_t seq;    // sequence number of the draw, stored last (release)
};

constexpr uint64_t kNoPick = ~0ull;
constexpr uint32_t kNoProfile = ~0u; // step prologue: no configuration to mark

// ---- neighbourhood-restricted steps
// Candidates are the configurations that differ from the profiled one in
// 1..radius parameters, ordered by the set of changed parameters (a table of
// subsets in that order, with the offset of each subset's first candidate)
// and then by the new digits.  Arguments of one step, by value.
constexpr uint32_t kNbMaxCandidates = 65536;
constexpr int kNbBlockLog2 = 12;
constexpr uint32_t kNbBlocks = kNbMaxCandidates >> kNbBlockLog2;
struct NbStep {
  uint32_t profile_raw;
  uint32_t profile;  // valid index of the profiled configuration
  uint32_t total;    // candidates before filtering
  uint32_t n_subsets;
  uint32_t stride[CGS_MAX_PARAMS]; // raw place values
  uint8_t radix[CGS_MAX_PARAMS];
  uint8_t pdig[CGS_MAX_PARAMS];    // the profile's digits
  ActiveCounters act;
};
// Per-step results of the restricted step (device memory).
struct NbStats {
  uint32_t count;    // candidates kept (valid, unexplored)
  uint32_t pad;
  uint64_t total;    // sum of their quantised weights
  uint32_t min_key, max_key;
};

// ---- batched sessions: one descriptor per session (device memory) and one
// step record per session (refreshed from pinned memory before each step)
struct BatchSess {
  const float *P;
  uint64_t stride;
  uint32_t *explored;
  float *s;
  uint64_t *bsum;
  StepAcc *acc; // 2 sets of kAccSlots
  const uint32_t *idx;
  DrawResult *res;
  uint32_t n_valid, n_blocks;
  int32_t block_log2;
  uint32_t tile0, blk0; // first global score tile / weight block of the session
  float gamma, w_min;
  uint32_t pad;
};
struct BatchStep {
  uint32_t profile; // valid index, kNoProfile for none
  int32_t n_act;
  int32_t parity;   // accumulator set of this step
  int32_t draw;     // 0: score and weigh only (timing)
  uint64_t u64;
  uint64_t seq;     // sequence number the draw publishes
  uint32_t ctr[CGS_MAX_COUNTERS];
  float delta[CGS_MAX_COUNTERS];
};
constexpr uint32_t kBatchTile = 1024; // configurations per score tile

// variant: 0..kBatchScoreVariants-1, counter rows in flight x waves per SIMD
// (0: 8 rows, unconstrained; 1: 4 rows, 4 waves; 2: 16 rows, 2 waves;
// 3: 8 rows, 4 waves; 4: 4 rows, 8 waves)
constexpr int kBatchScoreVariants = 5;
hipError_t launch_batch_score(const BatchSess *d_sess, const BatchStep *d_step,
                              const uint16_t *d_tile_sess, uint32_t total_tiles, uint32_t grid,
                              int variant, hipStream_t stream);
hipError_t launch_batch_weight(const BatchSess *d_sess, const BatchStep *d_step,
                               const uint16_t *d_blk_sess, uint32_t total_blocks, uint32_t grid,
                               hipStream_t stream);
hipError_t launch_batch_draw(const BatchSess *d_sess, const BatchStep *d_step, uint32_t n_sess,
                             hipStream_t stream);

// ---- perceptron surrogate
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;

// F inputs (one per parameter, padded to K1 = 16 or 32), H hidden units per
// layer (64, 128, 256 or 512), C outputs (padded to 32 or 64).
struct MlpShape {
  int F, H, C, K1;
};

struct MlpFwdArgs {
  const SpaceDev *sp;
  const uint32_t *idx;     // valid raw indices
  uint32_t n;
  int F, H, C, K1, n_cu;
  const bf16x8 *w1p, *w2p, *w3p;
  const float *b1, *b2, *b3;
  float *P;
  uint64_t stride;
};

hipError_t launch_mlp_forward(const MlpFwdArgs &a, bool train, hipStream_t stream);

// ---- launchers (each enqueues on `stream`; return hipSuccess or an error)
hipError_t launch_enumeration(const SpaceDev *d_space, uint32_t n_raw, uint32_t *d_mask,
                              uint32_t *d_tile_count, uint32_t *d_tile_off, uint64_t *d_total,
                              uint32_t *d_idx, uint32_t *d_rank, int phase, hipStream_t stream);
uint32_t enumeration_tiles(uint32_t n_raw);

hipError_t launch_forest_eval(const SpaceDev *d_space, const uint32_t *d_idx, uint32_t n_valid,
                              const uint16_t *d_nodes, const float *d_leaves, int n_trees,
                              int depth, int n_counters, float *d_P, uint64_t stride,
                              uint16_t *d_leaf_out, uint32_t leaf_first, uint32_t leaf_count,
                              hipStream_t stream);

hipError_t launch_gather_rows(const float *P, uint64_t stride, int n_counters,
                              const uint32_t *d_idx, uint32_t n, float *d_out,
                              hipStream_t stream);
hipError_t launch_sq_diff(const float *Pa, const float *Pb, uint64_t stride_a, uint64_t stride_b,
                          int n_counters, const uint32_t *sample, uint32_t n, double *partial,
                          uint32_t grid, hipStream_t stream);
hipError_t launch_reset_acc(StepAcc *d_acc, int n, hipStream_t stream);
// The step's kernels take the profiled configuration's valid index either
// as `profile` or, when d_prof is given, from device memory (the previous
// draw's d_prof_out), so steps can be enqueued before the pick they profile
// is known on the host.
hipError_t launch_score_pass(const float *d_P, uint64_t stride, uint32_t profile,
                             const ActiveCounters &act, const uint32_t *d_explored,
                             uint32_t n_valid, float *d_s, StepAcc *d_acc, hipStream_t stream,
                             const uint32_t *d_prof = nullptr);
hipError_t launch_weight_pass(const float *d_s, const uint32_t *d_explored, uint32_t n_valid,
                              uint32_t profile, const StepAcc *d_acc, StepAcc *d_acc_next,
                              float gamma, float w_min, int block_log2, uint64_t *d_bsum,
                              uint32_t n_blocks, hipStream_t stream,
                              const uint32_t *d_prof = nullptr);
// The draw stores its result, then `seq` with a system-scope release; with
// d_prof_out also the pick's valid index (kNoProfile without a pick).
// Up to kMaxDrawSeries further draws of one step in one launch (draw_many).
constexpr int kMaxDrawSeries = 32;
struct DrawSeries {
  int32_t n;
  int32_t pad;
  uint64_t u64[kMaxDrawSeries];
};
hipError_t launch_draw_many(const float *d_s, uint32_t *d_explored, uint32_t n_valid,
                            const StepAcc *d_acc, float gamma, float w_min, int block_log2,
                            uint64_t *d_bsum, uint32_t n_blocks, const DrawSeries &series,
                            const uint32_t *d_idx, DrawResult *d_res, uint64_t seq0,
                            hipStream_t stream);
hipError_t launch_draw(const float *d_s, uint32_t *d_explored, uint32_t n_valid, uint32_t profile,
                       bool mark_profile, const StepAcc *d_acc, float gamma, float w_min,
                       int block_log2, uint64_t *d_bsum, uint32_t n_blocks, uint64_t u64,
                       const uint32_t *d_idx, DrawResult *d_res, uint64_t seq,
                       hipStream_t stream, const uint32_t *d_prof = nullptr,
                       uint32_t *d_prof_out = nullptr);
hipError_t launch_mark_one(uint32_t *d_explored, uint32_t l, uint32_t n_valid, hipStream_t stream);
// Neighbourhood-restricted step: score the candidates (tmp arrays indexed by
// candidate, accumulators in nb_acc), then compact, weigh and block-sum them.
hipError_t launch_nb_score(const NbStep &st, const uint32_t *d_sub_off, const uint32_t *d_sub_code,
                           const uint32_t *d_mask, const uint32_t *d_rank,
                           const uint32_t *d_explored, const float *d_P, uint64_t stride,
                           uint32_t *d_tmp_idx, float *d_tmp_s, StepAcc *d_nb_acc,
                           hipStream_t stream);
hipError_t launch_nb_finish(uint32_t total, const uint32_t *d_tmp_idx, const float *d_tmp_s,
                            StepAcc *d_nb_acc, float gamma, float w_min, uint32_t *d_nb_idx,
                            float *d_nb_s, uint32_t *d_nb_q, uint64_t *d_nb_bsum,
                            NbStats *d_stats, hipStream_t stream);
// One draw among the candidates; the step's first draw also marks `profile`.
hipError_t launch_nb_draw(uint32_t *d_nb_q, const uint32_t *d_nb_idx, const NbStats *d_stats,
                          uint64_t *d_nb_bsum, uint32_t *d_explored, uint32_t profile,
                          int mark_profile, uint32_t n_valid, uint64_t u64, const uint32_t *d_idx,
                          DrawResult *d_res, uint64_t seq, hipStream_t stream);
hipError_t launch_copy_weights(const float *d_s, uint32_t *d_explored, uint32_t n_valid,
                               const StepAcc *d_acc, float gamma, float w_min, uint32_t first,
                               uint32_t count, uint32_t *d_q, hipStream_t stream);
// Standalone sampler over an integer weight array.
hipError_t launch_array_block_sums(const uint32_t *d_q, uint32_t n, int block_log2,
                                   uint64_t *d_bsum, hipStream_t stream);
hipError_t launch_array_draw(uint32_t *d_q, uint32_t n, int block_log2, uint64_t *d_bsum,
                             uint32_t n_blocks, uint64_t u64, DrawResult *d_res,
                             hipStream_t stream);

} // namespace cgs
