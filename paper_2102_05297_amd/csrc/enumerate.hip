// Tuning-space enumeration with constraint pruning and stable compaction
// (Sect. 1: the space is the cross product of the parameters' value sets
// restricted by a-priori constraints; Alg. 1 takes it as the array TS).
//
// Three passes over the raw index range [0, n_raw), in tiles of 2048 raw
// indices per 256-thread workgroup (4 waves x 8 rows of 64):
//   mark     decode + constraints -> one ballot per row of 64; the ballot is
//            the validity bitmask (two uint32 words); per-tile valid count
//   scan     one workgroup: exclusive scan of the tile counts -> tile offsets
//            and the number of valid configurations
//   compact  per tile: re-read the bitmask, rank set bits with popcounts and
//            write the raw indices, ascending, and the rank of every mask
//            word (valid configurations before it), so that a raw index
//            maps to its valid index with one load and a popcount
// Integer-only; the output is independent of scheduling.
#include "device_common.h"

namespace cgs {

namespace {

constexpr int kEnumThreads = 256;
constexpr int kRowsPerWave = 8;
constexpr uint32_t kTile = kEnumThreads * kRowsPerWave; // 2048 raw indices

__global__ __launch_bounds__(kEnumThreads) void enum_mark(const SpaceDev *__restrict__ sp,
                                                          uint32_t *__restrict__ mask,
                                                          uint32_t *__restrict__ tile_count) {
  __shared__ int32_t table[CGS_MAX_PARAMS * CGS_MAX_RADIX];
  __shared__ uint32_t wave_cnt[kEnumThreads / kWave];
  for (int i = threadIdx.x; i < CGS_MAX_PARAMS * CGS_MAX_RADIX; i += kEnumThreads)
    table[i] = sp->table[i];
  __syncthreads();

  const uint32_t n_raw = sp->n_raw, n_words = sp->n_words;
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint64_t wave_base = (uint64_t)blockIdx.x * kTile + (uint64_t)wave * (kWave * kRowsPerWave);
  uint32_t cnt = 0;
  for (int row = 0; row < kRowsPerWave; ++row) {
    const uint64_t row_base = wave_base + (uint64_t)row * kWave;
    const uint64_t k = row_base + lane;
    bool valid = false;
    if (k < n_raw) {
      uint64_t lo, hi;
      decode_packed((uint32_t)k, sp, lo, hi);
      valid = satisfies_all(sp, table, lo, hi);
    }
    const uint64_t bal = __ballot(valid);
    const uint64_t w = row_base >> 5;
    if (lane < 2 && w + lane < n_words) mask[w + lane] = (uint32_t)(bal >> (32 * lane));
    cnt += (uint32_t)__popcll(bal);
  }
  if (lane == 0) wave_cnt[wave] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kEnumThreads / kWave; ++w) t += wave_cnt[w];
    tile_count[blockIdx.x] = t;
  }
}

constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void enum_scan(const uint32_t *__restrict__ tile_count,
                                                          uint32_t n_tiles,
                                                          uint32_t *__restrict__ tile_off,
                                                          uint64_t *__restrict__ total) {
  __shared__ uint64_t scratch[kScanThreads / kWave];
  const uint32_t per = (n_tiles + kScanThreads - 1) / kScanThreads;
  const uint32_t begin = min(n_tiles, threadIdx.x * per);
  const uint32_t end = min(n_tiles, begin + per);
  uint64_t local = 0;
  for (uint32_t i = begin; i < end; ++i) local += tile_count[i];
  uint64_t all;
  uint64_t run = block_excl_scan<kScanThreads>(local, scratch, all);
  for (uint32_t i = begin; i < end; ++i) {
    tile_off[i] = (uint32_t)run;
    run += tile_count[i];
  }
  if (threadIdx.x == 0) *total = all;
}

__global__ __launch_bounds__(kEnumThreads) void enum_compact(const SpaceDev *__restrict__ sp,
                                                             const uint32_t *__restrict__ mask,
                                                             const uint32_t *__restrict__ tile_off,
                                                             uint32_t *__restrict__ idx,
                                                             uint32_t *__restrict__ word_rank) {
  __shared__ uint32_t wave_cnt[kEnumThreads / kWave];
  const uint32_t n_words = sp->n_words;
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  const uint64_t wave_base = (uint64_t)blockIdx.x * kTile + (uint64_t)wave * (kWave * kRowsPerWave);
  const uint64_t w0 = wave_base >> 5; // 16 words per wave
  uint32_t c = 0;
  if (lane < 2 * kRowsPerWave && w0 + lane < n_words) c = (uint32_t)__popc(mask[w0 + lane]);
  c = wave_sum(c);
  if (lane == 0) wave_cnt[wave] = c;
  __syncthreads();
  uint32_t off = tile_off[blockIdx.x];
  for (uint32_t w = 0; w < wave; ++w) off += wave_cnt[w];
  for (int row = 0; row < kRowsPerWave; ++row) {
    const uint64_t wi = w0 + 2 * row;
    const uint64_t lo = wi < n_words ? mask[wi] : 0u;
    const uint64_t hi = wi + 1 < n_words ? mask[wi + 1] : 0u;
    const uint64_t bits = lo | (hi << 32);
    if (lane == 0 && wi < n_words) word_rank[wi] = off;
    if (lane == 1 && wi + 1 < n_words) word_rank[wi + 1] = off + (uint32_t)__popc((uint32_t)lo);
    if ((bits >> lane) & 1ull) {
      const uint32_t rank = (uint32_t)__popcll(bits & ((1ull << lane) - 1ull));
      idx[off + rank] = (uint32_t)(wave_base + (uint64_t)row * kWave + lane);
    }
    off += (uint32_t)__popcll(bits);
  }
}

} // namespace

uint32_t enumeration_tiles(uint32_t n_raw) {
  return (uint32_t)(((uint64_t)n_raw + kTile - 1) / kTile);
}

// phase 0: mark + scan (then the host reads *d_total); phase 1: compact and
// word ranks.
hipError_t launch_enumeration(const SpaceDev *d_space, uint32_t n_raw, uint32_t *d_mask,
                              uint32_t *d_tile_count, uint32_t *d_tile_off, uint64_t *d_total,
                              uint32_t *d_idx, uint32_t *d_rank, int phase, hipStream_t stream) {
  const uint32_t n_tiles = enumeration_tiles(n_raw);
  if (n_tiles == 0) return hipSuccess;
  if (phase == 0) {
    hipLaunchKernelGGL(enum_mark, dim3(n_tiles), dim3(kEnumThreads), 0, stream, d_space, d_mask,
                       d_tile_count);
    hipLaunchKernelGGL(enum_scan, dim3(1), dim3(kScanThreads), 0, stream, d_tile_count, n_tiles,
                       d_tile_off, d_total);
  } else {
    hipLaunchKernelGGL(enum_compact, dim3(n_tiles), dim3(kEnumThreads), 0, stream, d_space,
                       d_mask, d_tile_off, d_idx, d_rank);
  }
  return hipGetLastError();
}

} // namespace cgs
