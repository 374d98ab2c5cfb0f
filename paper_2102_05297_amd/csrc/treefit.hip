// Regression-tree fitting on the device (Sect. 3.4.2).
//
// The paper grows its counter model as a regression tree: greedy top-down
// splits chosen by a squared-error criterion, a set of candidate trees, a
// random half of the measured configurations for training and the other half
// for testing, and the candidate with the lowest test MAE (then RMSE) kept.
//
// Readings (shared with the CPU restatement the tests compare against):
//  * training half: the ceil(n/2) points first in the order of
//    (key >> 32, index), found by an 8-pass radix select over the distinct
//    64-bit keys ((key >> 32) << 32) | index;
//  * targets are quantised per counter, q = rint(y 2^s_c), s_c = 22 - e_c
//    with 2^(e_c-1) <= max|y_c| < 2^e_c, so node sums are exact integers and
//    nothing depends on the order of the device's additions;
//  * binary splits on a parameter's digit (left when digit <= t); score of an
//    admissible split sum_c (S_L^2/n_L + S_R^2/n_R) in float64, c ascending;
//    the best score wins, ties to the lower (parameter, threshold); a node
//    splits only when that beats its own sum_c S^2/n;
//  * level-by-level growth to depth D; a node that does not split becomes
//    "always left" (parameter 0, threshold 255) and is not searched again;
//  * node value rint(S/n) (float64 quotient); candidates are the tree cut at
//    depths 0..D, scored on the test half with exact integer sums of |e| and
//    e^2; the selected depth minimises (sum|e|, sum e^2, depth).
//
// Layout: every point becomes a row of W = PW + C 32-bit words: the digits
// (one byte per parameter, PW = ceil(P/4) words), then q[C]; the training
// rows' digit words are also kept alone (PW words per row) for the chunk
// counts.  The training rows of the nodes still searched are kept
// contiguous, one segment per node, and are repartitioned into the next
// level's segments after each level.  Segments are cut into chunks of at
// most 256 rows; the partition counts each chunk's rows per child, scans the
// counts and moves every chunk to fixed offsets, so the row order within a
// segment is stable and no two workgroups contend for an output cursor.
// Histograms hold, per open node, the sum of q for every (parameter, digit,
// counter) plus a count column: [sum_j R_j][C + 1] int64.  Of two open
// siblings only the one with fewer rows is histogrammed from its rows (its
// segment is laid out first); the other's histogram is the parent's minus
// it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

#include "device_common.h"
#include "models.h"

namespace cgs {

// Device-resident state of one fit.  The host fills the first block; the
// kernels write the rest (uploaded as zeros).
struct FitDev {
  uint32_t n, n_train, n_test, n_valid;
  uint32_t C, P, PW, W;
  uint32_t D, min_leaf, min_split, sumR;
  uint32_t entries, items, Cp, pad0;
  FastDiv divW, divC;
  uint32_t radix[CGS_MAX_PARAMS];
  uint32_t roff[CGS_MAX_PARAMS + 1]; // first bin of parameter j; roff[P] = sumR
  // written by the kernels
  uint32_t err;
  uint32_t key_done;
  uint64_t key_prefix, key_k, key_T;
  uint32_t key_hist[256];
  uint32_t absmax[CGS_MAX_COUNTERS];
  int32_t s[CGS_MAX_COUNTERS];
  uint32_t n_split;
  uint32_t lvl_K[2], lvl_R[2], lvl_NCH[2];
  uint32_t lvl_Kd[2], lvl_Rd[2]; // open nodes whose histogram is built from rows, their rows
  int32_t depth_sel;
  uint64_t A[CGS_MAX_DEPTH + 1], Blo[CGS_MAX_DEPTH + 1], Bhi[CGS_MAX_DEPTH + 1];
};

namespace {

constexpr int kFitThreads = 256;
constexpr uint32_t kFitGrid = 1024;       // workgroups of the grid-stride passes
constexpr uint32_t kTile = 256;           // rows per chunk / staged tile
constexpr uint16_t kAlwaysLeftNode = (uint16_t)(255u << 8);
constexpr uint32_t kScanThreads = 1024;
constexpr uint32_t kHistGrid = 1024;      // workgroups of the histogram pass
constexpr uint32_t kHistTile = 128;       // rows per staged tile of the histogram pass

__device__ __forceinline__ uint64_t split_key(uint64_t key, uint64_t i) {
  return (key & 0xFFFFFFFF00000000ull) | i;
}

__device__ __forceinline__ uint32_t row_digit(const uint32_t *row, uint32_t j) {
  return (row[j >> 2] >> (8u * (j & 3u))) & 255u;
}

// Words in flight per thread in the staging copies below: a plain loop would
// wait for each load before its LDS store (one memory latency per word).
constexpr int kStageBatch = 16;

// lds[k] = src[k] for k < n, by the whole workgroup (kFitThreads threads).
template <typename T>
__device__ __forceinline__ void stage_words(const T *__restrict__ src, uint32_t n, T *lds) {
  constexpr uint32_t kSpan = kStageBatch * kFitThreads;
  const uint32_t full = n / kSpan * kSpan; // whole batches need no bounds checks
  uint32_t k0 = threadIdx.x;
  for (; k0 < full; k0 += kSpan) {
    T v[kStageBatch];
#pragma unroll
    for (int b = 0; b < kStageBatch; ++b) v[b] = src[k0 + b * kFitThreads];
#pragma unroll
    for (int b = 0; b < kStageBatch; ++b) lds[k0 + b * kFitThreads] = v[b];
  }
  if (k0 < n) {
    T v[kStageBatch];
#pragma unroll
    for (int b = 0; b < kStageBatch; ++b) {
      const uint32_t k = k0 + b * kFitThreads;
      v[b] = k < n ? src[k] : T(0);
    }
#pragma unroll
    for (int b = 0; b < kStageBatch; ++b) {
      const uint32_t k = k0 + b * kFitThreads;
      if (k < n) lds[k] = v[b];
    }
  }
}

// Row `first + r` of `dst` (W words per row) = staged row src[r], for
// r < count; rows at or past `cap` are dropped.  When `digs` is given, its
// row `first + r` (PW words) gets the row's digit words too.  Words go out
// in batches so their LDS reads overlap.
__device__ __forceinline__ void copy_rows_out(const uint32_t *lds, const uint32_t *src,
                                              uint32_t count, uint32_t W, FastDiv divW,
                                              uint32_t *__restrict__ dst, uint32_t first,
                                              uint32_t cap, uint32_t *__restrict__ digs = nullptr,
                                              uint32_t PW = 0) {
  if (first >= cap) return;
  const uint32_t words = min(count, cap - first) * W;
  uint32_t *out = dst + (uint64_t)first * W;
  for (uint32_t k0 = threadIdx.x; k0 < words; k0 += kStageBatch * kFitThreads) {
    uint32_t v[kStageBatch], rr[kStageBatch];
#pragma unroll
    for (int b = 0; b < kStageBatch; ++b) {
      const uint32_t k = min(k0 + b * kFitThreads, words - 1);
      rr[b] = fastdiv(k, divW);
      v[b] = lds[src[rr[b]] * W + (k - rr[b] * W)];
    }
#pragma unroll
    for (int b = 0; b < kStageBatch; ++b) {
      const uint32_t k = k0 + b * kFitThreads;
      if (k < words) {
        out[k] = v[b];
        const uint32_t w = k - rr[b] * W;
        if (digs && w < PW) digs[(uint64_t)(first + rr[b]) * PW + w] = v[b];
      }
    }
  }
}

// Largest s in [0, K) with start[s] <= a (start ascending, start[0] = 0).
__device__ __forceinline__ uint32_t last_at_or_below(const uint32_t *start, uint32_t K,
                                                     uint32_t a) {
  uint32_t lo = 0, hi = K;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (start[mid] <= a) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ void fit_zero(uint64_t *__restrict__ p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// Exclusive prefix sums of in[0..n) (one workgroup; each thread scans a run
// of consecutive entries).  n is *n_dev when given, else n_host.
__global__ __launch_bounds__(kScanThreads) void fit_excl_scan(const uint64_t *__restrict__ in,
                                                              uint64_t *__restrict__ out,
                                                              const uint32_t *__restrict__ n_dev,
                                                              uint32_t n_host) {
  __shared__ uint64_t scratch[kScanThreads / 64];
  const uint32_t n = n_dev ? *n_dev : n_host;
  const uint32_t t = threadIdx.x, per = (n + kScanThreads - 1) / kScanThreads;
  const uint32_t a = min(n, t * per), b = min(n, a + per);
  // the run is read in batches of kStageBatch loads in flight (a plain loop
  // waits for every load before the next)
  uint64_t mine = 0;
  for (uint32_t i0 = a; i0 < b; i0 += kStageBatch) {
    uint64_t v[kStageBatch];
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) v[u] = i0 + u < b ? in[i0 + u] : 0ull;
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) mine += v[u];
  }
  uint64_t tot;
  uint64_t run = block_excl_scan<kScanThreads>(mine, scratch, tot);
  for (uint32_t i0 = a; i0 < b; i0 += kStageBatch) {
    uint64_t v[kStageBatch];
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) v[u] = i0 + u < b ? in[i0 + u] : 0ull;
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) {
      if (i0 + u < b) {
        out[i0 + u] = run;
        run += v[u];
      }
    }
  }
}

// Validation, per-counter max |y| and the histogram of the keys' top byte.
__global__ __launch_bounds__(kFitThreads) void fit_prepare(FitDev *__restrict__ fd,
                                                           const uint32_t *__restrict__ pts,
                                                           const float *__restrict__ Y,
                                                           const uint64_t *__restrict__ keys) {
  __shared__ uint32_t s_max[CGS_MAX_COUNTERS];
  __shared__ uint32_t s_hist[256];
  __shared__ uint32_t s_err;
  const uint32_t t = threadIdx.x;
  const uint32_t n = fd->n, C = fd->C, nv = fd->n_valid;
  if (t < CGS_MAX_COUNTERS) s_max[t] = 0;
  s_hist[t] = 0;
  if (t == 0) s_err = 0;
  __syncthreads();
  uint32_t err = 0;
  const uint64_t gsz = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + t;
  // a stride that is a multiple of C keeps each thread on one counter
  const uint64_t step = gsz / C * C, total = (uint64_t)n * C;
  if (gid < step) {
    uint32_t mx = 0;
    uint64_t k = gid;
    for (; k + 3 * step < total; k += 4 * step) {
      float y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) y[u] = Y[k + u * step];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (!(y[u] >= 0.0f) || !isfinite(y[u])) err |= 2u; // counters are non-negative
        else mx = max(mx, __float_as_uint(fabsf(y[u])));
      }
    }
    for (; k < total; k += step) {
      const float y = Y[k];
      if (!(y >= 0.0f) || !isfinite(y)) err |= 2u;
      else mx = max(mx, __float_as_uint(fabsf(y)));
    }
    if (mx) atomicMax(&s_max[gid % C], mx);
  }
  uint64_t i = gid;
  for (; i + 3 * gsz < n; i += 4 * gsz) {
    uint32_t p[4];
    uint64_t kk[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      p[u] = pts[i + u * gsz];
      kk[u] = keys[i + u * gsz];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (p[u] >= nv) err |= 1u;
      atomicAdd(&s_hist[(uint32_t)(split_key(kk[u], i + u * gsz) >> 56)], 1u);
    }
  }
  for (; i < n; i += gsz) {
    if (pts[i] >= nv) err |= 1u;
    atomicAdd(&s_hist[(uint32_t)(split_key(keys[i], i) >> 56)], 1u);
  }
  if (err) atomicOr(&s_err, err);
  __syncthreads();
  if (t < C && s_max[t]) atomicMax(&fd->absmax[t], s_max[t]);
  if (s_hist[t]) atomicAdd(&fd->key_hist[t], s_hist[t]);
  if (t == 0 && s_err) atomicOr(&fd->err, s_err);
}

// Radix select, pass `pass` (bits 56 - 8 pass .. 63 - 8 pass): pick the bin
// holding the key of rank key_k within the current prefix.  When that bin is
// taken whole (or the last byte is fixed), the threshold is final.
__global__ __launch_bounds__(256) void fit_key_pick(FitDev *__restrict__ fd, int pass) {
  __shared__ uint64_t scratch[4];
  if (fd->key_done) return;
  const uint32_t t = threadIdx.x;
  const uint32_t h = fd->key_hist[t];
  // read the state before the scan's barriers: one thread rewrites it below
  const uint64_t k = fd->key_k, prefix0 = fd->key_prefix;
  uint64_t tot;
  const uint64_t before = block_excl_scan<256>(h, scratch, tot);
  const int shift = 56 - 8 * pass;
  if (before < k && k <= before + h) {
    const uint64_t prefix = prefix0 | ((uint64_t)t << shift);
    const uint64_t kn = k - before;
    fd->key_prefix = prefix;
    fd->key_k = kn;
    if (h == kn || shift == 0) {
      fd->key_T = prefix | (shift ? ((1ull << shift) - 1ull) : 0ull);
      fd->key_done = 1;
    }
  }
  __syncthreads();
  fd->key_hist[t] = 0;
}

__global__ __launch_bounds__(kFitThreads) void fit_key_hist(FitDev *__restrict__ fd,
                                                            const uint64_t *__restrict__ keys,
                                                            int pass) {
  __shared__ uint32_t s_hist[256];
  if (fd->key_done) return;
  const uint32_t t = threadIdx.x;
  s_hist[t] = 0;
  __syncthreads();
  const int shift = 56 - 8 * pass; // pass >= 1
  const uint64_t want = fd->key_prefix >> (shift + 8);
  const uint64_t n = fd->n, gsz = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + t; i < n; i += gsz) {
    const uint64_t kk = split_key(keys[i], i);
    if ((kk >> (shift + 8)) == want) atomicAdd(&s_hist[(uint32_t)(kk >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (s_hist[t]) atomicAdd(&fd->key_hist[t], s_hist[t]);
}

// Training points per tile of 256 points (for the scatter's offsets).
__global__ __launch_bounds__(kFitThreads) void fit_tile_count(const FitDev *__restrict__ fd,
                                                              const uint64_t *__restrict__ keys,
                                                              uint64_t *__restrict__ cnt) {
  __shared__ uint64_t scratch[kFitThreads / 64];
  const uint32_t n = fd->n, t = threadIdx.x;
  const uint64_t T = fd->key_T;
  for (uint32_t tile = blockIdx.x; (uint64_t)tile * kTile < n; tile += gridDim.x) {
    const uint32_t i = tile * kTile + t;
    const uint64_t f = (i < n && split_key(keys[i], i) <= T) ? 1ull : 0ull;
    const uint64_t s = block_sum<kFitThreads>(f, scratch);
    if (t == 0) cnt[tile] = s;
  }
}

// Rows of every point: digits and quantised targets, training and test
// rows each packed contiguously in point order.
__global__ __launch_bounds__(kFitThreads) void fit_scatter(
    FitDev *__restrict__ fd, const SpaceDev *__restrict__ sp, const uint32_t *__restrict__ idx,
    const uint32_t *__restrict__ pts, const float *__restrict__ Y,
    const uint64_t *__restrict__ keys, const uint64_t *__restrict__ tile_off,
    uint32_t *__restrict__ rows, uint32_t *__restrict__ digs, uint32_t *__restrict__ test_rows) {
  extern __shared__ uint32_t lds[]; // [kTile][W] rows, then [kTile][Cp] targets
  __shared__ int32_t s_scale[CGS_MAX_COUNTERS];
  __shared__ uint32_t s_src[2][kTile];
  __shared__ uint64_t scratch[kFitThreads / 64];
  const uint32_t t = threadIdx.x;
  const uint32_t n = fd->n, C = fd->C, Cp = fd->Cp, P = fd->P, PW = fd->PW, W = fd->W;
  const uint32_t nv = fd->n_valid;
  const uint64_t T = fd->key_T;
  float *ytile = reinterpret_cast<float *>(lds + kTile * W);
  if (t < C) {
    const float mx = __uint_as_float(fd->absmax[t]);
    int e = 0;
    if (mx > 0.0f) (void)frexpf(mx, &e);
    s_scale[t] = 22 - e;
    if (blockIdx.x == 0) fd->s[t] = 22 - e;
  }
  for (uint32_t tile = blockIdx.x; (uint64_t)tile * kTile < n; tile += gridDim.x) {
    const uint32_t first = tile * kTile, nr = min(kTile, n - first);
    __syncthreads();
    const float *ysrc = Y + (uint64_t)first * C;
    for (uint32_t k0 = t; k0 < nr * C; k0 += kStageBatch * kFitThreads) {
      float v[kStageBatch]; // all loads in flight before the first LDS store
#pragma unroll
      for (int b = 0; b < kStageBatch; ++b) {
        const uint32_t k = k0 + b * kFitThreads;
        v[b] = k < nr * C ? ysrc[k] : 0.0f;
      }
#pragma unroll
      for (int b = 0; b < kStageBatch; ++b) {
        const uint32_t k = k0 + b * kFitThreads;
        if (k < nr * C) {
          const uint32_t r = fastdiv(k, fd->divC);
          ytile[r * Cp + (k - r * C)] = v[b];
        }
      }
    }
    __syncthreads();
    const bool live = t < nr;
    bool train = false;
    if (live) {
      const uint32_t i = first + t;
      train = split_key(keys[i], i) <= T;
      const uint32_t p = pts[i];
      uint64_t lo = 0, hi = 0;
      if (p < nv) decode_packed(idx[p], sp, lo, hi);
      uint32_t *row = lds + t * W;
      for (uint32_t w = 0; w < PW; ++w) {
        uint32_t word = 0;
        for (uint32_t b = 0; b < 4; ++b) {
          const uint32_t j = 4 * w + b;
          if (j < P) word |= digit_of(lo, hi, j) << (8 * b);
        }
        row[w] = word;
      }
      for (uint32_t c = 0; c < C; ++c) {
        const float y = ytile[t * Cp + c];
        const double v = isfinite(y) ? ldexp((double)y, s_scale[c]) : 0.0;
        row[PW + c] = (uint32_t)(int32_t)rint(v);
      }
    }
    const uint64_t flag = live ? (train ? 1ull : (1ull << 32)) : 0ull;
    uint64_t tot;
    const uint64_t rank = block_excl_scan<kFitThreads>(flag, scratch, tot);
    const uint32_t ntr = (uint32_t)tot, nte = (uint32_t)(tot >> 32);
    if (live) {
      if (train) s_src[0][(uint32_t)rank] = t;
      else s_src[1][(uint32_t)(rank >> 32)] = t;
    }
    __syncthreads();
    const uint32_t base_tr = (uint32_t)tile_off[tile], base_te = first - base_tr;
    copy_rows_out(lds, s_src[0], ntr, W, fd->divW, rows, base_tr, fd->n_train, digs, PW);
    copy_rows_out(lds, s_src[1], nte, W, fd->divW, test_rows, base_te, fd->n_test);
  }
}

// Sum of q over the training rows: the root's sums.
__global__ __launch_bounds__(kFitThreads) void fit_root_sums(const FitDev *__restrict__ fd,
                                                             const uint32_t *__restrict__ rows,
                                                             int64_t *__restrict__ nsum) {
  __shared__ int64_t s_sum[CGS_MAX_COUNTERS];
  const uint32_t t = threadIdx.x, C = fd->C, PW = fd->PW, W = fd->W;
  const uint64_t n = fd->n_train;
  if (t < CGS_MAX_COUNTERS) s_sum[t] = 0;
  __syncthreads();
  const uint64_t gsz = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + t;
  const uint64_t rstep = gsz / C; // rows per round; thread keeps counter gid % C
  if (gid < rstep * C) {
    const uint32_t c = (uint32_t)(gid % C);
    int64_t acc = 0;
    uint64_t r = gid / C;
    for (; r + 3 * rstep < n; r += 4 * rstep) {
      int32_t v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = (int32_t)rows[(r + u * rstep) * W + PW + c];
      acc += (int64_t)v[0] + v[1] + v[2] + v[3];
    }
    for (; r < n; r += rstep) acc += (int32_t)rows[r * W + PW + c];
    if (acc) atomicAdd(reinterpret_cast<unsigned long long *>(&s_sum[c]), (unsigned long long)acc);
  }
  __syncthreads();
  if (t < C && s_sum[t])
    atomicAdd(reinterpret_cast<unsigned long long *>(&nsum[t]), (unsigned long long)s_sum[t]);
}

__device__ __forceinline__ int32_t node_value(int64_t S, uint32_t n) {
  return (int32_t)rint((double)S / (double)n);
}

__global__ void fit_root(const FitDev *__restrict__ fd, uint32_t *__restrict__ ncount,
                         const int64_t *__restrict__ nsum, int32_t *__restrict__ nmean,
                         uint8_t *__restrict__ nstate) {
  const uint32_t n = fd->n_train, C = fd->C;
  for (uint32_t c = threadIdx.x; c < C; c += blockDim.x) nmean[c] = node_value(nsum[c], n);
  if (threadIdx.x == 0) {
    ncount[0] = n;
    nstate[0] = (fd->D > 0 && n >= fd->min_split) ? 1 : 0;
  }
}

// Segments of the open nodes of level L.  Of two open siblings the one with
// more rows (the right one on a tie) is "derived": its histogram is the
// parent's minus its sibling's, so only the other ("direct") nodes' rows are
// histogrammed.  Slots and segments list the direct nodes first, then the
// derived ones, each group in heap order; der_parent / der_sib hold the
// parent's slot (level L - 1) and the sibling's slot of every derived slot.
__global__ __launch_bounds__(kFitThreads) void fit_layout(
    FitDev *__restrict__ fd, int L, const uint8_t *__restrict__ nstate,
    const uint32_t *__restrict__ ncount, uint32_t *__restrict__ open_node,
    uint32_t *__restrict__ seg_start, uint32_t *__restrict__ chunk_start,
    uint32_t *__restrict__ slot_of, const uint32_t *__restrict__ slot_of_prev,
    uint32_t *__restrict__ der_parent, uint32_t *__restrict__ der_sib,
    uint4 *__restrict__ slot_info_prev, uint32_t kcap) {
  __shared__ uint64_t scratch[kFitThreads / 64];
  const uint32_t t = threadIdx.x, cnt = 1u << L, base = cnt - 1;
  const uint32_t per = (cnt + kFitThreads - 1) / kFitThreads;
  const uint32_t a = min(cnt, t * per), b = min(cnt, a + per);
  auto derived = [&](uint32_t k) { // k: heap index of an open node
    if (L == 0) return false;
    const uint32_t sib = (k & 1u) ? k + 1 : k - 1;
    if (!nstate[sib]) return false;
    return ncount[k] > ncount[sib] || (ncount[k] == ncount[sib] && !(k & 1u));
  };
  // rows << 16 | open nodes, and chunks, of the direct and the derived nodes
  uint64_t md = 0, mdc = 0, mv = 0, mvc = 0;
  for (uint32_t k = a; k < b; ++k) {
    const uint32_t node = base + k;
    if (!nstate[node]) continue;
    const uint64_t rows = ((uint64_t)ncount[node] << 16) | 1ull;
    const uint64_t chunks = (ncount[node] + kTile - 1) / kTile;
    if (derived(node)) {
      mv += rows;
      mvc += chunks;
    } else {
      md += rows;
      mdc += chunks;
    }
  }
  uint64_t td, tdc, tv, tvc;
  const uint64_t bd = block_excl_scan<kFitThreads>(md, scratch, td);
  const uint64_t bdc = block_excl_scan<kFitThreads>(mdc, scratch, tdc);
  const uint64_t bv = block_excl_scan<kFitThreads>(mv, scratch, tv);
  const uint64_t bvc = block_excl_scan<kFitThreads>(mvc, scratch, tvc);
  const uint32_t Kd = (uint32_t)(td & 0xffffu), Rd = (uint32_t)(td >> 16);
  uint32_t sd = (uint32_t)(bd & 0xffffu), rd = (uint32_t)(bd >> 16), cd = (uint32_t)bdc;
  uint32_t sv = Kd + (uint32_t)(bv & 0xffffu), rv = Rd + (uint32_t)(bv >> 16);
  uint32_t cv = (uint32_t)tdc + (uint32_t)bvc;
  for (uint32_t k = a; k < b; ++k) {
    const uint32_t node = base + k;
    slot_of[k] = ~0u;
    if (!nstate[node]) continue;
    const bool der = derived(node);
    const uint32_t slot = der ? sv : sd, row = der ? rv : rd, ch = der ? cv : cd;
    if (slot < kcap) {
      open_node[slot] = node;
      seg_start[slot] = row;
      chunk_start[slot] = ch;
      slot_of[k] = slot;
    }
    const uint32_t nr = ncount[node], nch = (nr + kTile - 1) / kTile;
    if (der) {
      ++sv;
      rv += nr;
      cv += nch;
    } else {
      ++sd;
      rd += nr;
      cd += nch;
    }
  }
  __syncthreads();
  // the parent's (level L - 1) record gets each open child's first row; a
  // derived slot's parent and sibling slots
  for (uint32_t k = a; k < b; ++k) {
    const uint32_t node = base + k, slot = slot_of[k];
    if (slot == ~0u || L == 0) continue;
    const uint32_t parent = (node - 1) / 2;
    const uint32_t pslot = slot_of_prev[parent - ((1u << (L - 1)) - 1)];
    if (pslot < kcap) {
      if (node & 1u) slot_info_prev[pslot].y = seg_start[slot];
      else slot_info_prev[pslot].z = seg_start[slot];
    }
    if (slot < Kd) continue;
    const uint32_t sib = (node & 1u) ? node + 1 : node - 1;
    der_parent[slot - Kd] = pslot;
    der_sib[slot - Kd] = slot_of[sib - base]; // ~0u only after a slot overflow
  }
  if (t == 0) {
    // at most n_train / min_split nodes hold min_split rows each
    const uint32_t Kall = Kd + (uint32_t)(tv & 0xffffu);
    const uint32_t K = min(Kall, kcap);
    if (K < Kall) atomicOr(&fd->err, 4u);
    seg_start[K] = Rd + (uint32_t)(tv >> 16);
    chunk_start[K] = (uint32_t)(tdc + tvc);
    fd->lvl_K[L & 1] = K;
    fd->lvl_R[L & 1] = Rd + (uint32_t)(tv >> 16);
    fd->lvl_NCH[L & 1] = (uint32_t)(tdc + tvc);
    fd->lvl_Kd[L & 1] = min(Kd, K);
    fd->lvl_Rd[L & 1] = Rd;
  }
}

// Histograms of the derived slots of level L: parent minus sibling (exact
// int64 sums).  A parent has one derived child, so its entries are read here
// once and cleared for the level after next.
__global__ __launch_bounds__(kFitThreads) void fit_hist_derive(
    const FitDev *__restrict__ fd, int L, int64_t *__restrict__ hist_prev,
    int64_t *__restrict__ hist, const uint32_t *__restrict__ der_parent,
    const uint32_t *__restrict__ der_sib, uint32_t kcap) {
  const uint32_t set = L & 1, K = fd->lvl_K[set], Kd = fd->lvl_Kd[set], E = fd->entries;
  const uint64_t total = (uint64_t)(K - Kd) * E;
  for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t v = (uint32_t)(e / E), i = (uint32_t)(e - (uint64_t)v * E);
    const uint32_t ps = der_parent[v], ss = der_sib[v];
    if (ps >= kcap || ss >= kcap) continue; // only after a slot overflow (err bit 4)
    int64_t *hp = hist_prev + (uint64_t)ps * E + i;
    hist[(uint64_t)(Kd + v) * E + i] = *hp - hist[(uint64_t)ss * E + i];
    *hp = 0;
  }
}

// Histograms of level L.  Each workgroup takes a contiguous range of the
// level's rows and cuts it at segment (node) boundaries; one node's part
// passes through LDS in tiles of kHistTile rows, row group g of
// G = 256 / (C + 1) groups takes a contiguous share of each tile and lane
// (g, c) handles column c of those rows (column C is the count).
// Rows arrive in configuration order, so most parameters keep their digit
// over long runs and consecutive rows differ in few digits: each lane keeps
// the running sum of its column and, per parameter, the sum at which the
// current run of equal digits began; a word compare with the previous row
// finds the parameters whose digit changed, and only those add their run's
// sum to the workgroup's int64 LDS histogram.  At the end of a node's part the
// workgroup adds its LDS histogram to the node's histogram in device memory.
template <int MAXP>
__global__ __launch_bounds__(kFitThreads) void fit_hist(const FitDev *__restrict__ fd, int L,
                                                        const uint32_t *__restrict__ rows,
                                                        const uint32_t *__restrict__ seg_start,
                                                        int64_t *__restrict__ ghist) {
  extern __shared__ int64_t h64[]; // [entries], then a [kHistTile][W] row tile
  uint32_t *rl = reinterpret_cast<uint32_t *>(h64 + fd->entries);
  // the direct nodes' rows come first: [0, Rd), segments 0..Kd-1
  const uint32_t set = L & 1, K = fd->lvl_Kd[set], R = fd->lvl_Rd[set];
  if (R == 0) return;
  const uint32_t a = (uint32_t)((uint64_t)R * blockIdx.x / gridDim.x);
  const uint32_t b = (uint32_t)((uint64_t)R * (blockIdx.x + 1) / gridDim.x);
  if (a >= b) return;
  const uint32_t t = threadIdx.x;
  const uint32_t C = fd->C, C1 = C + 1, P = fd->P, PW = fd->PW, W = fd->W, E = fd->entries;
  const uint32_t G = kFitThreads / C1, g = t / C1, c = t - g * C1;
  const bool active = g < G;
  uint32_t roffc[MAXP]; // (first bin of j) * (C + 1) + c
#pragma unroll
  for (int j = 0; j < MAXP; ++j) roffc[j] = (j < (int)P) ? fd->roff[j] * C1 + c : 0u;
  for (uint32_t e = t; e < E; e += kFitThreads) h64[e] = 0;
  __syncthreads();

  uint32_t slot = last_at_or_below(seg_start, K, a);
  uint32_t pos = a;
  while (pos < b) {
    const uint32_t seg_end = seg_start[slot + 1];
    const uint32_t end = min(b, seg_end);
    if (end <= pos) break; // segments are never empty
    constexpr int NW = (MAXP + 3) / 4;
    // S: running sum of column c over the lane's rows; st[j]: S where
    // parameter j's current run of equal digits began.  A run's sum
    // S - st[j] goes to the LDS bin of its digit when the digit changes.
    // prev holds the previous row's packed digits (0xff bytes: no run yet).
    uint32_t prev[NW];
    int64_t st[MAXP];
#pragma unroll
    for (int w = 0; w < NW; ++w) prev[w] = 0xffffffffu;
#pragma unroll
    for (int j = 0; j < MAXP; ++j) st[j] = 0;
    int64_t S = 0;
    auto process = [&](const uint32_t (&dw)[NW], int64_t q) {
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const uint32_t x = dw[w] ^ prev[w];
        if (w < (int)PW && x) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int j = 4 * w + k;
            if (j < (int)P && ((x >> (8 * k)) & 255u)) {
              const uint32_t old = (prev[w] >> (8 * k)) & 255u;
              if (old != 0xffu)
                atomicAdd(reinterpret_cast<unsigned long long *>(&h64[roffc[j] + old * C1]),
                          (unsigned long long)(S - st[j]));
              st[j] = S;
            }
          }
          prev[w] = dw[w];
        }
      }
      S += q;
    };
    // the node's rows pass through LDS in tiles (all loads of a tile in
    // flight together); group g takes a contiguous share of each tile
    for (uint32_t tp = pos; tp < end; tp += kHistTile) {
      const uint32_t nr = min(kHistTile, end - tp);
      __syncthreads();
      stage_words(rows + (uint64_t)tp * W, nr * W, rl);
      __syncthreads();
      if (active) {
        const uint32_t r0 = (uint32_t)((uint64_t)nr * g / G);
        const uint32_t r1 = (uint32_t)((uint64_t)nr * (g + 1) / G);
        for (uint32_t r = r0; r < r1; ++r) {
          const uint32_t *row = rl + r * W;
          uint32_t dw[NW];
#pragma unroll
          for (int w = 0; w < NW; ++w) dw[w] = (w < (int)PW) ? row[w] : 0u;
          process(dw, c < C ? (int64_t)(int32_t)row[PW + c] : 1);
        }
      }
    }
    if (active) {
#pragma unroll
      for (int j = 0; j < MAXP; ++j) {
        const uint32_t old = (prev[j >> 2] >> (8 * (j & 3))) & 255u;
        if (j < (int)P && old != 0xffu)
          atomicAdd(reinterpret_cast<unsigned long long *>(&h64[roffc[j] + old * C1]),
                    (unsigned long long)(S - st[j]));
      }
    }
    __syncthreads();
    int64_t *H = ghist + (uint64_t)slot * E;
    for (uint32_t e = t; e < E; e += kFitThreads) {
      const int64_t v = h64[e];
      if (v) {
        atomicAdd(reinterpret_cast<unsigned long long *>(H + e), (unsigned long long)v);
        h64[e] = 0;
      }
    }
    __syncthreads();
    pos = end;
    ++slot;
  }
}

__device__ __forceinline__ void inherit_children(uint32_t node, uint32_t C,
                                                 uint32_t *__restrict__ ncount,
                                                 int64_t *__restrict__ nsum,
                                                 int32_t *__restrict__ nmean,
                                                 uint8_t *__restrict__ nstate,
                                                 uint16_t *__restrict__ nodes) {
  const uint32_t l = 2 * node + 1, r = l + 1;
  if (threadIdx.x == 0) {
    nodes[node] = kAlwaysLeftNode;
    ncount[l] = ncount[node];
    ncount[r] = 0;
    nstate[l] = 0;
    nstate[r] = 0;
  }
  for (uint32_t c = threadIdx.x; c < C; c += blockDim.x) {
    const int32_t m = nmean[(uint64_t)node * C + c];
    nsum[(uint64_t)l * C + c] = nsum[(uint64_t)node * C + c];
    nsum[(uint64_t)r * C + c] = 0;
    nmean[(uint64_t)l * C + c] = m;
    nmean[(uint64_t)r * C + c] = m;
  }
}

__device__ __forceinline__ bool better(double s, uint32_t k, double s2, uint32_t k2) {
  // (s, k) beats (s2, k2): a valid candidate, higher score, then lower index
  if (k == ~0u) return false;
  if (k2 == ~0u) return true;
  return s > s2 || (s == s2 && k < k2);
}

// Split search of level L: one workgroup per node of the level.  Candidate
// k enumerates (parameter, threshold) pairs in ascending order: parameter j
// contributes thresholds 0 .. R_j - 2, from index roff[j] - j.
__global__ __launch_bounds__(kFitThreads) void fit_split(
    FitDev *__restrict__ fd, int L, int64_t *__restrict__ ghist,
    const uint32_t *__restrict__ slot_of, uint32_t cap_entries, uint32_t *__restrict__ ncount,
    int64_t *__restrict__ nsum, int32_t *__restrict__ nmean, uint8_t *__restrict__ nstate,
    uint16_t *__restrict__ nodes, uint4 *__restrict__ slot_info) {
  extern __shared__ int64_t ps[]; // prefix sums over digits of one parameter group
  __shared__ int64_t s_S[CGS_MAX_COUNTERS];
  __shared__ double s_score[kFitThreads / 64];
  __shared__ uint32_t s_k[kFitThreads / 64];
  __shared__ uint32_t s_split, s_j, s_t, s_nl, s_keep;
  const uint32_t t = threadIdx.x, local = blockIdx.x;
  const uint32_t node = (1u << L) - 1 + local;
  const uint32_t C = fd->C, C1 = C + 1, P = fd->P;
  if (!nstate[node]) {
    inherit_children(node, C, ncount, nsum, nmean, nstate, nodes);
    return;
  }
  const uint32_t slot = slot_of[local];
  int64_t *H = ghist + (uint64_t)slot * fd->entries;
  const uint32_t n = ncount[node], min_leaf = fd->min_leaf;
  for (uint32_t c = t; c < C; c += kFitThreads) s_S[c] = nsum[(uint64_t)node * C + c];

  double best = 0.0;
  uint32_t best_k = ~0u;
  uint32_t j0 = 0;
  while (j0 < P) {
    uint32_t j1 = j0, bins = 0;
    while (j1 < P && (bins + fd->radix[j1]) * C1 <= cap_entries) bins += fd->radix[j1++];
    const uint32_t b0 = fd->roff[j0];
    __syncthreads();
    for (uint32_t it = t; it < (j1 - j0) * C1; it += kFitThreads) {
      const uint32_t jl = j0 + it / C1, c = it % C1;
      const uint32_t rb = fd->roff[jl], R = fd->radix[jl];
      int64_t hv[CGS_MAX_RADIX]; // every digit's entry in flight at once
#pragma unroll
      for (uint32_t v = 0; v < CGS_MAX_RADIX; ++v)
        hv[v] = H[(uint64_t)(rb + min(v, R - 1)) * C1 + c]; // in bounds; v >= R unused
      int64_t run = 0;
#pragma unroll
      for (uint32_t v = 0; v < CGS_MAX_RADIX; ++v) {
        if (v < R) {
          run += hv[v];
          ps[(rb - b0 + v) * C1 + c] = run;
        }
      }
    }
    __syncthreads();
    const uint32_t k0 = fd->roff[j0] - j0, k1 = fd->roff[j1] - j1;
    for (uint32_t k = k0 + t; k < k1; k += kFitThreads) {
      uint32_t jl = j0;
      while (fd->roff[jl + 1] - (jl + 1) <= k) ++jl;
      const uint32_t th = k - (fd->roff[jl] - jl);
      const int64_t *pr = ps + (fd->roff[jl] - b0 + th) * C1;
      const uint32_t nL = (uint32_t)pr[C], nR = n - nL;
      if (nL < min_leaf || nR < min_leaf) continue;
      const double dL = (double)nL, dR = (double)nR;
      double acc = 0.0;
      for (uint32_t c = 0; c < C; ++c) {
        const double x = (double)pr[c];
        const double y = (double)(s_S[c] - pr[c]);
        acc = acc + ((x * x) / dL + (y * y) / dR);
      }
      if (better(acc, k, best, best_k)) {
        best = acc;
        best_k = k;
      }
    }
    j0 = j1;
  }
  // argmax over the workgroup
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double s2 = __shfl_xor(best, o, 64);
    const uint32_t k2 = (uint32_t)__shfl_xor((int)best_k, o, 64);
    if (better(s2, k2, best, best_k)) {
      best = s2;
      best_k = k2;
    }
  }
  if ((t & 63u) == 0) {
    s_score[t >> 6] = best;
    s_k[t >> 6] = best_k;
  }
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < kFitThreads / 64; ++w)
      if (better(s_score[w], s_k[w], best, best_k)) {
        best = s_score[w];
        best_k = s_k[w];
      }
    double parent = 0.0;
    const double dn = (double)n;
    for (uint32_t c = 0; c < C; ++c) {
      const double x = (double)s_S[c];
      parent = parent + (x * x) / dn;
    }
    uint32_t split = 0, j = 0, th = 0;
    if (best_k != ~0u && best > parent) {
      split = 1;
      while (fd->roff[j + 1] - (j + 1) <= best_k) ++j;
      th = best_k - (fd->roff[j] - j);
      uint32_t nl = 0;
#pragma unroll
      for (uint32_t v = 0; v < CGS_MAX_RADIX; ++v) {
        const uint32_t x = (uint32_t)H[(uint64_t)(fd->roff[j] + min(v, th)) * C1 + C];
        nl += v <= th ? x : 0u;
      }
      s_nl = nl;
    }
    s_split = split;
    s_j = j;
    s_t = th;
  }
  __syncthreads();
  if (!s_split) {
    inherit_children(node, C, ncount, nsum, nmean, nstate, nodes);
    if (t == 0) slot_info[slot].x = kAlwaysLeftNode; // no child is searched
  } else {
    const uint32_t j = s_j, th = s_t, nl = s_nl, nr = n - nl;
    const uint32_t l = 2 * node + 1, r = l + 1;
    for (uint32_t c = t; c < C; c += kFitThreads) {
      int64_t sl = 0;
#pragma unroll
      for (uint32_t v = 0; v < CGS_MAX_RADIX; ++v) {
        const int64_t x = H[(uint64_t)(fd->roff[j] + min(v, th)) * C1 + c];
        sl += v <= th ? x : 0;
      }
      const int64_t sr = s_S[c] - sl;
      nsum[(uint64_t)l * C + c] = sl;
      nsum[(uint64_t)r * C + c] = sr;
      nmean[(uint64_t)l * C + c] = node_value(sl, nl);
      nmean[(uint64_t)r * C + c] = node_value(sr, nr);
    }
    if (t == 0) {
      const bool deeper = (uint32_t)L + 1 < fd->D;
      const bool lo = deeper && nl >= fd->min_split, ro = deeper && nr >= fd->min_split;
      nodes[node] = (uint16_t)(j | (th << 8));
      ncount[l] = nl;
      ncount[r] = nr;
      nstate[l] = lo ? 1 : 0;
      nstate[r] = ro ? 1 : 0;
      slot_info[slot].x = (j | (th << 8)) | (lo ? 1u << 16 : 0u) | (ro ? 1u << 17 : 0u);
      s_keep = lo && ro;
      atomicAdd(&fd->n_split, 1u);
    }
  }
  // The slot is used again two levels down.  With both children open, one
  // child's histogram is derived from this one, which clears it there;
  // otherwise clear it now.
  __syncthreads();
  if (!(s_split && s_keep))
    for (uint32_t e = t; e < fd->entries; e += kFitThreads) H[e] = 0;
}

// Chunk ch of level L: its segment, first row, row count and the segment's
// first chunk, from the level's segment and chunk starts staged in LDS.
struct ChunkRef {
  uint32_t slot, first, nr, first_chunk;
};
__device__ __forceinline__ ChunkRef chunk_ref(uint32_t ch, const uint32_t *cs, const uint32_t *ss,
                                              uint32_t K) {
  ChunkRef c;
  c.slot = last_at_or_below(cs, K, ch);
  c.first_chunk = cs[c.slot];
  c.first = ss[c.slot] + (ch - c.first_chunk) * kTile;
  c.nr = min(kTile, ss[c.slot + 1] - c.first);
  return c;
}

// seg_start[0..K] and chunk_start[0..K] of a level into LDS.
__device__ __forceinline__ void stage_starts(const uint32_t *__restrict__ seg_start,
                                             const uint32_t *__restrict__ chunk_start, uint32_t K,
                                             uint32_t *ss, uint32_t *cs) {
  stage_words(seg_start, K + 1, ss);
  stage_words(chunk_start, K + 1, cs);
  __syncthreads();
}

// The split a slot's rows follow (slot_info[slot].x): parameter, threshold,
// and whether each child is searched at the next level (rows of the others
// are dropped).
struct SlotSplit {
  uint32_t j, thr;
  bool lopen, ropen;
};
__device__ __forceinline__ SlotSplit slot_split(uint32_t x) {
  SlotSplit s;
  s.j = x & 255u;
  s.thr = (x >> 8) & 255u;
  s.lopen = (x >> 16) & 1u;
  s.ropen = (x >> 17) & 1u;
  return s;
}

// Rows of each chunk kept for the left and the right child:
// cnt[ch] = n_left | n_right << 32.
__global__ __launch_bounds__(kFitThreads) void fit_pcount(
    const FitDev *__restrict__ fd, int L, const uint32_t *__restrict__ digs_in,
    const uint32_t *__restrict__ seg_start, const uint32_t *__restrict__ chunk_start,
    const uint4 *__restrict__ slot_info, uint64_t *__restrict__ cnt,
    uint32_t *__restrict__ chunk_slot) {
  extern __shared__ uint32_t starts[]; // [K + 1] segment starts, [K + 1] chunk starts
  __shared__ uint64_t scratch[kFitThreads / 64];
  const uint32_t set = L & 1, K = fd->lvl_K[set], NCH = fd->lvl_NCH[set], PW = fd->PW;
  const uint32_t t = threadIdx.x;
  uint32_t *ss = starts, *cs = starts + K + 1;
  stage_starts(seg_start, chunk_start, K, ss, cs);
  for (uint32_t ch = blockIdx.x; ch < NCH; ch += gridDim.x) {
    const ChunkRef c = chunk_ref(ch, cs, ss, K);
    const SlotSplit s = slot_split(slot_info[c.slot].x);
    uint64_t f = 0;
    if (t < c.nr) {
      const bool left = row_digit(digs_in + (uint64_t)(c.first + t) * PW, s.j) <= s.thr;
      if (left ? s.lopen : s.ropen) f = left ? 1ull : (1ull << 32);
    }
    const uint64_t sum = block_sum<kFitThreads>(f, scratch);
    if (t == 0) {
      cnt[ch] = sum;
      chunk_slot[ch] = c.slot;
    }
  }
}

// Moves the rows of level L's open nodes into the segments of their open
// children, chunk by chunk at the offsets the scanned counts give (stable).
__global__ __launch_bounds__(kFitThreads) void fit_partition(
    const FitDev *__restrict__ fd, int L, const uint32_t *__restrict__ rows_in,
    uint32_t *__restrict__ rows_out, const uint32_t *__restrict__ seg_start,
    const uint32_t *__restrict__ chunk_start, const uint64_t *__restrict__ pre,
    const uint4 *__restrict__ slot_info, const uint32_t *__restrict__ chunk_slot,
    uint32_t *__restrict__ digs_out) {
  extern __shared__ uint32_t rl[]; // [kTile][W]
  __shared__ uint32_t s_src[2][kTile];
  __shared__ uint64_t scratch[kFitThreads / 64];
  const uint32_t NCH = fd->lvl_NCH[L & 1], W = fd->W;
  const uint32_t t = threadIdx.x;
  for (uint32_t ch = blockIdx.x; ch < NCH; ch += gridDim.x) {
    // the chunk's slot (found by fit_pcount), then its segment and record
    ChunkRef c;
    c.slot = chunk_slot[ch];
    c.first_chunk = chunk_start[c.slot];
    c.first = seg_start[c.slot] + (ch - c.first_chunk) * kTile;
    c.nr = min(kTile, seg_start[c.slot + 1] - c.first);
    const uint4 info = slot_info[c.slot];
    const SlotSplit s = slot_split(info.x);
    const uint64_t before = pre[ch] - pre[c.first_chunk];
    __syncthreads();
    const uint32_t *src = rows_in + (uint64_t)c.first * W;
    stage_words(src, c.nr * W, rl);
    __syncthreads();
    bool keep = false, left = false;
    if (t < c.nr) {
      left = row_digit(rl + t * W, s.j) <= s.thr;
      keep = left ? s.lopen : s.ropen;
    }
    const uint64_t flag = keep ? (left ? 1ull : (1ull << 32)) : 0ull;
    uint64_t tot;
    const uint64_t rank = block_excl_scan<kFitThreads>(flag, scratch, tot);
    if (keep) {
      if (left) s_src[0][(uint32_t)rank] = t;
      else s_src[1][(uint32_t)(rank >> 32)] = t;
    }
    __syncthreads();
    // offsets within each child's segment (info.y, info.z): kept rows of
    // this segment's earlier chunks
    const uint32_t nl = (uint32_t)tot, nrr = (uint32_t)(tot >> 32);
    // rows and their digit words (the compact copy fit_pcount reads)
    const uint32_t PW = fd->PW;
    const uint32_t bl = info.y + (uint32_t)before, br = info.z + (uint32_t)(before >> 32);
    if (nl) copy_rows_out(rl, s_src[0], nl, W, fd->divW, rows_out, bl, fd->n_train, digs_out, PW);
    if (nrr)
      copy_rows_out(rl, s_src[1], nrr, W, fd->divW, rows_out, br, fd->n_train, digs_out, PW);
  }
}

// Test errors of the cut trees, per staged tile of test rows in two phases:
// one thread per row walks the grown tree (node table in LDS) and records
// the node it reaches at every depth; then thread t handles counter t % C of
// rows t / C, t / C + 256 / C, ... and adds |e| and e^2 at every depth, the
// C lanes of one row reading one node's values together.  Each workgroup
// writes its sums to part[q * gridDim.x + blockIdx.x], q = 3 d + (0: sum |e|,
// 1: sum of the low 32 bits of e^2, 2: sum of the high 32 bits).
// ND >= D + 1 depths are evaluated (a few instantiations cover every D).
template <int ND>
__global__ __launch_bounds__(kFitThreads) void fit_test(const FitDev *__restrict__ fd,
                                                        const uint32_t *__restrict__ test_rows,
                                                        const uint16_t *__restrict__ nodes,
                                                        const int32_t *__restrict__ nmean,
                                                        uint64_t *__restrict__ part) {
  extern __shared__ uint32_t lds[]; // [kTile][W] rows, [kTile][ND] path, nodes
  constexpr int NQ = 3 * (CGS_MAX_DEPTH + 1); // partial sums per workgroup (all depths)
  __shared__ uint64_t s_red[kFitThreads / 64][NQ];
  const uint32_t t = threadIdx.x, n = fd->n_test, C = fd->C, PW = fd->PW, W = fd->W;
  const uint32_t D = fd->D, n_int = (1u << D) - 1;
  uint32_t *rl = lds;
  uint32_t *path = lds + kTile * W; // node * C at every depth
  uint16_t *tree = reinterpret_cast<uint16_t *>(path + kTile * ND);
  stage_words(nodes, n_int, tree);
  const uint32_t RP = kFitThreads / C; // rows per round (C <= 64)
  const uint32_t rs = t / C, c = t - rs * C;
  const bool active = rs < RP;
  // per thread: |e| and e^2 sums (at most 2^46 per term, few terms per thread)
  uint64_t A[ND], B[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) A[d] = B[d] = 0;
  for (uint32_t tile = blockIdx.x; (uint64_t)tile * kTile < n; tile += gridDim.x) {
    const uint32_t first = tile * kTile, nr = min(kTile, n - first);
    __syncthreads();
    const uint32_t *src = test_rows + (uint64_t)first * W;
    stage_words(src, nr * W, rl);
    __syncthreads();
    // every path entry holds a node of the grown tree (depths past D repeat
    // the leaf, rows past the tile the root), so phase two loads without
    // conditions; kFitThreads == kTile, one path per thread
    {
      const uint32_t *row = rl + t * W;
      uint32_t node = 0;
      path[t * ND] = 0;
      for (uint32_t d = 0; d < D; ++d) {
        if (t < nr) {
          const uint16_t nd = tree[node];
          node = 2 * node + (row_digit(row, nd & 255u) <= (uint32_t)(nd >> 8) ? 1u : 2u);
        }
        path[t * ND + d + 1] = node * C;
      }
      for (uint32_t d = D + 1; d < (uint32_t)ND; ++d) path[t * ND + d] = node * C;
    }
    __syncthreads();
    if (active) {
      // four rows per round: their node-value loads are in flight together;
      // only the last round of a tile can hold rows past its end (TAIL)
      auto round = [&](uint32_t r, auto tail) {
        constexpr bool TAIL = decltype(tail)::value;
        int32_t m[4][ND], q[4];
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint32_t ru = r + u * RP;
          ok[u] = !TAIL || ru < nr;
          const uint32_t rr = ok[u] ? ru : r; // r < nr
          q[u] = (int32_t)rl[rr * W + PW + c];
          const uint32_t *pr = path + rr * ND;
#pragma unroll
          for (int d = 0; d < ND; ++d) m[u][d] = nmean[pr[d] + c];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
          for (int d = 0; d < ND; ++d) {
            // |m|, |q| <= 2^22: |e| < 2^24 and e^2 < 2^48; repeated rows
            // count zero, depths past D are never read
            const int32_t e = (!TAIL || ok[u]) ? m[u][d] - q[u] : 0;
            const uint32_t ae = (uint32_t)(e < 0 ? -e : e);
            A[d] += ae;
            B[d] += (uint64_t)ae * ae;
          }
        }
      };
      uint32_t r = rs;
      for (; r + 3 * RP < nr; r += 4 * RP) round(r, std::false_type{});
      if (r < nr) round(r, std::true_type{});
    }
  }
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    const uint64_t a = wave_sum(A[d]);
    const uint64_t l = wave_sum(B[d] & 0xffffffffull), h = wave_sum(B[d] >> 32);
    if ((t & 63u) == 0) {
      s_red[t >> 6][3 * d] = a;
      s_red[t >> 6][3 * d + 1] = l;
      s_red[t >> 6][3 * d + 2] = h;
    }
  }
  for (uint32_t q = 3 * ND + (t & 63u); q < (uint32_t)NQ; q += 64) s_red[t >> 6][q] = 0;
  __syncthreads();
  if (t < (uint32_t)NQ) {
    uint64_t s = 0;
    for (int w = 0; w < kFitThreads / 64; ++w) s += s_red[w][t];
    part[(uint64_t)t * gridDim.x + blockIdx.x] = s;
  }
}

// Sums of the test workgroups' partials (one wave per quantity, exact), then
// the lowest (sum|e|, sum e^2, depth); sum e^2 = Bhi 2^32 + Blo.
__global__ __launch_bounds__(kScanThreads) void fit_select(FitDev *__restrict__ fd,
                                                           const uint64_t *__restrict__ part,
                                                           uint32_t G) {
  constexpr int ND = CGS_MAX_DEPTH + 1;
  const uint32_t t = threadIdx.x, lane = t & 63u;
  for (uint32_t q = t >> 6; q < 3 * ND; q += kScanThreads / 64) {
    uint64_t s = 0;
#pragma unroll
    for (uint32_t i = 0; i < kFitGrid / 64; ++i) { // G <= kFitGrid: all loads in flight
      const uint32_t g = lane + 64 * i;
      if (g < G) s += part[(uint64_t)q * G + g];
    }
    s = wave_sum(s);
    if (lane == 0) {
      const uint32_t d = q / 3, k = q - 3 * d;
      (k == 0 ? fd->A : k == 1 ? fd->Blo : fd->Bhi)[d] = s;
    }
  }
  __syncthreads();
  if (t != 0) return;
  uint32_t best = 0;
  auto hi = [&](uint32_t d) { return fd->Bhi[d] + (fd->Blo[d] >> 32); };
  auto lo = [&](uint32_t d) { return fd->Blo[d] & 0xffffffffull; };
  for (uint32_t d = 1; d <= fd->D; ++d) {
    const bool lt = fd->A[d] < fd->A[best] ||
                    (fd->A[d] == fd->A[best] &&
                     (hi(d) < hi(best) || (hi(d) == hi(best) && lo(d) < lo(best))));
    if (lt) best = d;
  }
  fd->depth_sel = (int32_t)best;
}

// The tree cut at `depth` in the evaluator's layout: heap nodes, leaf
// values float32(m 2^-s_c).
__global__ void fit_emit(const FitDev *__restrict__ fd, int depth,
                         const uint16_t *__restrict__ nodes, const int32_t *__restrict__ nmean,
                         uint16_t *__restrict__ out_nodes, float *__restrict__ out_leaves) {
  const uint32_t C = fd->C, n_int = (1u << depth) - 1, n_leaf_vals = (1u << depth) * C;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < max(n_int, n_leaf_vals);
       i += gridDim.x * blockDim.x) {
    if (i < n_int) out_nodes[i] = nodes[i];
    if (i < n_leaf_vals) {
      const uint32_t c = i % C;
      out_leaves[i] = (float)ldexp((double)nmean[(uint64_t)n_int * C + i], -fd->s[c]);
    }
  }
}

template <typename K> hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

} // namespace

struct TreeFitWork {
  void *base = nullptr;
  FitDev *fd = nullptr;
  uint16_t *nodes = nullptr;
  int32_t *nmean = nullptr;
  int C = 0;
};

hipError_t tree_fit_run(const TreeFitIn &in, TreeFitOut &out, TreeFitWork **work_out,
                        hipStream_t stream) {
  *work_out = nullptr;
  std::memset(&out, 0, sizeof(out));
  const uint32_t n = in.n, C = (uint32_t)in.n_counters, P = (uint32_t)in.n_params;
  const uint32_t D = (uint32_t)in.max_depth;
  const uint32_t n_train = n - n / 2, n_test = n / 2;

  FitDev h{};
  h.n = n;
  h.n_train = n_train;
  h.n_test = n_test;
  h.n_valid = in.n_valid;
  h.C = C;
  h.Cp = C | 1u; // odd LDS stride for the staged targets
  h.P = P;
  h.PW = (P + 3) / 4;
  h.W = h.PW + C;
  h.D = D;
  h.min_leaf = (uint32_t)in.min_leaf;
  h.min_split = std::max<uint32_t>(2u, 2u * (uint32_t)in.min_leaf);
  h.divW = make_fastdiv(h.W);
  h.divC = make_fastdiv(C);
  uint32_t sumR = 0;
  for (uint32_t j = 0; j < P; ++j) {
    h.radix[j] = (uint32_t)in.radix[j];
    h.roff[j] = sumR;
    sumR += (uint32_t)in.radix[j];
  }
  h.roff[P] = sumR;
  h.sumR = sumR;
  h.entries = sumR * (C + 1);
  h.items = P * (C + 1);
  h.key_k = n_train;
  // the level histogram (int64) and a row tile live in LDS: sum_j R_j <= 137
  // for any space with fewer than 2^32 raw configurations, so this always fits
  if ((size_t)h.entries * 8 + (size_t)kHistTile * h.W * 4 > 160 * 1024)
    return hipErrorInvalidValue;

  // open nodes of one level: at most 2^(D-1), and each holds min_split rows
  const uint64_t n_nodes = ((uint64_t)2 << D) - 1;
  const uint64_t n_int = ((uint64_t)1 << D) - 1;
  const uint64_t level_cap = D ? ((uint64_t)1 << (D - 1)) : 1;
  const uint64_t kcap = std::max<uint64_t>(1, std::min<uint64_t>(level_cap, n_train / h.min_split));
  // level histograms, one set per level parity (a derived histogram reads
  // its parent's from the level above)
  const uint64_t hist_entries = D ? 2 * kcap * h.entries : 0;
  const uint64_t n_tiles = ((uint64_t)n + kTile - 1) / kTile;
  const uint64_t max_chunks = (uint64_t)n_train / kTile + kcap + 1;

  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(std::max<size_t>(bytes, 1));
    return o;
  };
  const size_t o_fd = take(sizeof(FitDev));
  const size_t o_hist = take(hist_entries * sizeof(int64_t));
  const size_t o_nsum = take(n_nodes * C * sizeof(int64_t));
  const size_t zero_end = off; // the histograms and node sums start at zero
  const size_t o_rows0 = take((size_t)n_train * h.W * 4);
  const size_t o_rows1 = take(D > 1 ? (size_t)n_train * h.W * 4 : 0);
  // the training rows' digit words alone, per row parity (read by fit_pcount)
  const size_t o_dig0 = take((size_t)n_train * h.PW * 4);
  const size_t o_dig1 = take(D > 1 ? (size_t)n_train * h.PW * 4 : 0);
  const size_t o_test = take((size_t)n_test * h.W * 4);
  const size_t o_ncount = take(n_nodes * 4);
  const size_t o_nmean = take(n_nodes * C * 4);
  const size_t o_nstate = take(n_nodes);
  const size_t o_nodes = take(n_int * 2);
  const size_t o_tcnt = take(n_tiles * 8);
  const size_t o_toff = take(n_tiles * 8);
  const size_t o_ccnt = take(max_chunks * 8);
  const size_t o_cpre = take(max_chunks * 8);
  const size_t o_part = take((size_t)3 * (CGS_MAX_DEPTH + 1) * kFitGrid * 8);
  const size_t o_sinfo = take(kcap * sizeof(uint4));
  const size_t o_cslot = take(max_chunks * 4);
  const size_t o_dpar = take(kcap * 4);
  const size_t o_dsib = take(kcap * 4);
  size_t o_open[2], o_seg[2], o_chs[2], o_slot[2];
  for (int s = 0; s < 2; ++s) {
    o_open[s] = take(kcap * 4);
    o_seg[s] = take((kcap + 1) * 4);
    o_chs[s] = take((kcap + 1) * 4);
    o_slot[s] = take(level_cap * 4);
  }
  char *base = nullptr;
  hipError_t e = hipMalloc(reinterpret_cast<void **>(&base), off);
  if (e != hipSuccess) return e;
  TreeFitWork *w = new (std::nothrow) TreeFitWork();
  if (!w) {
    (void)hipFree(base);
    return hipErrorOutOfMemory;
  }
  w->base = base;
  w->fd = reinterpret_cast<FitDev *>(base + o_fd);
  w->nodes = reinterpret_cast<uint16_t *>(base + o_nodes);
  w->nmean = reinterpret_cast<int32_t *>(base + o_nmean);
  w->C = (int)C;
  *work_out = w;

  FitDev *fd = w->fd;
  int64_t *ghist[2] = {reinterpret_cast<int64_t *>(base + o_hist),
                       reinterpret_cast<int64_t *>(base + o_hist) + hist_entries / 2};
  uint32_t *der_parent = reinterpret_cast<uint32_t *>(base + o_dpar);
  uint64_t *test_part = reinterpret_cast<uint64_t *>(base + o_part);
  uint4 *slot_info = reinterpret_cast<uint4 *>(base + o_sinfo);
  uint32_t *chunk_slot = reinterpret_cast<uint32_t *>(base + o_cslot);
  uint32_t *der_sib = reinterpret_cast<uint32_t *>(base + o_dsib);
  int64_t *nsum = reinterpret_cast<int64_t *>(base + o_nsum);
  uint32_t *rows[2] = {reinterpret_cast<uint32_t *>(base + o_rows0),
                       reinterpret_cast<uint32_t *>(base + o_rows1)};
  uint32_t *digs[2] = {reinterpret_cast<uint32_t *>(base + o_dig0),
                       reinterpret_cast<uint32_t *>(base + o_dig1)};
  uint32_t *test_rows = reinterpret_cast<uint32_t *>(base + o_test);
  uint32_t *ncount = reinterpret_cast<uint32_t *>(base + o_ncount);
  uint8_t *nstate = reinterpret_cast<uint8_t *>(base + o_nstate);
  uint64_t *tile_cnt = reinterpret_cast<uint64_t *>(base + o_tcnt);
  uint64_t *tile_off = reinterpret_cast<uint64_t *>(base + o_toff);
  uint64_t *chunk_cnt = reinterpret_cast<uint64_t *>(base + o_ccnt);
  uint64_t *chunk_pre = reinterpret_cast<uint64_t *>(base + o_cpre);
  uint32_t *open_node[2], *seg_start[2], *chunk_start[2], *slot_of[2];
  for (int s = 0; s < 2; ++s) {
    open_node[s] = reinterpret_cast<uint32_t *>(base + o_open[s]);
    seg_start[s] = reinterpret_cast<uint32_t *>(base + o_seg[s]);
    chunk_start[s] = reinterpret_cast<uint32_t *>(base + o_chs[s]);
    slot_of[s] = reinterpret_cast<uint32_t *>(base + o_slot[s]);
  }

  // launch shapes
  const size_t hist_lds = (size_t)h.entries * 8 + (size_t)kHistTile * h.W * 4;
  const uint32_t cap_entries =
      std::max<uint32_t>(CGS_MAX_RADIX * (C + 1), std::min<uint32_t>(h.entries, 8192));
  const size_t split_lds = (size_t)cap_entries * 8;
  const size_t tile_lds = (size_t)kTile * h.W * 4;
  const size_t starts_lds = (size_t)2 * (kcap + 1) * 4; // a level's segment and chunk starts
  const size_t test_lds = tile_lds + (size_t)kTile * (CGS_MAX_DEPTH + 1) * 4 + n_int * 2;
  const size_t scatter_lds = tile_lds + (size_t)kTile * h.Cp * 4;
  auto grid_for = [](uint64_t items) {
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(kFitGrid, (items + kTile - 1) / kTile));
  };
  const uint32_t g_rows = grid_for(n_train), g_test = grid_for(n_test), g_pts = grid_for(n);
  const uint32_t g_hist =
      (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(kHistGrid, ((uint64_t)n_train + 63) / 64));
  const uint32_t g_chunks = (uint32_t)std::min<uint64_t>(4 * kFitGrid, max_chunks);
  const uint32_t g_derive =
      (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(kFitGrid, (kcap / 2 * h.entries + 255) / 256));

  auto kh = P <= 8 ? fit_hist<8> : P <= 16 ? fit_hist<16> : fit_hist<32>;
  if (e == hipSuccess) e = allow_lds(kh, hist_lds);
  if (e == hipSuccess) e = allow_lds(fit_split, split_lds);
  if (e == hipSuccess) e = allow_lds(fit_pcount, starts_lds);
  if (e == hipSuccess) e = allow_lds(fit_partition, tile_lds);
  static_assert(CGS_MAX_DEPTH + 1 <= 15, "fit_test instantiations");
  auto kt = D + 1 <= 5 ? fit_test<5> : D + 1 <= 9 ? fit_test<9> : D + 1 <= 13 ? fit_test<13>
                                                                               : fit_test<15>;
  if (e == hipSuccess) e = allow_lds(kt, test_lds);
  if (e == hipSuccess) e = allow_lds(fit_scatter, scatter_lds);
  if (e != hipSuccess) return e;

  hipEvent_t ev[2] = {nullptr, nullptr};
  e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  if (e == hipSuccess) e = hipMemcpyAsync(fd, &h, sizeof(h), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipEventRecord(ev[0], stream);
  const uint64_t zwords = (zero_end - o_hist) / 8;
  if (e == hipSuccess) {
    fit_zero<<<(uint32_t)std::min<uint64_t>(2048, (zwords + 255) / 256), 256, 0, stream>>>(
        reinterpret_cast<uint64_t *>(base + o_hist), zwords);
    fit_prepare<<<g_pts, kFitThreads, 0, stream>>>(fd, in.d_points, in.d_targets, in.d_keys);
    fit_key_pick<<<1, 256, 0, stream>>>(fd, 0);
    for (int p = 1; p < 8; ++p) {
      fit_key_hist<<<g_pts, kFitThreads, 0, stream>>>(fd, in.d_keys, p);
      fit_key_pick<<<1, 256, 0, stream>>>(fd, p);
    }
    fit_tile_count<<<g_pts, kFitThreads, 0, stream>>>(fd, in.d_keys, tile_cnt);
    fit_excl_scan<<<1, kScanThreads, 0, stream>>>(tile_cnt, tile_off, nullptr, (uint32_t)n_tiles);
    fit_scatter<<<g_pts, kFitThreads, scatter_lds, stream>>>(fd, in.d_space, in.d_idx,
                                                            in.d_points, in.d_targets,
                                                            in.d_keys, tile_off, rows[0],
                                                            digs[0], test_rows);
    fit_root_sums<<<g_rows, kFitThreads, 0, stream>>>(fd, rows[0], nsum);
    fit_root<<<1, 64, 0, stream>>>(fd, ncount, nsum, w->nmean, nstate);
    if (D > 0)
      fit_layout<<<1, kFitThreads, 0, stream>>>(fd, 0, nstate, ncount, open_node[0],
                                                seg_start[0], chunk_start[0], slot_of[0],
                                                slot_of[1], der_parent, der_sib, slot_info,
                                                (uint32_t)kcap);
    for (uint32_t L = 0; L < D; ++L) {
      const int s = L & 1, s1 = s ^ 1;
      kh<<<g_hist, kFitThreads, hist_lds, stream>>>(fd, (int)L, rows[s], seg_start[s], ghist[s]);
      if (L > 0)
        fit_hist_derive<<<g_derive, kFitThreads, 0, stream>>>(fd, (int)L, ghist[s1], ghist[s],
                                                              der_parent, der_sib,
                                                              (uint32_t)kcap);
      fit_split<<<1u << L, kFitThreads, split_lds, stream>>>(fd, (int)L, ghist[s], slot_of[s],
                                                             cap_entries, ncount, nsum,
                                                             w->nmean, nstate, w->nodes,
                                                             slot_info);
      if (L + 1 < D) {
        fit_layout<<<1, kFitThreads, 0, stream>>>(fd, (int)L + 1, nstate, ncount,
                                                  open_node[s1], seg_start[s1], chunk_start[s1],
                                                  slot_of[s1], slot_of[s], der_parent, der_sib,
                                                  slot_info, (uint32_t)kcap);
        fit_pcount<<<g_chunks, kFitThreads, starts_lds, stream>>>(
            fd, (int)L, digs[s], seg_start[s], chunk_start[s], slot_info, chunk_cnt, chunk_slot);
        fit_excl_scan<<<1, kScanThreads, 0, stream>>>(chunk_cnt, chunk_pre, &fd->lvl_NCH[s], 0);
        fit_partition<<<g_chunks, kFitThreads, tile_lds, stream>>>(
            fd, (int)L, rows[s], rows[s1], seg_start[s], chunk_start[s], chunk_pre, slot_info,
            chunk_slot, digs[s1]);
      }
    }
    kt<<<g_test, kFitThreads, test_lds, stream>>>(fd, test_rows, w->nodes, w->nmean, test_part);
    fit_select<<<1, kScanThreads, 0, stream>>>(fd, test_part, g_test);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(ev[1], stream);
  FitDev r{};
  if (e == hipSuccess) e = hipMemcpyAsync(&r, fd, sizeof(r), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (e != hipSuccess) return e;
  out.err = r.err;
  out.depth = r.depth_sel;
  out.n_train = n_train;
  out.n_test = n_test;
  out.n_split = r.n_split;
  for (uint32_t c = 0; c < C; ++c) out.scale[c] = r.s[c];
  for (uint32_t d = 0; d <= D; ++d) {
    out.abs_err[d] = r.A[d];
    out.sq_lo32[d] = r.Blo[d];
    out.sq_hi32[d] = r.Bhi[d];
  }
  out.ms = ms;
  return hipSuccess;
}

hipError_t tree_fit_emit(const TreeFitWork *w, int depth, uint16_t *d_nodes, float *d_leaves,
                         hipStream_t stream) {
  const uint32_t n = std::max<uint32_t>((1u << depth) - 1, (1u << depth) * (uint32_t)w->C);
  fit_emit<<<std::min<uint32_t>(1024, (n + 255) / 256), 256, 0, stream>>>(
      w->fd, depth, w->nodes, w->nmean, d_nodes, d_leaves);
  return hipGetLastError();
}

void tree_fit_release(TreeFitWork *w) {
  if (!w) return;
  if (w->base) (void)hipFree(w->base);
  delete w;
}

} // namespace cgs
