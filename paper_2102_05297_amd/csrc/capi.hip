// Host runtime of libcgs: argument validation, device buffers, kernel
// sequencing and the extern "C" entry points declared in include/cgs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "cgs.h"
#include "internal.h"
#include "models.h"

using namespace cgs;

// ------------------------------------------------------------------ errors
namespace {

thread_local std::string g_error;

cgs_status fail(cgs_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(e_ == hipErrorOutOfMemory ? CGS_ENOMEM : CGS_EDEVICE, "%s: %s (%s:%d)",     \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                          \
  } while (0)

template <typename T> hipError_t dalloc(T **p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc(reinterpret_cast<void **>(p), n * sizeof(T));
}
template <typename T> void dfree(T *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

constexpr int kVersion = 1;
constexpr int kDefaultBlockLog2 = 12;

} // namespace

// ------------------------------------------------------------------ handles
struct cgs_space_s {
  // 1 for the caller's handle + 1 per live model or session; the space is
  // freed when the count drops to 0, so destruction order does not matter
  int refs = 1;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int n_params = 0;
  std::vector<int32_t> radix;
  uint64_t n_raw = 0, n_valid = 0;
  SpaceDev host_desc{};
  SpaceDev *d_desc = nullptr;
  uint32_t *d_mask = nullptr;
  uint32_t *d_idx = nullptr;
  uint32_t *d_rank = nullptr;  // valid configurations before each mask word
  std::vector<uint32_t> h_idx; // valid raw indices, for raw -> valid lookups
  // scratch for the standalone sampler
  DrawResult *d_res = nullptr;
  DrawResult *h_res = nullptr;
};

struct cgs_model_s {
  cgs_space space = nullptr;
  int kind = 0; // 0 = forest, 1 = perceptron, 2 = least-squares polynomials, 3 = table
  int n_counters = 0;
  float *d_P = nullptr; // predictions [C][stride] of every valid configuration
  uint64_t stride = 0;
  float eval_ms = 0.0f;
  // d_P lags the parameters (a perceptron retrained inside cgs_online_run
  // whose predictions are not needed yet); never true outside that call
  bool p_stale = false;
  // forest
  int n_trees = 0, depth = 0;
  uint16_t *d_nodes = nullptr;
  float *d_leaves = nullptr;
  // perceptron: fp32 master parameters, Adam moments, gradient, packed bf16
  MlpShape sh{};
  uint64_t n_theta = 0;
  size_t off_b1 = 0, off_w2 = 0, off_b2 = 0, off_w3 = 0, off_b3 = 0;
  float *d_theta = nullptr, *d_m = nullptr, *d_v = nullptr, *d_grad = nullptr;
  __bf16 *d_w1p = nullptr, *d_w2p = nullptr, *d_w3p = nullptr;
  __bf16 *d_w2t = nullptr, *d_w3t = nullptr; // [H][H], [H][Cp]: backward operands
  __bf16 *d_w1n = nullptr, *d_w2n = nullptr, *d_w3n = nullptr; // row-major, training forward
  size_t n_w1p = 0, n_w2p = 0, n_w3p = 0;
  uint64_t adam_t = 0;
  int n_cu = 256;
  // training step buffers for batches of up to scratch_rows rows: the
  // weight gradients' operands [feature][rows rounded up to 32] (bf16), the
  // per-block column sums and squared errors, and Y of the forward pass
  uint32_t scratch_rows = 0;
  __bf16 *d_xt = nullptr, *d_h1t = nullptr, *d_h2t = nullptr, *d_dyt = nullptr,
         *d_dz2t = nullptr, *d_dz1t = nullptr;
  float *d_bp1 = nullptr, *d_bp2 = nullptr, *d_bp3 = nullptr, *d_lossp = nullptr,
        *d_y = nullptr;
  // gathered features [kGatherSteps][rows rounded up to 32][K1] and targets
  // [kGatherSteps][rows][C] of a run of steps
  __bf16 *d_xg = nullptr;
  float *d_tg = nullptr;
  // least-squares polynomials: descriptor and coefficients [S][T][C]
  PolyDev poly{};
  PolyDev *d_poly = nullptr;
  double *d_beta64 = nullptr;
  float *d_beta32 = nullptr;
};

constexpr uint32_t kTimeEvents = 512; // event markers of 128 timed steps
constexpr uint32_t kGatherSteps = 64;  // perceptron training steps gathered at once
constexpr uint32_t kResultRing = 256; // draw results of steps enqueued ahead

// Launches between consecutive markers t_ev[ev .. ev + n]: kernel k runs
// between markers ev + k and ev + k + 1.
struct TimedSpan {
  uint32_t ev;
  int n;
  int kind[3]; // 0 score, 1 weight, 2 draw, 3 profile mark, 4 neighbourhood score / finish
};

struct cgs_session_s {
  cgs_space space = nullptr;
  cgs_params params{};
  int block_log2 = kDefaultBlockLog2;
  uint32_t n_blocks = 0;
  uint32_t *d_explored = nullptr;
  float *d_s = nullptr;
  uint64_t *d_bsum = nullptr;
  StepAcc *d_acc = nullptr; // [2][kAccSlots]
  DrawResult *d_res = nullptr;
  DrawResult *h_res = nullptr; // pinned
  StepAcc *h_acc = nullptr;    // pinned, [kAccSlots]
  // timing mode: event markers (timing only, no system-scope fence) around
  // the kernels of every params.timing-th step, summed when the pool is
  // full or when times are read, so reading them costs the step loop nothing
  std::vector<hipEvent_t> t_ev; // kTimeEvents markers
  uint32_t t_ev_used = 0;
  std::vector<TimedSpan> t_spans;
  int32_t t_step = -1;  // span of the last timed step, -1 once summed
  float step_ms = 0.0f; // score start to first draw end of the last timed step
  uint64_t n_launched = 0; // steps launched so far
  bool step_timed = false; // the last launched step is timed
  double kernel_ms[4] = {0, 0, 0, 0};
  uint64_t kernel_n[4] = {0, 0, 0, 0};
  // the recorded step, launched with its first draw (or when results are read)
  bool pending = false;
  cgs_model pending_model = nullptr;
  uint32_t pending_profile = kNoProfile;
  ActiveCounters pending_act{};
  int parity = 0;     // accumulator set of the next launched step
  int cur_acc = 0;    // accumulator set of the last launched step
  bool stepped = false;
  // neighbourhood-restricted steps: the recorded one, the last launched one,
  // the subset table on the device (built per radius) and candidate buffers
  bool pending_nb = false;
  NbStep pending_nbstep{};
  bool last_nb = false;
  int nb_radius = 0;
  uint32_t *d_sub_off = nullptr, *d_sub_code = nullptr;
  uint32_t *d_nb_tmp_idx = nullptr, *d_nb_idx = nullptr, *d_nb_q = nullptr;
  float *d_nb_tmp_s = nullptr, *d_nb_s = nullptr;
  uint64_t *d_nb_bsum = nullptr;
  NbStats *d_nb_stats = nullptr;
  StepAcc *d_nb_acc = nullptr;
  bool ran_in_batch = false; // the last step ran inside a batch step
  float batch_ms = 0.0f;     // device time of that batch step
  uint64_t seq = 0;          // sequence number of the last launched draw
  int n_active = 0;
  uint64_t last_total = 0;
  // steps enqueued ahead of their picks (cgs_search_run): the profiled
  // configuration passes between steps in device memory (two words used
  // alternately), the results land in a ring of pinned slots
  uint32_t *d_prof = nullptr;     // [2]
  DrawResult *h_ring = nullptr;   // pinned, mapped, [kResultRing]
  DrawResult *d_ring = nullptr;
};

// ------------------------------------------------------------------ misc
extern "C" const char *cgs_last_error(void) { return g_error.c_str(); }
extern "C" int cgs_version(void) { return kVersion; }

extern "C" void cgs_default_params(cgs_params *out) {
  if (!out) return;
  out->gamma = -0.25f;
  out->w_min = 1e-4f;
  out->block_log2 = 0;
  out->timing = 0;
}

extern "C" void cgs_default_expert_params(cgs_expert_params *out) {
  if (!out) return;
  out->inst_reaction = 0.7;
  out->volta = 0;
  out->reserved = 0;
  out->cores = 1.0;
  out->threads = 5.0;
}

extern "C" cgs_status cgs_synchronize(cgs_space sp) {
  if (!sp) return fail(CGS_EINVAL, "cgs_synchronize: NULL space");
  HIP_TRY(hipStreamSynchronize(sp->stream));
  return CGS_OK;
}

// ------------------------------------------------------------------ space
FastDiv cgs::make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  const uint64_t m = ((((uint64_t)1 << l) - d) << 32) / d + 1;
  const uint32_t sh1 = l < 1 ? l : 1, sh2 = l > 1 ? l - 1 : 0;
  return FastDiv{(uint32_t)m, sh1 | (sh2 << 8)};
}

namespace {

void destroy_space(cgs_space sp) {
  if (!sp) return;
  if (--sp->refs > 0) return;
  if (sp->stream) (void)hipStreamSynchronize(sp->stream);
  dfree(sp->d_desc);
  dfree(sp->d_mask);
  dfree(sp->d_idx);
  dfree(sp->d_rank);
  if (sp->h_res) (void)hipHostFree(sp->h_res);
  if (sp->own_stream && sp->stream) (void)hipStreamDestroy(sp->stream);
  delete sp;
}

} // namespace

extern "C" cgs_status cgs_space_create(int n_params, const int32_t *radix, const int64_t *values,
                                       int n_cons, const cgs_constraint *cons, void *hip_stream,
                                       cgs_space *out) {
  if (!out) return fail(CGS_EINVAL, "cgs_space_create: NULL out");
  *out = nullptr;
  if (n_params < 1 || n_params > CGS_MAX_PARAMS)
    return fail(CGS_ERANGE, "n_params %d outside 1..%d", n_params, CGS_MAX_PARAMS);
  if (!radix || !values) return fail(CGS_EINVAL, "NULL radix or values");
  if (n_cons < 0 || n_cons > CGS_MAX_CONSTRAINTS)
    return fail(CGS_ERANGE, "n_cons %d outside 0..%d", n_cons, CGS_MAX_CONSTRAINTS);
  if (n_cons > 0 && !cons) return fail(CGS_EINVAL, "NULL constraints");

  SpaceDev desc{};
  desc.n_params = n_params;
  desc.n_cons = n_cons;
  uint64_t n_raw = 1;
  size_t off = 0;
  for (int j = 0; j < n_params; ++j) {
    const int32_t r = radix[j];
    if (r < 1 || r > CGS_MAX_RADIX)
      return fail(CGS_ERANGE, "radix[%d] = %d outside 1..%d", j, r, CGS_MAX_RADIX);
    n_raw *= (uint64_t)r;
    if (n_raw > 0xffffffffull)
      return fail(CGS_ERANGE, "raw space size exceeds 2^32 - 1 configurations");
    desc.radix[j] = (uint32_t)r;
    desc.div[j] = make_fastdiv((uint32_t)r);
    for (int d = 0; d < r; ++d) {
      const int64_t v = values[off + d];
      if (v <= -CGS_MAX_ABS_VALUE || v >= CGS_MAX_ABS_VALUE)
        return fail(CGS_ERANGE, "value %lld of parameter %d: |v| must be < %d", (long long)v, j,
                    CGS_MAX_ABS_VALUE);
      if (d > 0 && !(values[off + d - 1] < v))
        return fail(CGS_EINVAL, "values of parameter %d are not strictly ascending", j);
      desc.table[j * CGS_MAX_RADIX + d] = (int32_t)v;
    }
    off += (size_t)r;
  }
  for (int c = 0; c < n_cons; ++c) {
    const cgs_constraint &k = cons[c];
    if (k.kind < CGS_DIV || k.kind > CGS_LE)
      return fail(CGS_EINVAL, "constraint %d: unknown kind %d", c, k.kind);
    if (k.a < 0 || k.a >= n_params || k.b < 0 || k.b >= n_params || k.c < 0 || k.c >= n_params)
      return fail(CGS_EINVAL, "constraint %d: parameter index out of range", c);
    desc.cons_code[c] = (uint32_t)k.kind | ((uint32_t)k.a << 8) | ((uint32_t)k.b << 16) |
                        ((uint32_t)k.c << 24);
    desc.cons_bound[c] = k.bound;
  }
  desc.n_raw = (uint32_t)n_raw;
  desc.n_words = (uint32_t)((n_raw + 31) / 32);

  cgs_space sp = new (std::nothrow) cgs_space_s();
  if (!sp) return fail(CGS_ENOMEM, "host allocation");
  sp->n_params = n_params;
  sp->radix.assign(radix, radix + n_params);
  sp->n_raw = n_raw;
  sp->host_desc = desc;
  cgs_status st = CGS_OK;
  auto guard = [&](cgs_status s) {
    destroy_space(sp);
    return s;
  };
#define SP_TRY(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return guard(fail(e_ == hipErrorOutOfMemory ? CGS_ENOMEM : CGS_EDEVICE, "%s: %s", #expr,  \
                        hipGetErrorString(e_)));                                              \
  } while (0)

  if (hip_stream) {
    sp->stream = reinterpret_cast<hipStream_t>(hip_stream);
  } else {
    SP_TRY(hipStreamCreateWithFlags(&sp->stream, hipStreamNonBlocking));
    sp->own_stream = true;
  }
  SP_TRY(dalloc(&sp->d_desc, 1));
  SP_TRY(dalloc(&sp->d_mask, desc.n_words));
  SP_TRY(dalloc(&sp->d_rank, desc.n_words));
  SP_TRY(hipHostMalloc(reinterpret_cast<void **>(&sp->h_res), sizeof(DrawResult),
                       hipHostMallocMapped));
  SP_TRY(hipHostGetDevicePointer(reinterpret_cast<void **>(&sp->d_res), sp->h_res, 0));
  const uint32_t n_tiles = enumeration_tiles((uint32_t)n_raw);
  uint32_t *d_tile_count = nullptr, *d_tile_off = nullptr;
  uint64_t *d_total = nullptr;
  SP_TRY(dalloc(&d_tile_count, n_tiles));
  SP_TRY(dalloc(&d_tile_off, n_tiles));
  SP_TRY(dalloc(&d_total, 1));
  auto free_tmp = [&]() {
    dfree(d_tile_count);
    dfree(d_tile_off);
    dfree(d_total);
  };
  hipError_t e = hipMemcpyAsync(sp->d_desc, &desc, sizeof(desc), hipMemcpyHostToDevice, sp->stream);
  if (e == hipSuccess)
    e = launch_enumeration(sp->d_desc, (uint32_t)n_raw, sp->d_mask, d_tile_count, d_tile_off,
                           d_total, nullptr, nullptr, 0, sp->stream);
  uint64_t n_valid = 0;
  if (e == hipSuccess)
    e = hipMemcpyAsync(&n_valid, d_total, sizeof(uint64_t), hipMemcpyDeviceToHost, sp->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(sp->stream);
  if (e == hipSuccess) e = dalloc(&sp->d_idx, n_valid);
  if (e == hipSuccess && n_valid > 0)
    e = launch_enumeration(sp->d_desc, (uint32_t)n_raw, sp->d_mask, d_tile_count, d_tile_off,
                           d_total, sp->d_idx, sp->d_rank, 1, sp->stream);
  if (e == hipSuccess && n_valid > 0) {
    try {
      sp->h_idx.resize(n_valid);
    } catch (...) {
      free_tmp();
      return guard(fail(CGS_ENOMEM, "host copy of the valid list"));
    }
    e = hipMemcpyAsync(sp->h_idx.data(), sp->d_idx, n_valid * sizeof(uint32_t),
                       hipMemcpyDeviceToHost, sp->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(sp->stream);
  free_tmp();
  if (e != hipSuccess)
    return guard(fail(e == hipErrorOutOfMemory ? CGS_ENOMEM : CGS_EDEVICE, "enumeration: %s",
                      hipGetErrorString(e)));
  sp->n_valid = n_valid;
  *out = sp;
  (void)st;
  return CGS_OK;
#undef SP_TRY
}

extern "C" cgs_status cgs_space_info(cgs_space sp, uint64_t *n_raw, uint64_t *n_valid) {
  if (!sp) return fail(CGS_EINVAL, "NULL space");
  if (n_raw) *n_raw = sp->n_raw;
  if (n_valid) *n_valid = sp->n_valid;
  return CGS_OK;
}

extern "C" cgs_status cgs_space_decode(cgs_space sp, uint64_t k, int32_t *digits) {
  if (!sp || !digits) return fail(CGS_EINVAL, "NULL argument");
  if (k >= sp->n_raw) return fail(CGS_ERANGE, "raw index %llu >= n_raw", (unsigned long long)k);
  for (int j = sp->n_params - 1; j >= 0; --j) {
    digits[j] = (int32_t)(k % (uint64_t)sp->radix[j]);
    k /= (uint64_t)sp->radix[j];
  }
  return CGS_OK;
}

namespace {
int64_t valid_index_of(cgs_space sp, uint64_t k) {
  if (k >= sp->n_raw) return -1;
  auto it = std::lower_bound(sp->h_idx.begin(), sp->h_idx.end(), (uint32_t)k);
  if (it == sp->h_idx.end() || *it != (uint32_t)k) return -1;
  return (int64_t)(it - sp->h_idx.begin());
}
} // namespace

extern "C" cgs_status cgs_space_valid_index(cgs_space sp, uint64_t k, int64_t *out) {
  if (!sp || !out) return fail(CGS_EINVAL, "NULL argument");
  *out = valid_index_of(sp, k);
  return CGS_OK;
}

extern "C" cgs_status cgs_space_copy_valid(cgs_space sp, uint64_t first, uint64_t count,
                                           uint32_t *dst) {
  if (!sp || (!dst && count)) return fail(CGS_EINVAL, "NULL argument");
  if (first > sp->n_valid || count > sp->n_valid - first)
    return fail(CGS_ERANGE, "range [%llu, +%llu) outside the valid list", (unsigned long long)first,
                (unsigned long long)count);
  if (count == 0) return CGS_OK;
  HIP_TRY(hipMemcpyAsync(dst, sp->d_idx + first, count * sizeof(uint32_t), hipMemcpyDeviceToHost,
                         sp->stream));
  HIP_TRY(hipStreamSynchronize(sp->stream));
  return CGS_OK;
}

extern "C" cgs_status cgs_space_copy_mask(cgs_space sp, uint32_t *dst, uint64_t n_words) {
  if (!sp || !dst) return fail(CGS_EINVAL, "NULL argument");
  if (n_words != sp->host_desc.n_words)
    return fail(CGS_EINVAL, "mask has %u words, %llu requested", sp->host_desc.n_words,
                (unsigned long long)n_words);
  HIP_TRY(hipMemcpyAsync(dst, sp->d_mask, n_words * sizeof(uint32_t), hipMemcpyDeviceToHost,
                         sp->stream));
  HIP_TRY(hipStreamSynchronize(sp->stream));
  return CGS_OK;
}

extern "C" void cgs_space_destroy(cgs_space sp) { destroy_space(sp); }

// ------------------------------------------------------------------ model
namespace {

void free_mlp_scratch(cgs_model m) {
  dfree(m->d_xt);
  dfree(m->d_h1t);
  dfree(m->d_h2t);
  dfree(m->d_dyt);
  dfree(m->d_dz2t);
  dfree(m->d_dz1t);
  dfree(m->d_bp1);
  dfree(m->d_bp2);
  dfree(m->d_bp3);
  dfree(m->d_lossp);
  dfree(m->d_y);
  dfree(m->d_xg);
  dfree(m->d_tg);
  m->scratch_rows = 0;
}

void destroy_model(cgs_model m) {
  if (!m) return;
  if (m->space && m->space->stream) (void)hipStreamSynchronize(m->space->stream);
  dfree(m->d_nodes);
  dfree(m->d_leaves);
  dfree(m->d_P);
  dfree(m->d_theta);
  dfree(m->d_m);
  dfree(m->d_v);
  dfree(m->d_grad);
  dfree(m->d_w1p);
  dfree(m->d_w2p);
  dfree(m->d_w3p);
  dfree(m->d_w2t);
  dfree(m->d_w3t);
  dfree(m->d_w1n);
  dfree(m->d_w2n);
  dfree(m->d_w3n);
  dfree(m->d_poly);
  dfree(m->d_beta64);
  dfree(m->d_beta32);
  free_mlp_scratch(m);
  destroy_space(m->space);
  delete m;
}

MlpCopies mlp_copies(cgs_model m) {
  return MlpCopies{m->d_w1p, m->d_w2p, m->d_w3p, m->d_w2t, m->d_w3t,
                   m->d_w1n, m->d_w2n, m->d_w3n};
}

MlpFwdArgs mlp_args(cgs_model m) {
  cgs_space sp = m->space;
  MlpFwdArgs a{};
  a.sp = sp->d_desc;
  a.idx = sp->d_idx;
  a.F = m->sh.F;
  a.H = m->sh.H;
  a.C = m->sh.C;
  a.K1 = m->sh.K1;
  a.n_cu = m->n_cu;
  a.w1p = reinterpret_cast<const bf16x8 *>(m->d_w1p);
  a.w2p = reinterpret_cast<const bf16x8 *>(m->d_w2p);
  a.w3p = reinterpret_cast<const bf16x8 *>(m->d_w3p);
  a.b1 = m->d_theta + m->off_b1;
  a.b2 = m->d_theta + m->off_b2;
  a.b3 = m->d_theta + m->off_b3;
  a.P = m->d_P;
  a.stride = m->stride;
  return a;
}

cgs_status evaluate_model(cgs_model m) {
  cgs_space sp = m->space;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, sp->stream));
  hipError_t e = hipSuccess;
  if (m->kind == 0) {
    e = launch_forest_eval(sp->d_desc, sp->d_idx, (uint32_t)sp->n_valid, m->d_nodes, m->d_leaves,
                           m->n_trees, m->depth, m->n_counters, m->d_P, m->stride, nullptr, 0, 0,
                           sp->stream);
  } else if (m->kind == 3) {
    // predictions given by the caller: nothing to evaluate
  } else if (m->kind == 2) {
    e = launch_poly_eval(m->d_poly, m->poly.T, m->poly.C, m->poly.S, sp->d_desc, sp->d_idx,
                         (uint32_t)sp->n_valid, m->d_beta32, m->d_P, m->stride, sp->stream);
  } else {
    MlpFwdArgs a = mlp_args(m);
    a.n = (uint32_t)sp->n_valid;
    e = launch_mlp_forward(a, false, sp->stream);
  }
  if (e == hipSuccess) e = hipEventRecord(e1, sp->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(CGS_EDEVICE, "model evaluation: %s", hipGetErrorString(e));
  m->eval_ms = ms;
  return CGS_OK;
}

} // namespace

extern "C" cgs_status cgs_model_load_forest(cgs_space sp, int n_trees, int depth, int n_counters,
                                            const uint8_t *feat, const uint8_t *thr,
                                            const float *leaves, cgs_model *out) {
  if (!out) return fail(CGS_EINVAL, "NULL out");
  *out = nullptr;
  if (!sp || !leaves || (depth > 0 && (!feat || !thr))) return fail(CGS_EINVAL, "NULL argument");
  if (n_trees < 1 || n_trees > CGS_MAX_TREES)
    return fail(CGS_ERANGE, "n_trees %d outside 1..%d", n_trees, CGS_MAX_TREES);
  if (depth < 0 || depth > CGS_MAX_DEPTH)
    return fail(CGS_ERANGE, "depth %d outside 0..%d", depth, CGS_MAX_DEPTH);
  if (n_counters < 1 || n_counters > CGS_MAX_COUNTERS)
    return fail(CGS_ERANGE, "n_counters %d outside 1..%d", n_counters, CGS_MAX_COUNTERS);
  const size_t n_int = ((size_t)1 << depth) - 1, n_leaf = (size_t)1 << depth;
  std::vector<uint16_t> nodes((size_t)n_trees * n_int);
  for (size_t i = 0; i < nodes.size(); ++i) {
    const uint8_t f = feat[i];
    if (f >= sp->n_params)
      return fail(CGS_EINVAL, "node %zu splits on parameter %u of %d", i, f, sp->n_params);
    nodes[i] = (uint16_t)(f | ((uint16_t)thr[i] << 8));
  }
  const size_t n_leaf_vals = (size_t)n_trees * n_leaf * n_counters;
  for (size_t i = 0; i < n_leaf_vals; ++i)
    if (!(leaves[i] >= 0.0f) || !std::isfinite(leaves[i]))
      return fail(CGS_EINVAL, "leaf value %zu is negative or not finite", i);

  cgs_model m = new (std::nothrow) cgs_model_s();
  if (!m) return fail(CGS_ENOMEM, "host allocation");
  m->space = sp;
  ++sp->refs;
  m->kind = 0;
  m->n_counters = n_counters;
  m->n_trees = n_trees;
  m->depth = depth;
  m->stride = (sp->n_valid + 63) & ~(uint64_t)63;
  hipError_t e = dalloc(&m->d_nodes, nodes.size());
  if (e == hipSuccess) e = dalloc(&m->d_leaves, n_leaf_vals);
  if (e == hipSuccess) e = dalloc(&m->d_P, (size_t)n_counters * m->stride);
  if (e == hipSuccess && !nodes.empty())
    e = hipMemcpyAsync(m->d_nodes, nodes.data(), nodes.size() * sizeof(uint16_t),
                       hipMemcpyHostToDevice, sp->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(m->d_leaves, leaves, n_leaf_vals * sizeof(float), hipMemcpyHostToDevice,
                       sp->stream);
  // padding columns of P (past n_valid) hold zeros
  if (e == hipSuccess)
    e = hipMemsetAsync(m->d_P, 0, (size_t)n_counters * m->stride * sizeof(float), sp->stream);
  if (e != hipSuccess) {
    destroy_model(m);
    return fail(e == hipErrorOutOfMemory ? CGS_ENOMEM : CGS_EDEVICE, "model buffers: %s",
                hipGetErrorString(e));
  }
  const cgs_status st = evaluate_model(m);
  if (st != CGS_OK) {
    destroy_model(m);
    return st;
  }
  *out = m;
  return CGS_OK;
}

extern "C" cgs_status cgs_model_fit_tree(cgs_space sp, uint64_t n, int n_counters,
                                         const uint32_t *points, const float *targets,
                                         const uint64_t *keys, int max_depth, int min_leaf,
                                         cgs_model *out, cgs_tree_fit_report *report) {
  if (!out) return fail(CGS_EINVAL, "NULL out");
  *out = nullptr;
  if (!sp || !points || !targets || !keys) return fail(CGS_EINVAL, "NULL argument");
  if (n_counters < 1 || n_counters > CGS_MAX_COUNTERS)
    return fail(CGS_ERANGE, "n_counters %d outside 1..%d", n_counters, CGS_MAX_COUNTERS);
  if (n < 2 || n * (uint64_t)n_counters >= ((uint64_t)1 << 31))
    return fail(CGS_ERANGE, "need 2 <= n and n * n_counters < 2^31 (n = %llu)",
                (unsigned long long)n);
  if (max_depth < 0 || max_depth > CGS_MAX_DEPTH)
    return fail(CGS_ERANGE, "max_depth %d outside 0..%d", max_depth, CGS_MAX_DEPTH);
  if (min_leaf < 1 || (uint64_t)min_leaf > n)
    return fail(CGS_ERANGE, "min_leaf %d outside 1..n", min_leaf);
  if (sp->n_valid == 0) return fail(CGS_EEMPTY, "the space has no valid configuration");

  uint32_t *d_pts = nullptr;
  float *d_y = nullptr;
  uint64_t *d_keys = nullptr;
  TreeFitWork *work = nullptr;
  cgs_model m = nullptr;
  auto cleanup = [&]() {
    if (sp->stream) (void)hipStreamSynchronize(sp->stream);
    dfree(d_pts);
    dfree(d_y);
    dfree(d_keys);
    tree_fit_release(work);
    work = nullptr;
  };
  hipError_t e = dalloc(&d_pts, n);
  if (e == hipSuccess) e = dalloc(&d_y, n * (size_t)n_counters);
  if (e == hipSuccess) e = dalloc(&d_keys, n);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_pts, points, n * 4, hipMemcpyHostToDevice, sp->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_y, targets, n * (size_t)n_counters * 4, hipMemcpyHostToDevice,
                       sp->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_keys, keys, n * 8, hipMemcpyHostToDevice, sp->stream);
  TreeFitOut fo{};
  if (e == hipSuccess) {
    TreeFitIn in{};
    in.d_space = sp->d_desc;
    in.d_idx = sp->d_idx;
    in.n_valid = (uint32_t)sp->n_valid;
    in.n_params = sp->n_params;
    in.radix = sp->radix.data();
    in.n = (uint32_t)n;
    in.n_counters = n_counters;
    in.d_points = d_pts;
    in.d_targets = d_y;
    in.d_keys = d_keys;
    in.max_depth = max_depth;
    in.min_leaf = min_leaf;
    e = tree_fit_run(in, fo, &work, sp->stream);
  }
  if (e != hipSuccess) {
    cleanup();
    return fail(e == hipErrorOutOfMemory ? CGS_ENOMEM : CGS_EDEVICE, "tree fit: %s",
                hipGetErrorString(e));
  }
  if (fo.err) {
    cleanup();
    return fail(CGS_EINVAL, "%s", (fo.err & 1u) ? "a point is outside the valid list"
                                                : "a target is negative or not finite");
  }
  const int depth = fo.depth;
  m = new (std::nothrow) cgs_model_s();
  if (!m) {
    cleanup();
    return fail(CGS_ENOMEM, "host allocation");
  }
  m->space = sp;
  ++sp->refs;
  m->kind = 0;
  m->n_counters = n_counters;
  m->n_trees = 1;
  m->depth = depth;
  m->stride = (sp->n_valid + 63) & ~(uint64_t)63;
  const size_t n_int = ((size_t)1 << depth) - 1, n_leaf_vals = ((size_t)1 << depth) * n_counters;
  e = dalloc(&m->d_nodes, n_int);
  if (e == hipSuccess) e = dalloc(&m->d_leaves, n_leaf_vals);
  if (e == hipSuccess) e = dalloc(&m->d_P, (size_t)n_counters * m->stride);
  if (e == hipSuccess) e = tree_fit_emit(work, depth, m->d_nodes, m->d_leaves, sp->stream);
  if (e == hipSuccess)
    e = hipMemsetAsync(m->d_P, 0, (size_t)n_counters * m->stride * sizeof(float), sp->stream);
  cleanup();
  if (e != hipSuccess) {
    destroy_model(m);
    return fail(e == hipErrorOutOfMemory ? CGS_ENOMEM : CGS_EDEVICE, "fitted model: %s",
                hipGetErrorString(e));
  }
  const cgs_status st = evaluate_model(m);
  if (st != CGS_OK) {
    destroy_model(m);
    return st;
  }
  if (report) {
    std::memset(report, 0, sizeof(*report));
    report->depth = depth;
    report->max_depth = max_depth;
    report->min_leaf = min_leaf;
    report->n_counters = n_counters;
    report->n_train = fo.n_train;
    report->n_test = fo.n_test;
    report->n_split = fo.n_split;
    report->fit_ms = fo.ms;
    for (int c = 0; c < n_counters; ++c) report->scale_log2[c] = fo.scale[c];
    for (int d = 0; d <= max_depth; ++d) {
      report->abs_err[d] = fo.abs_err[d];
      const unsigned __int128 b =
          ((unsigned __int128)fo.sq_hi32[d] << 32) + (unsigned __int128)fo.sq_lo32[d];
      report->sq_err[d][0] = (uint64_t)b;
      report->sq_err[d][1] = (uint64_t)(b >> 64);
    }
  }
  *out = m;
  return CGS_OK;
}

// ------------------------------------------------------- polynomial models
namespace {

// Digit of parameter j whose value is nearest to the middle of its range
// (the lower one on a tie).
int mid_digit(const cgs_space_s *sp, int j) {
  const int r = sp->radix[j];
  const double lo = sp->host_desc.table[j * CGS_MAX_RADIX],
               hi = sp->host_desc.table[j * CGS_MAX_RADIX + r - 1];
  const double mid = (lo + hi) / 2.0;
  int best = 0;
  for (int d = 1; d < r; ++d)
    if (std::fabs(sp->host_desc.table[j * CGS_MAX_RADIX + d] - mid) <
        std::fabs(sp->host_desc.table[j * CGS_MAX_RADIX + best] - mid))
      best = d;
  return best;
}

// Binary parameters (two values) pick the subspace; non-binary ones (three or
// more) carry features; the basis is every set of non-binary parameters of
// size <= order (by size, then lexicographically), then their squares.
cgs_status poly_describe(const cgs_space_s *sp, int order, int n_counters, PolyDev &pd) {
  std::memset(&pd, 0, sizeof(pd));
  std::vector<int> nb;
  for (int j = 0; j < sp->n_params; ++j) {
    if (sp->radix[j] == 2) {
      if (pd.B >= kPolyMaxBinary)
        return fail(CGS_ERANGE, "more than %d binary parameters", kPolyMaxBinary);
      pd.bin_params[pd.B++] = (uint32_t)j;
    } else if (sp->radix[j] >= 3) {
      nb.push_back(j);
    }
  }
  pd.P = sp->n_params;
  pd.k = (int)nb.size();
  pd.S = 1 << pd.B;
  pd.C = n_counters;
  pd.order = order;
  std::vector<uint32_t> terms;
  const int k = pd.k, top = std::min(order, k);
  for (int size = 0; size <= top && terms.size() <= (size_t)kPolyMaxTerms; ++size) {
    std::vector<int> pick(size);
    for (int i = 0; i < size; ++i) pick[i] = i;
    while (terms.size() <= (size_t)kPolyMaxTerms) {
      uint32_t d = (uint32_t)size;
      for (int i = 0; i < size; ++i) d |= (uint32_t)nb[pick[i]] << (3 + 5 * i);
      terms.push_back(d);
      int i = size - 1;
      while (i >= 0 && pick[i] == k - size + i) --i;
      if (i < 0) break;
      ++pick[i];
      for (int q = i + 1; q < size; ++q) pick[q] = pick[q - 1] + 1;
    }
  }
  for (int i = 0; i < k && terms.size() <= (size_t)kPolyMaxTerms; ++i)
    terms.push_back(2u | ((uint32_t)nb[i] << 3) | ((uint32_t)nb[i] << 8));
  if (terms.size() > (size_t)kPolyMaxTerms)
    return fail(CGS_ERANGE, "order %d gives more than %d basis terms for %d non-binary parameters",
                order, kPolyMaxTerms, k);
  pd.T = (int)terms.size();
  for (size_t i = 0; i < terms.size(); ++i) pd.terms[i] = terms[i];
  for (int j : nb) {
    const int r = sp->radix[j];
    const double lo = sp->host_desc.table[j * CGS_MAX_RADIX],
                 hi = sp->host_desc.table[j * CGS_MAX_RADIX + r - 1];
    for (int d = 0; d < r; ++d) {
      const double v = sp->host_desc.table[j * CGS_MAX_RADIX + d];
      const double x = (2.0 * v - hi - lo) / (hi - lo);
      pd.xv64[j * CGS_MAX_RADIX + d] = x;
      pd.xv32[j * CGS_MAX_RADIX + d] = (float)x;
    }
  }
  return CGS_OK;
}

} // namespace

extern "C" cgs_status cgs_poly_design(cgs_space sp, uint64_t capacity, uint32_t *valid_idx,
                                      uint64_t *count) {
  if (!sp || !count || (capacity && !valid_idx)) return fail(CGS_EINVAL, "NULL argument");
  *count = 0;
  const uint32_t nv = (uint32_t)sp->n_valid;
  if (nv == 0) return CGS_OK;
  std::vector<uint32_t> allowed(CGS_MAX_PARAMS, 0);
  for (int j = 0; j < sp->n_params; ++j) {
    const int r = sp->radix[j];
    if (r >= 3) allowed[j] = (1u << 0) | (1u << mid_digit(sp, j)) | (1u << (r - 1));
    else allowed[j] = (1u << r) - 1u;
  }
  const uint32_t tiles = (nv + 255) / 256;
  uint32_t *d_allowed = nullptr, *d_out = nullptr;
  uint64_t *d_cnt = nullptr, *d_off = nullptr;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(sp->stream);
    dfree(d_allowed);
    dfree(d_out);
    dfree(d_cnt);
    dfree(d_off);
  };
  hipError_t e = dalloc(&d_allowed, CGS_MAX_PARAMS);
  if (e == hipSuccess) e = dalloc(&d_out, nv);
  if (e == hipSuccess) e = dalloc(&d_cnt, tiles);
  if (e == hipSuccess) e = dalloc(&d_off, tiles);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_allowed, allowed.data(), CGS_MAX_PARAMS * 4, hipMemcpyHostToDevice,
                       sp->stream);
  if (e == hipSuccess)
    e = launch_poly_design(sp->d_desc, sp->d_idx, nv, d_allowed, d_cnt, d_off, d_out, sp->stream);
  uint64_t last[2] = {0, 0};
  if (e == hipSuccess)
    e = hipMemcpyAsync(&last[0], d_off + tiles - 1, 8, hipMemcpyDeviceToHost, sp->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(&last[1], d_cnt + tiles - 1, 8, hipMemcpyDeviceToHost, sp->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(sp->stream);
  const uint64_t n = last[0] + last[1];
  if (e == hipSuccess && capacity && n)
    e = hipMemcpy(valid_idx, d_out, std::min<uint64_t>(n, capacity) * 4, hipMemcpyDeviceToHost);
  cleanup();
  if (e != hipSuccess) return fail(CGS_EDEVICE, "design: %s", hipGetErrorString(e));
  *count = n;
  if (capacity < n)
    return fail(CGS_ERANGE, "the design has %llu configurations, capacity %llu",
                (unsigned long long)n, (unsigned long long)capacity);
  return CGS_OK;
}

extern "C" cgs_status cgs_model_fit_poly(cgs_space sp, uint64_t n, int n_counters,
                                         const uint32_t *points, const float *targets, int order,
                                         cgs_model *out, cgs_poly_fit_report *report) {
  if (!out) return fail(CGS_EINVAL, "NULL out");
  *out = nullptr;
  if (!sp || !points || !targets) return fail(CGS_EINVAL, "NULL argument");
  if (n_counters < 1 || n_counters > CGS_MAX_COUNTERS)
    return fail(CGS_ERANGE, "n_counters %d outside 1..%d", n_counters, CGS_MAX_COUNTERS);
  if (order < 0 || order > kPolyMaxOrder)
    return fail(CGS_ERANGE, "order %d outside 0..%d", order, kPolyMaxOrder);
  if (n < 1 || n >= ((uint64_t)1 << 31)) return fail(CGS_ERANGE, "n = %llu", (unsigned long long)n);
  if (sp->n_valid == 0) return fail(CGS_EEMPTY, "the space has no valid configuration");
  PolyDev pd;
  cgs_status st = poly_describe(sp, order, n_counters, pd);
  if (st != CGS_OK) return st;
  const int T = pd.T, C = n_counters, S = pd.S, Ta = T + C;
  if ((uint64_t)n * Ta * 8 > ((uint64_t)16 << 30))
    return fail(CGS_ERANGE, "n * (terms + counters) too large for the feature matrix");
  if ((uint64_t)S * Ta * Ta * 8 > ((uint64_t)16 << 30))
    return fail(CGS_ERANGE, "%d subspaces of %d columns: Gram matrices too large", S, Ta);
  const int nbk = (Ta + 31) / 32;
  std::vector<uint32_t> pairs;
  for (int a = 0; a < nbk; ++a)
    for (int b = a; b < nbk; ++b) pairs.push_back((uint32_t)a | ((uint32_t)b << 16));

  cgs_model m = new (std::nothrow) cgs_model_s();
  if (!m) return fail(CGS_ENOMEM, "host allocation");
  m->space = sp;
  ++sp->refs;
  m->kind = 2;
  m->n_counters = C;
  m->poly = pd;
  m->stride = (sp->n_valid + 63) & ~(uint64_t)63;
  // each subspace's points in input order (a stable counting sort on the
  // host: digits of the points' raw indices, parameter 0 most significant)
  std::vector<uint32_t> h_off((size_t)S + 1, 0), h_list, h_sub(n);
  {
    const int P = (int)sp->radix.size();
    std::vector<uint32_t> dg(P);
    for (uint64_t i = 0; i < n; ++i) {
      h_sub[i] = (uint32_t)S; // points outside the valid list: in no list (the fit flags them)
      if (points[i] >= sp->n_valid) continue;
      uint64_t raw = sp->h_idx[points[i]];
      for (int j = P - 1; j >= 0; --j) {
        dg[j] = (uint32_t)(raw % (uint64_t)sp->radix[j]);
        raw /= (uint64_t)sp->radix[j];
      }
      uint32_t s = 0;
      for (int b = 0; b < pd.B; ++b) s |= dg[pd.bin_params[b]] << b;
      h_sub[i] = s;
      ++h_off[(size_t)s + 1];
    }
    for (int s = 0; s < S; ++s) h_off[(size_t)s + 1] += h_off[s];
    h_list.resize(h_off[S]);
    std::vector<uint32_t> pos(h_off.begin(), h_off.end() - 1);
    for (uint64_t i = 0; i < n; ++i)
      if (h_sub[i] < (uint32_t)S) h_list[pos[h_sub[i]]++] = (uint32_t)i;
  }
  uint32_t *d_pts = nullptr, *d_sub = nullptr, *d_pairs = nullptr, *d_err = nullptr;
  uint32_t *d_list = nullptr, *d_off = nullptr;
  float *d_y = nullptr;
  double *d_F = nullptr, *d_G = nullptr, *d_Gp = nullptr;
  // the Gram sums of each subspace split into parts when there are few
  // subspaces (a partial buffer, only when it stays modest)
  uint32_t parts = poly_gram_parts(S, (uint32_t)pairs.size());
  if ((uint64_t)parts * S * Ta * Ta * 8 > ((uint64_t)1 << 30)) parts = 1;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(sp->stream);
    dfree(d_pts);
    dfree(d_list);
    dfree(d_off);
    dfree(d_sub);
    dfree(d_pairs);
    dfree(d_err);
    dfree(d_y);
    dfree(d_F);
    dfree(d_G);
    dfree(d_Gp);
  };
  hipError_t e = dalloc(&m->d_poly, 1);
  if (e == hipSuccess) e = dalloc(&m->d_beta64, (size_t)S * T * C);
  if (e == hipSuccess) e = dalloc(&m->d_beta32, (size_t)S * T * C);
  if (e == hipSuccess) e = dalloc(&m->d_P, (size_t)C * m->stride);
  if (e == hipSuccess) e = dalloc(&d_pts, n);
  if (e == hipSuccess) e = dalloc(&d_y, n * (size_t)C);
  if (e == hipSuccess) e = dalloc(&d_sub, n);
  if (e == hipSuccess) e = dalloc(&d_list, std::max<size_t>(1, h_list.size()));
  if (e == hipSuccess) e = dalloc(&d_off, h_off.size());
  if (e == hipSuccess && !h_list.empty())
    e = hipMemcpyAsync(d_list, h_list.data(), h_list.size() * 4, hipMemcpyHostToDevice,
                       sp->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_off, h_off.data(), h_off.size() * 4, hipMemcpyHostToDevice, sp->stream);
  if (e == hipSuccess) e = dalloc(&d_F, n * (size_t)Ta);
  if (e == hipSuccess) e = dalloc(&d_G, (size_t)S * Ta * Ta);
  if (e == hipSuccess && parts > 1) e = dalloc(&d_Gp, (size_t)parts * S * Ta * Ta);
  if (e == hipSuccess) e = dalloc(&d_pairs, pairs.size());
  if (e == hipSuccess) e = dalloc(&d_err, 1);
  if (e == hipSuccess)
    e = hipMemcpyAsync(m->d_poly, &pd, sizeof(pd), hipMemcpyHostToDevice, sp->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_pts, points, n * 4, hipMemcpyHostToDevice, sp->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_y, targets, n * (size_t)C * 4, hipMemcpyHostToDevice, sp->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_pairs, pairs.data(), pairs.size() * 4, hipMemcpyHostToDevice,
                       sp->stream);
  if (e == hipSuccess) e = hipMemsetAsync(d_err, 0, 4, sp->stream);
  if (e == hipSuccess)
    e = hipMemsetAsync(m->d_P, 0, (size_t)C * m->stride * sizeof(float), sp->stream);
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (e == hipSuccess) e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  if (e == hipSuccess) e = hipEventRecord(ev[0], sp->stream);
  if (e == hipSuccess)
    e = launch_poly_fit(m->d_poly, T, C, S, sp->d_desc, sp->d_idx, (uint32_t)sp->n_valid, d_pts,
                        d_y, (uint32_t)n, d_F, d_sub, d_list, d_off, d_pairs,
                        (uint32_t)pairs.size(), d_G, d_Gp,
                        m->d_beta64, m->d_beta32, d_err, sp->stream);
  if (e == hipSuccess) e = hipEventRecord(ev[1], sp->stream);
  uint32_t err = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&err, d_err, 4, hipMemcpyDeviceToHost, sp->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(sp->stream);
  float fit_ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&fit_ms, ev[0], ev[1]);
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  cleanup();
  if (e != hipSuccess) {
    destroy_model(m);
    return fail(e == hipErrorOutOfMemory ? CGS_ENOMEM : CGS_EDEVICE, "polynomial fit: %s",
                hipGetErrorString(e));
  }
  if (err & 3u) {
    destroy_model(m);
    return fail(CGS_EINVAL, "%s",
                (err & 1u) ? "a point is outside the valid list" : "a target is not finite");
  }
  st = evaluate_model(m);
  if (st != CGS_OK) {
    destroy_model(m);
    return st;
  }
  if (report) {
    std::memset(report, 0, sizeof(*report));
    report->n_subspaces = S;
    report->n_terms = T;
    report->order = order;
    report->n_counters = C;
    report->n_points = n;
    report->fit_ms = fit_ms;
    report->eval_ms = m->eval_ms;
    report->pivot_clamped = (err & 4u) ? 1 : 0;
  }
  *out = m;
  return CGS_OK;
}

extern "C" cgs_status cgs_poly_shape(cgs_model m, int *n_subspaces, int *n_terms) {
  if (!m) return fail(CGS_EINVAL, "NULL model");
  if (m->kind != 2) return fail(CGS_EINVAL, "not a polynomial model");
  if (n_subspaces) *n_subspaces = m->poly.S;
  if (n_terms) *n_terms = m->poly.T;
  return CGS_OK;
}

extern "C" cgs_status cgs_poly_copy_coefficients(cgs_model m, double *beta) {
  if (!m || !beta) return fail(CGS_EINVAL, "NULL argument");
  if (m->kind != 2) return fail(CGS_EINVAL, "not a polynomial model");
  const size_t n = (size_t)m->poly.S * m->poly.T * m->poly.C;
  HIP_TRY(hipMemcpyAsync(beta, m->d_beta64, n * 8, hipMemcpyDeviceToHost, m->space->stream));
  HIP_TRY(hipStreamSynchronize(m->space->stream));
  return CGS_OK;
}

// ------------------------------------------------- prediction tables, Alg. 1
extern "C" cgs_status cgs_model_load_predictions(cgs_space sp, int n_counters,
                                                 const float *pred_host, cgs_model *out) {
  if (!out) return fail(CGS_EINVAL, "NULL out");
  *out = nullptr;
  if (!sp || !pred_host) return fail(CGS_EINVAL, "NULL argument");
  if (n_counters < 1 || n_counters > CGS_MAX_COUNTERS)
    return fail(CGS_ERANGE, "n_counters %d outside 1..%d", n_counters, CGS_MAX_COUNTERS);
  const uint64_t nv = sp->n_valid;
  if (nv == 0) return fail(CGS_EEMPTY, "the space has no valid configuration");
  for (uint64_t i = 0; i < nv * (uint64_t)n_counters; ++i)
    if (!(pred_host[i] >= 0.0f) || !std::isfinite(pred_host[i]))
      return fail(CGS_EINVAL, "prediction %llu is negative or not finite", (unsigned long long)i);
  cgs_model m = new (std::nothrow) cgs_model_s();
  if (!m) return fail(CGS_ENOMEM, "host allocation");
  m->space = sp;
  ++sp->refs;
  m->kind = 3;
  m->n_counters = n_counters;
  m->stride = (nv + 63) & ~(uint64_t)63;
  float *d_src = nullptr;
  hipError_t e = dalloc(&m->d_P, (size_t)n_counters * m->stride);
  if (e == hipSuccess) e = dalloc(&d_src, nv * (size_t)n_counters);
  if (e == hipSuccess)
    e = hipMemsetAsync(m->d_P, 0, (size_t)n_counters * m->stride * sizeof(float), sp->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_src, pred_host, nv * (size_t)n_counters * sizeof(float),
                       hipMemcpyHostToDevice, sp->stream);
  if (e == hipSuccess)
    e = launch_rows_to_columns(d_src, (uint32_t)nv, n_counters, m->d_P, m->stride, sp->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(sp->stream);
  dfree(d_src);
  if (e != hipSuccess) {
    destroy_model(m);
    return fail(e == hipErrorOutOfMemory ? CGS_ENOMEM : CGS_EDEVICE, "prediction table: %s",
                hipGetErrorString(e));
  }
  *out = m;
  return CGS_OK;
}

extern "C" void cgs_default_tuning_opts(cgs_tuning_opts *out) {
  if (!out) return;
  out->draws = 5;
  out->stop_at_well = 1;
  out->max_tests = UINT64_MAX;
  out->well_factor = 1.1;
}

namespace {

hipError_t launch_pending(cgs_session s, bool do_draw, uint64_t u64);
cgs_status wait_draw(cgs_session s, const DrawResult *res, uint64_t seq);

// The next n draws of a full step (1 <= n <= kMaxDrawSeries + 1) with
// uniforms u64[0..n): the first as cgs_sample_next makes it (launching a
// recorded step), the others in one draw_many launch, all enqueued before
// the host waits; each removes its pick before the next, so the picks are
// those of n cgs_sample_next calls.  valid[0..*made) receives the picks;
// *made < n when a draw found nothing to draw (Q == 0; the later ones find
// nothing either).
cgs_status draw_series(cgs_session s, int n, const uint64_t *u64, uint64_t *valid, int *made) {
  cgs_space sp = s->space;
  *made = 0;
  if (s->pending) {
    HIP_TRY(launch_pending(s, true, u64[0]));
  } else {
    HIP_TRY(launch_draw(s->d_s, s->d_explored, (uint32_t)sp->n_valid, kNoProfile, false,
                        s->d_acc + s->cur_acc * kAccSlots, s->params.gamma, s->params.w_min,
                        s->block_log2, s->d_bsum, s->n_blocks, u64[0], sp->d_idx, s->d_res,
                        ++s->seq, sp->stream));
  }
  const uint64_t seq_first = s->seq;
  if (n > 1) {
    DrawSeries ser{};
    ser.n = n - 1;
    for (int i = 1; i < n; ++i) ser.u64[i - 1] = u64[i];
    HIP_TRY(launch_draw_many(s->d_s, s->d_explored, (uint32_t)sp->n_valid,
                             s->d_acc + s->cur_acc * kAccSlots, s->params.gamma, s->params.w_min,
                             s->block_log2, s->d_bsum, s->n_blocks, ser, sp->d_idx, s->d_ring,
                             seq_first + 1, sp->stream));
    s->seq += (uint64_t)(n - 1);
  }
  for (int i = 0; i < n; ++i) {
    const DrawResult *slot = i == 0 ? s->h_res : s->h_ring + (i - 1);
    const cgs_status ws = wait_draw(s, slot, seq_first + (uint64_t)i);
    if (ws != CGS_OK) return ws;
    DrawResult r;
    std::memcpy(&r, const_cast<const DrawResult *>(static_cast<volatile const DrawResult *>(slot)),
                sizeof r);
    s->last_total = r.total;
    if (r.total == 0) return CGS_OK;
    if (r.valid == kNoPick)
      return fail(CGS_EDEVICE, "draw found no configuration although Q = %llu",
                  (unsigned long long)r.total);
    valid[i] = r.valid;
    *made = i + 1;
  }
  return CGS_OK;
}

} // namespace

extern "C" cgs_status cgs_tuning_run(cgs_session s, cgs_model m, const float *runtime,
                                     const double *counters, const cgs_expert_params *expert,
                                     const uint64_t *uniforms, uint64_t n_uniforms,
                                     const cgs_tuning_opts *opts, uint64_t capacity,
                                     uint64_t *tested, uint8_t *profiled, uint64_t *n_tests,
                                     uint64_t *tests_to_well) {
  if (!s || !m || !runtime || !counters || !uniforms || !opts || !n_tests || !tests_to_well ||
      (capacity && !tested))
    return fail(CGS_EINVAL, "NULL argument");
  *n_tests = 0;
  *tests_to_well = 0;
  cgs_space sp = s->space;
  if (m->space != sp) return fail(CGS_EINVAL, "model and session belong to different spaces");
  if (m->n_counters != 24) return fail(CGS_EINVAL, "the loop needs a model of the 24 counters");
  if (opts->draws < 1) return fail(CGS_ERANGE, "draws %d < 1", opts->draws);
  if (opts->max_tests < 1 || opts->max_tests > capacity)
    return fail(CGS_ERANGE, "max_tests must be 1..capacity");
  const uint64_t nv = sp->n_valid;
  if (nv == 0) return fail(CGS_EEMPTY, "the space has no valid configuration");
  float rmin = runtime[0];
  for (uint64_t l = 1; l < nv; ++l) rmin = std::min(rmin, runtime[l]);
  const double thresh = opts->well_factor * (double)rmin;
  uint64_t u = 0, nt = 0, found = 0;
  auto test = [&](uint64_t l, bool prof) {
    tested[nt] = l;
    if (profiled) profiled[nt] = prof ? 1 : 0;
    ++nt;
    if (!found && (double)runtime[l] <= thresh) found = nt;
    return (opts->stop_at_well && found) || nt >= opts->max_tests;
  };
  auto draw = [&](uint64_t *l) -> cgs_status {
    if (u >= n_uniforms) return fail(CGS_ERANGE, "the run needs more than %llu random numbers",
                                     (unsigned long long)n_uniforms);
    uint64_t raw = 0;
    return cgs_sample_next(s, uniforms[u++], &raw, l);
  };
  cgs_status st = cgs_search_step(s, m, CGS_NO_PROFILE, nullptr, nullptr, expert);
  uint64_t c = 0;
  if (st == CGS_OK) st = draw(&c);
  bool have = st == CGS_OK;
  if (st == CGS_EEMPTY) st = CGS_OK;
  while (st == CGS_OK && have) {
    if (test(c, true)) break;
    st = cgs_search_step(s, m, sp->h_idx[c], nullptr, counters + c * 24, expert);
    if (st != CGS_OK) break;
    float best = INFINITY;
    bool next = false, stop = false;
    auto consider = [&](uint64_t l) {
      if (test(l, false)) return stop = true;
      if (runtime[l] <= best) {
        best = runtime[l];
        c = l;
        next = true;
      }
      return false;
    };
    if (opts->draws <= kMaxDrawSeries + 1 && !s->pending_nb && (s->pending || !s->last_nb)) {
      // the step's draws in one go: they depend on its weights and the
      // uniforms only, the tests decide where the run stops
      const int want = (int)std::min<uint64_t>((uint64_t)opts->draws, n_uniforms - u);
      uint64_t picks[kMaxDrawSeries + 1];
      int made = 0;
      if (want > 0) st = draw_series(s, want, uniforms + u, picks, &made);
      u += (uint64_t)std::max(want, 0);
      if (st != CGS_OK) break;
      for (int k = 0; k < made && !stop; ++k) consider(picks[k]);
      if (!stop && made == want && want < opts->draws) {
        st = fail(CGS_ERANGE, "the run needs more than %llu random numbers",
                  (unsigned long long)n_uniforms);
        break;
      }
    } else {
      for (int k = 0; k < opts->draws; ++k) {
        uint64_t l = 0;
        st = draw(&l);
        if (st == CGS_EEMPTY) {
          st = CGS_OK;
          break;
        }
        if (st != CGS_OK) break;
        if (consider(l)) break;
      }
      if (st != CGS_OK) break;
    }
    if (stop || !next) break;
  }
  *n_tests = nt;
  *tests_to_well = found;
  return st;
}

extern "C" cgs_status cgs_model_forest_shape(cgs_model m, int *n_trees, int *depth) {
  if (!m) return fail(CGS_EINVAL, "NULL model");
  if (m->kind != 0) return fail(CGS_EINVAL, "not a forest model");
  if (n_trees) *n_trees = m->n_trees;
  if (depth) *depth = m->depth;
  return CGS_OK;
}

extern "C" cgs_status cgs_model_copy_forest(cgs_model m, uint8_t *feat, uint8_t *thr,
                                            float *leaves) {
  if (!m) return fail(CGS_EINVAL, "NULL model");
  if (m->kind != 0) return fail(CGS_EINVAL, "not a forest model");
  const size_t n_int = (size_t)m->n_trees * (((size_t)1 << m->depth) - 1);
  const size_t n_leaf_vals = (size_t)m->n_trees * ((size_t)1 << m->depth) * m->n_counters;
  if ((n_int && (!feat || !thr)) || !leaves) return fail(CGS_EINVAL, "NULL argument");
  std::vector<uint16_t> nodes(n_int);
  cgs_space sp = m->space;
  if (n_int)
    HIP_TRY(hipMemcpyAsync(nodes.data(), m->d_nodes, n_int * sizeof(uint16_t),
                           hipMemcpyDeviceToHost, sp->stream));
  HIP_TRY(hipMemcpyAsync(leaves, m->d_leaves, n_leaf_vals * sizeof(float), hipMemcpyDeviceToHost,
                         sp->stream));
  HIP_TRY(hipStreamSynchronize(sp->stream));
  for (size_t i = 0; i < n_int; ++i) {
    feat[i] = (uint8_t)(nodes[i] & 0xffu);
    thr[i] = (uint8_t)(nodes[i] >> 8);
  }
  return CGS_OK;
}

extern "C" cgs_status cgs_model_info(cgs_model m, int *n_counters, float *eval_ms) {
  if (!m) return fail(CGS_EINVAL, "NULL model");
  if (n_counters) *n_counters = m->n_counters;
  if (eval_ms) *eval_ms = m->eval_ms;
  return CGS_OK;
}

extern "C" cgs_status cgs_model_refresh(cgs_model m) {
  if (!m) return fail(CGS_EINVAL, "NULL model");
  return evaluate_model(m);
}

extern "C" cgs_status cgs_model_copy_predictions(cgs_model m, uint64_t first, uint64_t count,
                                                 float *dst) {
  if (!m || (!dst && count)) return fail(CGS_EINVAL, "NULL argument");
  cgs_space sp = m->space;
  if (first > sp->n_valid || count > sp->n_valid - first)
    return fail(CGS_ERANGE, "range outside the valid list");
  if (count == 0) return CGS_OK;
  std::vector<float> rows((size_t)m->n_counters * count);
  for (int c = 0; c < m->n_counters; ++c)
    HIP_TRY(hipMemcpyAsync(rows.data() + (size_t)c * count, m->d_P + (size_t)c * m->stride + first,
                           count * sizeof(float), hipMemcpyDeviceToHost, sp->stream));
  HIP_TRY(hipStreamSynchronize(sp->stream));
  for (uint64_t i = 0; i < count; ++i)
    for (int c = 0; c < m->n_counters; ++c)
      dst[i * m->n_counters + c] = rows[(size_t)c * count + i];
  return CGS_OK;
}

extern "C" cgs_status cgs_model_gather_predictions(cgs_model m, const uint32_t *idx, uint64_t n,
                                                   float *dst) {
  if (!m || ((!idx || !dst) && n)) return fail(CGS_EINVAL, "NULL argument");
  if (n > 0xffffffffull / (uint64_t)CGS_MAX_COUNTERS)
    return fail(CGS_ERANGE, "too many configurations in one gather");
  if (n == 0) return CGS_OK;
  cgs_space sp = m->space;
  for (uint64_t i = 0; i < n; ++i)
    if (idx[i] >= sp->n_valid)
      return fail(CGS_EINVAL, "index %llu = %u is outside the valid list", (unsigned long long)i,
                  idx[i]);
  uint32_t *d_idx = nullptr;
  float *d_out = nullptr;
  hipError_t e = dalloc(&d_idx, n);
  if (e == hipSuccess) e = dalloc(&d_out, n * (uint64_t)m->n_counters);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_idx, idx, n * sizeof(uint32_t), hipMemcpyHostToDevice, sp->stream);
  if (e == hipSuccess)
    e = launch_gather_rows(m->d_P, m->stride, m->n_counters, d_idx, (uint32_t)n, d_out,
                           sp->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst, d_out, n * (uint64_t)m->n_counters * sizeof(float),
                       hipMemcpyDeviceToHost, sp->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(sp->stream);
  dfree(d_idx);
  dfree(d_out);
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? CGS_ENOMEM : CGS_EDEVICE, "gather: %s",
                hipGetErrorString(e));
  return CGS_OK;
}

extern "C" cgs_status cgs_model_rmse(cgs_model a, cgs_model b, const uint32_t *sample,
                                     uint64_t n, double *rmse) {
  if (!a || !b || !rmse || (!sample && n)) return fail(CGS_EINVAL, "NULL argument");
  if (a->space != b->space) return fail(CGS_EINVAL, "models predict different spaces");
  if (a->n_counters != b->n_counters) return fail(CGS_EINVAL, "models differ in counters");
  if (n == 0 || n > 0xffffffffull) return fail(CGS_ERANGE, "need 1 .. 2^32-1 samples");
  cgs_space sp = a->space;
  for (uint64_t i = 0; i < n; ++i)
    if (sample[i] >= sp->n_valid) return fail(CGS_EINVAL, "sample %llu outside the valid list",
                                              (unsigned long long)i);
  const uint32_t grid = (uint32_t)std::min<uint64_t>((n + 255) / 256, 1024);
  uint32_t *d_s = nullptr;
  double *d_part = nullptr;
  std::vector<double> part(grid);
  hipError_t e = dalloc(&d_s, n);
  if (e == hipSuccess) e = dalloc(&d_part, grid);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_s, sample, n * sizeof(uint32_t), hipMemcpyHostToDevice, sp->stream);
  if (e == hipSuccess)
    e = launch_sq_diff(a->d_P, b->d_P, a->stride, b->stride, a->n_counters, d_s, (uint32_t)n,
                       d_part, grid, sp->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(part.data(), d_part, grid * sizeof(double), hipMemcpyDeviceToHost,
                       sp->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(sp->stream);
  dfree(d_s);
  dfree(d_part);
  if (e != hipSuccess) return fail(CGS_EDEVICE, "rmse: %s", hipGetErrorString(e));
  double sum = 0.0;
  for (double v : part) sum += v;
  *rmse = std::sqrt(sum / ((double)n * a->n_counters));
  return CGS_OK;
}

extern "C" cgs_status cgs_model_copy_leaf_ids(cgs_model m, uint64_t first, uint64_t count,
                                              uint16_t *dst) {
  if (!m || (!dst && count)) return fail(CGS_EINVAL, "NULL argument");
  if (m->kind != 0) return fail(CGS_EINVAL, "not a forest model");
  cgs_space sp = m->space;
  if (first > sp->n_valid || count > sp->n_valid - first)
    return fail(CGS_ERANGE, "range outside the valid list");
  if (count == 0) return CGS_OK;
  uint16_t *d_out = nullptr;
  HIP_TRY(dalloc(&d_out, (size_t)m->n_trees * count));
  hipError_t e = launch_forest_eval(sp->d_desc, sp->d_idx, (uint32_t)sp->n_valid, m->d_nodes,
                                    m->d_leaves, m->n_trees, m->depth, m->n_counters, m->d_P,
                                    m->stride, d_out, (uint32_t)first, (uint32_t)count, sp->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst, d_out, (size_t)m->n_trees * count * sizeof(uint16_t),
                       hipMemcpyDeviceToHost, sp->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(sp->stream);
  dfree(d_out);
  if (e != hipSuccess) return fail(CGS_EDEVICE, "leaf ids: %s", hipGetErrorString(e));
  return CGS_OK;
}

// ------------------------------------------------------------ perceptron
namespace {

bool mlp_desc_ok(const cgs_mlp_desc *d) {
  return d && d->n_in >= 1 && d->n_in <= 32 &&
         (d->hidden == 64 || d->hidden == 128 || d->hidden == 256 || d->hidden == 512) &&
         d->n_out >= 1 && d->n_out <= CGS_MAX_COUNTERS;
}

uint64_t mlp_count(int F, int H, int C) {
  return (uint64_t)H * F + H + (uint64_t)H * H + H + (uint64_t)C * H + C;
}

hipError_t ensure_mlp_scratch(cgs_model m, uint32_t rows) {
  if (m->scratch_rows >= rows) return hipSuccess;
  free_mlp_scratch(m);
  const size_t H = m->sh.H, Cp = (size_t)32 * ((m->sh.C + 31) / 32);
  const size_t n_pad = ((size_t)rows + 31) / 32 * 32, nblk = n_pad / 16; // 16-row blocks
  hipError_t e = dalloc(&m->d_xt, 32 * n_pad);
  if (e == hipSuccess) e = dalloc(&m->d_h1t, H * n_pad);
  if (e == hipSuccess) e = dalloc(&m->d_h2t, H * n_pad);
  if (e == hipSuccess) e = dalloc(&m->d_dyt, Cp * n_pad);
  if (e == hipSuccess) e = dalloc(&m->d_dz2t, H * n_pad);
  if (e == hipSuccess) e = dalloc(&m->d_dz1t, H * n_pad);
  if (e == hipSuccess) e = dalloc(&m->d_bp1, nblk * H);
  if (e == hipSuccess) e = dalloc(&m->d_bp2, nblk * H);
  if (e == hipSuccess) e = dalloc(&m->d_bp3, nblk * Cp);
  if (e == hipSuccess) e = dalloc(&m->d_lossp, nblk);
  if (e == hipSuccess) e = dalloc(&m->d_y, n_pad * Cp);
  if (e == hipSuccess) e = dalloc(&m->d_xg, kGatherSteps * n_pad * m->sh.K1);
  if (e == hipSuccess) e = dalloc(&m->d_tg, kGatherSteps * (size_t)rows * m->sh.C);
  if (e != hipSuccess) {
    free_mlp_scratch(m);
    return e;
  }
  m->scratch_rows = rows;
  return hipSuccess;
}

// Gathers the rows of `steps` steps of n rows (pair d_batch[s n + r], or r
// without a batch) into m->d_xg / m->d_tg (targets when d_targets is set).
hipError_t gather_rows(cgs_model m, const uint32_t *d_cfg, const float *d_targets,
                       const int32_t *d_batch, uint32_t steps, uint32_t n) {
  return launch_mlp_gather_rows(m->space->d_desc, d_cfg, d_batch, d_targets, steps, n,
                                (n + 31) / 32 * 32, m->sh.F, m->sh.K1, m->sh.C, m->d_xg,
                                m->d_tg, m->space->stream);
}

// Launch arguments of the row kernel for step k of the gathered run (n
// rows); train == false: forward only, Y into m->d_y.
TrainRowsArgs train_rows_args(cgs_model m, uint32_t k, uint32_t n, bool train) {
  TrainRowsArgs a{};
  const uint32_t n_pad = (n + 31) / 32 * 32;
  a.xin = m->d_xg + (size_t)k * n_pad * m->sh.K1;
  a.tin = train ? m->d_tg + (size_t)k * n * m->sh.C : nullptr;
  a.train = train;
  a.n = n;
  a.n_pad = (n + 31) / 32 * 32;
  a.H = m->sh.H;
  a.C = m->sh.C;
  a.K1 = m->sh.K1;
  a.scale = 2.0f / (float)(n * (uint32_t)m->sh.C);
  a.w1n = m->d_w1n;
  a.w2n = m->d_w2n;
  a.w3n = m->d_w3n;
  a.w2t = m->d_w2t;
  a.w3t = m->d_w3t;
  a.b1 = m->d_theta + m->off_b1;
  a.b2 = m->d_theta + m->off_b2;
  a.b3 = m->d_theta + m->off_b3;
  a.yout = m->d_y;
  a.xt = m->d_xt;
  a.h1t = m->d_h1t;
  a.h2t = m->d_h2t;
  a.dyt = m->d_dyt;
  a.dz2t = m->d_dz2t;
  a.dz1t = m->d_dz1t;
  a.bp1 = m->d_bp1;
  a.bp2 = m->d_bp2;
  a.bp3 = m->d_bp3;
  a.lossp = m->d_lossp;
  return a;
}

// Forward of n rows, Y into m->d_y ([n][Cp]).
hipError_t mlp_forward_rows(cgs_model m, const uint32_t *d_cfg, uint32_t n) {
  hipError_t e = gather_rows(m, d_cfg, nullptr, nullptr, 1, n);
  if (e != hipSuccess) return e;
  return launch_mlp_train_rows(train_rows_args(m, 0, n, false), m->space->stream);
}

// Adam settings of one step (c1, c2: this step's bias corrections).
struct AdamStep {
  float lr, beta1, beta2, eps, c1, c2;
};

// Forward, loss and backward of step k of the gathered run, n rows (two
// launches): with adam == nullptr the gradient goes to m->d_grad, otherwise
// the step is applied to the parameters; the loss goes to *d_loss.
hipError_t mlp_step_rows(cgs_model m, uint32_t k, uint32_t n, float *d_loss,
                         const AdamStep *adam) {
  hipStream_t st = m->space->stream;
  const TrainRowsArgs a = train_rows_args(m, k, n, true);
  hipError_t e = launch_mlp_train_rows(a, st);
  if (e != hipSuccess) return e;
  GradTilesArgs g{};
  g.sh = m->sh;
  g.n_pad = a.n_pad;
  g.xt = a.xt;
  g.h1t = a.h1t;
  g.h2t = a.h2t;
  g.dyt = a.dyt;
  g.dz2t = a.dz2t;
  g.dz1t = a.dz1t;
  g.bp1 = a.bp1;
  g.bp2 = a.bp2;
  g.bp3 = a.bp3;
  g.lossp = a.lossp;
  g.loss_out = d_loss;
  g.loss_div = (float)(n * (uint32_t)m->sh.C);
  g.theta = m->d_theta;
  g.m = m->d_m;
  g.v = m->d_v;
  g.cp = mlp_copies(m);
  if (adam) {
    g.lr = adam->lr;
    g.beta1 = adam->beta1;
    g.beta2 = adam->beta2;
    g.eps = adam->eps;
    g.c1 = adam->c1;
    g.c2 = adam->c2;
  } else {
    g.grad = m->d_grad;
  }
  return launch_mlp_grad_tiles(g, st);
}

// Uploads host pairs; returns device copies (caller frees).
hipError_t upload_pairs(cgs_model m, const uint32_t *cfg, const float *targets, uint64_t n,
                        uint32_t **d_cfg, float **d_t) {
  hipStream_t st = m->space->stream;
  hipError_t e = dalloc(d_cfg, n);
  if (e == hipSuccess && targets) e = dalloc(d_t, n * (size_t)m->sh.C);
  if (e == hipSuccess)
    e = hipMemcpyAsync(*d_cfg, cfg, n * sizeof(uint32_t), hipMemcpyHostToDevice, st);
  if (e == hipSuccess && targets)
    e = hipMemcpyAsync(*d_t, targets, n * (size_t)m->sh.C * sizeof(float), hipMemcpyHostToDevice,
                       st);
  return e;
}

cgs_status check_pairs(cgs_model m, const uint32_t *cfg, const float *targets, uint64_t n) {
  for (uint64_t i = 0; i < n; ++i)
    if (cfg[i] >= m->space->n_raw)
      return fail(CGS_EINVAL, "pair %llu: raw index %u >= n_raw", (unsigned long long)i, cfg[i]);
  if (targets)
    for (uint64_t i = 0; i < n * (uint64_t)m->sh.C; ++i)
      if (!std::isfinite(targets[i])) return fail(CGS_EINVAL, "target %llu not finite",
                                                  (unsigned long long)i);
  return CGS_OK;
}

} // namespace

extern "C" uint64_t cgs_mlp_param_count(const cgs_mlp_desc *d) {
  return mlp_desc_ok(d) ? mlp_count(d->n_in, d->hidden, d->n_out) : 0;
}

extern "C" cgs_status cgs_model_load_mlp(cgs_space sp, const cgs_mlp_desc *desc,
                                         const float *params, cgs_model *out) {
  if (!out) return fail(CGS_EINVAL, "NULL out");
  *out = nullptr;
  if (!sp || !params) return fail(CGS_EINVAL, "NULL argument");
  if (!mlp_desc_ok(desc))
    return fail(CGS_ERANGE, "perceptron shape: n_in 1..32, hidden 64/128/256/512, n_out 1..64");
  if (desc->n_in != sp->n_params)
    return fail(CGS_EINVAL, "n_in %d must equal the space's %d parameters", desc->n_in,
                sp->n_params);
  const uint64_t n = mlp_count(desc->n_in, desc->hidden, desc->n_out);
  for (uint64_t i = 0; i < n; ++i)
    if (!std::isfinite(params[i])) return fail(CGS_EINVAL, "parameter %llu not finite",
                                               (unsigned long long)i);
  cgs_model m = new (std::nothrow) cgs_model_s();
  if (!m) return fail(CGS_ENOMEM, "host allocation");
  m->space = sp;
  ++sp->refs;
  m->kind = 1;
  m->n_counters = desc->n_out;
  m->sh = MlpShape{desc->n_in, desc->hidden, desc->n_out, desc->n_in <= 16 ? 16 : 32};
  m->n_theta = n;
  const size_t H = desc->hidden, F = desc->n_in, C = desc->n_out;
  m->off_b1 = H * F;
  m->off_w2 = m->off_b1 + H;
  m->off_b2 = m->off_w2 + H * H;
  m->off_w3 = m->off_b2 + H;
  m->off_b3 = m->off_w3 + C * H;
  m->n_w1p = H * m->sh.K1;
  m->n_w2p = H * H;
  m->n_w3p = (size_t)32 * ((C + 31) / 32) * H;
  m->stride = (sp->n_valid + 63) & ~(uint64_t)63;
  hipDeviceProp_t prop;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    m->n_cu = prop.multiProcessorCount;
  hipStream_t st = sp->stream;
  hipError_t e = dalloc(&m->d_theta, n);
  if (e == hipSuccess) e = dalloc(&m->d_m, n);
  if (e == hipSuccess) e = dalloc(&m->d_v, n);
  if (e == hipSuccess) e = dalloc(&m->d_grad, n);
  if (e == hipSuccess) e = dalloc(&m->d_w1p, m->n_w1p);
  if (e == hipSuccess) e = dalloc(&m->d_w2p, m->n_w2p);
  if (e == hipSuccess) e = dalloc(&m->d_w3p, m->n_w3p);
  if (e == hipSuccess) e = dalloc(&m->d_w2t, m->n_w2p);
  if (e == hipSuccess) e = dalloc(&m->d_w3t, m->n_w3p);
  if (e == hipSuccess) e = dalloc(&m->d_w1n, H * 32);
  if (e == hipSuccess) e = dalloc(&m->d_w2n, m->n_w2p);
  if (e == hipSuccess) e = dalloc(&m->d_w3n, m->n_w3p);
  if (e == hipSuccess) e = dalloc(&m->d_P, (size_t)C * m->stride);
  if (e == hipSuccess)
    e = hipMemcpyAsync(m->d_theta, params, n * sizeof(float), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(m->d_m, 0, n * sizeof(float), st);
  if (e == hipSuccess) e = hipMemsetAsync(m->d_v, 0, n * sizeof(float), st);
  if (e == hipSuccess) e = hipMemsetAsync(m->d_w1p, 0, m->n_w1p * sizeof(__bf16), st);
  if (e == hipSuccess) e = hipMemsetAsync(m->d_w3p, 0, m->n_w3p * sizeof(__bf16), st);
  // the padding of w3t (columns C .. Cp-1), w1n (features F .. 31) and w3n
  // (rows C .. Cp-1) is read by the training products
  if (e == hipSuccess) e = hipMemsetAsync(m->d_w3t, 0, m->n_w3p * sizeof(__bf16), st);
  if (e == hipSuccess) e = hipMemsetAsync(m->d_w1n, 0, H * 32 * sizeof(__bf16), st);
  if (e == hipSuccess) e = hipMemsetAsync(m->d_w3n, 0, m->n_w3p * sizeof(__bf16), st);
  if (e == hipSuccess) e = hipMemsetAsync(m->d_P, 0, (size_t)C * m->stride * sizeof(float), st);
  if (e == hipSuccess)
    e = launch_pack_weights(m->sh, m->d_theta, n, mlp_copies(m), st);
  if (e != hipSuccess) {
    destroy_model(m);
    return fail(e == hipErrorOutOfMemory ? CGS_ENOMEM : CGS_EDEVICE, "perceptron buffers: %s",
                hipGetErrorString(e));
  }
  const cgs_status stt = evaluate_model(m);
  if (stt != CGS_OK) {
    destroy_model(m);
    return stt;
  }
  *out = m;
  return CGS_OK;
}

// The Adam steps of cgs_mlp_train; with evaluate, the predictions of every
// valid configuration are refreshed after them, otherwise they are marked
// stale (cgs_online_run refreshes them when they are used).
cgs_status mlp_train_run(cgs_model m, const uint32_t *cfg, const float *targets, uint64_t n,
                         const int32_t *batch_idx, const cgs_train_opts *o, float *loss_host,
                         bool evaluate) {
  if (!m || !cfg || !targets || !batch_idx || !o) return fail(CGS_EINVAL, "NULL argument");
  if (m->kind != 1) return fail(CGS_EINVAL, "not a perceptron model");
  if (n == 0 || n > 0xffffffffull) return fail(CGS_ERANGE, "need 1 .. 2^32-1 pairs");
  if (o->batch < 1 || o->batch > 4096 || o->steps < 0)
    return fail(CGS_ERANGE, "batch must be 1..4096 and steps >= 0");
  if (!(o->lr > 0.0f) || !(o->beta1 >= 0.0f && o->beta1 < 1.0f) ||
      !(o->beta2 >= 0.0f && o->beta2 < 1.0f) || !(o->eps > 0.0f))
    return fail(CGS_EINVAL, "Adam settings out of range");
  cgs_status cs = check_pairs(m, cfg, targets, n);
  if (cs != CGS_OK) return cs;
  const size_t nb = (size_t)o->steps * o->batch;
  for (size_t i = 0; i < nb; ++i)
    if (batch_idx[i] < 0 || (uint64_t)batch_idx[i] >= n)
      return fail(CGS_EINVAL, "batch entry %zu = %d outside the pairs", i, batch_idx[i]);
  hipStream_t st = m->space->stream;
  uint32_t *d_cfg = nullptr;
  float *d_t = nullptr, *d_loss = nullptr;
  int32_t *d_batch = nullptr;
  hipError_t e = ensure_mlp_scratch(m, (uint32_t)o->batch);
  if (e == hipSuccess) e = upload_pairs(m, cfg, targets, n, &d_cfg, &d_t);
  if (e == hipSuccess) e = dalloc(&d_batch, std::max<size_t>(nb, 1));
  if (e == hipSuccess) e = dalloc(&d_loss, std::max<int>(o->steps, 1));
  if (e == hipSuccess && nb)
    e = hipMemcpyAsync(d_batch, batch_idx, nb * sizeof(int32_t), hipMemcpyHostToDevice, st);
  for (int s = 0; s < o->steps && e == hipSuccess; ++s) {
    const uint32_t k = (uint32_t)s % kGatherSteps;
    if (k == 0) // the rows of the next run of steps
      e = gather_rows(m, d_cfg, d_t, d_batch + (size_t)s * o->batch,
                      (uint32_t)std::min<int>(kGatherSteps, o->steps - s), (uint32_t)o->batch);
    if (e != hipSuccess) break;
    m->adam_t += 1;
    const double c1 = 1.0 / (1.0 - std::pow((double)o->beta1, (double)m->adam_t));
    const double c2 = 1.0 / (1.0 - std::pow((double)o->beta2, (double)m->adam_t));
    const AdamStep adam{o->lr, o->beta1, o->beta2, o->eps, (float)c1, (float)c2};
    e = mlp_step_rows(m, k, (uint32_t)o->batch, d_loss + s, &adam);
  }
  if (e == hipSuccess && loss_host && o->steps > 0)
    e = hipMemcpyAsync(loss_host, d_loss, o->steps * sizeof(float), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dfree(d_cfg);
  dfree(d_t);
  dfree(d_batch);
  dfree(d_loss);
  if (e != hipSuccess) return fail(CGS_EDEVICE, "training: %s", hipGetErrorString(e));
  if (!evaluate) {
    m->p_stale = true;
    return CGS_OK;
  }
  m->p_stale = false;
  return evaluate_model(m);
}

extern "C" cgs_status cgs_mlp_train(cgs_model m, const uint32_t *cfg, const float *targets,
                                    uint64_t n, const int32_t *batch_idx,
                                    const cgs_train_opts *o, float *loss_host) {
  return mlp_train_run(m, cfg, targets, n, batch_idx, o, loss_host, true);
}

extern "C" cgs_status cgs_mlp_gradients(cgs_model m, const uint32_t *cfg, const float *targets,
                                        uint32_t n, float *grads, float *loss_host) {
  if (!m || !cfg || !targets || !grads) return fail(CGS_EINVAL, "NULL argument");
  if (m->kind != 1) return fail(CGS_EINVAL, "not a perceptron model");
  if (n < 1 || n > 4096) return fail(CGS_ERANGE, "n must be 1..4096");
  cgs_status cs = check_pairs(m, cfg, targets, n);
  if (cs != CGS_OK) return cs;
  hipStream_t st = m->space->stream;
  uint32_t *d_cfg = nullptr;
  float *d_t = nullptr, *d_loss = nullptr;
  hipError_t e = ensure_mlp_scratch(m, n);
  if (e == hipSuccess) e = upload_pairs(m, cfg, targets, n, &d_cfg, &d_t);
  if (e == hipSuccess) e = dalloc(&d_loss, 1);
  if (e == hipSuccess) e = gather_rows(m, d_cfg, d_t, nullptr, 1, n);
  if (e == hipSuccess) e = mlp_step_rows(m, 0, n, d_loss, nullptr);
  float loss = 0.0f;
  if (e == hipSuccess)
    e = hipMemcpyAsync(grads, m->d_grad, m->n_theta * sizeof(float), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&loss, d_loss, sizeof(float), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dfree(d_cfg);
  dfree(d_t);
  dfree(d_loss);
  if (e != hipSuccess) return fail(CGS_EDEVICE, "gradients: %s", hipGetErrorString(e));
  if (loss_host) *loss_host = loss;
  return CGS_OK;
}

extern "C" cgs_status cgs_mlp_forward(cgs_model m, const uint32_t *cfg, uint32_t n, float *y) {
  if (!m || !cfg || !y) return fail(CGS_EINVAL, "NULL argument");
  if (m->kind != 1) return fail(CGS_EINVAL, "not a perceptron model");
  if (n < 1 || n > 4096) return fail(CGS_ERANGE, "n must be 1..4096");
  cgs_status cs = check_pairs(m, cfg, nullptr, n);
  if (cs != CGS_OK) return cs;
  hipStream_t st = m->space->stream;
  uint32_t *d_cfg = nullptr;
  float *d_unused = nullptr;
  const int Cp = 32 * ((m->sh.C + 31) / 32);
  std::vector<float> rows((size_t)n * Cp);
  hipError_t e = ensure_mlp_scratch(m, n);
  if (e == hipSuccess) e = upload_pairs(m, cfg, nullptr, n, &d_cfg, &d_unused);
  if (e == hipSuccess) e = mlp_forward_rows(m, d_cfg, n);
  if (e == hipSuccess)
    e = hipMemcpyAsync(rows.data(), m->d_y, rows.size() * sizeof(float), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  dfree(d_cfg);
  if (e != hipSuccess) return fail(CGS_EDEVICE, "forward: %s", hipGetErrorString(e));
  for (uint32_t i = 0; i < n; ++i)
    for (int c = 0; c < m->sh.C; ++c) y[(size_t)i * m->sh.C + c] = rows[(size_t)i * Cp + c];
  return CGS_OK;
}

extern "C" cgs_status cgs_mlp_copy_params(cgs_model m, float *dst, uint64_t n) {
  if (!m || !dst) return fail(CGS_EINVAL, "NULL argument");
  if (m->kind != 1) return fail(CGS_EINVAL, "not a perceptron model");
  if (n != m->n_theta) return fail(CGS_EINVAL, "model has %llu parameters",
                                   (unsigned long long)m->n_theta);
  HIP_TRY(hipMemcpyAsync(dst, m->d_theta, n * sizeof(float), hipMemcpyDeviceToHost,
                         m->space->stream));
  HIP_TRY(hipStreamSynchronize(m->space->stream));
  return CGS_OK;
}

extern "C" void cgs_model_destroy(cgs_model m) { destroy_model(m); }

// ------------------------------------------------------------------ session
namespace {

void destroy_session(cgs_session s) {
  if (!s) return;
  if (s->space && s->space->stream) (void)hipStreamSynchronize(s->space->stream);
  dfree(s->d_explored);
  dfree(s->d_s);
  dfree(s->d_bsum);
  dfree(s->d_acc);
  dfree(s->d_sub_off);
  dfree(s->d_sub_code);
  dfree(s->d_nb_tmp_idx);
  dfree(s->d_nb_idx);
  dfree(s->d_nb_q);
  dfree(s->d_nb_tmp_s);
  dfree(s->d_nb_s);
  dfree(s->d_nb_bsum);
  dfree(s->d_nb_stats);
  dfree(s->d_nb_acc);
  dfree(s->d_prof);
  if (s->h_res) (void)hipHostFree(s->h_res);
  if (s->h_acc) (void)hipHostFree(s->h_acc);
  if (s->h_ring) (void)hipHostFree(s->h_ring);
  for (hipEvent_t ev : s->t_ev)
    if (ev) (void)hipEventDestroy(ev);
  destroy_space(s->space);
  delete s;
}

int auto_block_log2(uint64_t n_valid) {
  // at most 65536 blocks, at least 4096 configurations per block
  int lg = kDefaultBlockLog2;
  while (lg < 20 && (n_valid >> lg) >= 65536) ++lg;
  return lg;
}

// Starts a timed span of `n` kernels: reserves n + 1 markers (summing and
// emptying the pool first when it is full) and records the first.
hipError_t begin_span(cgs_session s, int n, const int *kinds, TimedSpan **out);

// Sums the durations of every recorded span and empties the pool.
hipError_t collect_times(cgs_session s) {
  if (s->t_spans.empty()) return hipSuccess;
  hipError_t e = hipEventSynchronize(s->t_ev[s->t_ev_used - 1]);
  for (const TimedSpan &sp : s->t_spans) {
    for (int k = 0; k < sp.n && e == hipSuccess; ++k) {
      float ms = 0.0f;
      e = hipEventElapsedTime(&ms, s->t_ev[sp.ev + k], s->t_ev[sp.ev + k + 1]);
      // slots: 0 scored score pass, 1 weight pass, 2 draws, 3 restricted
      // scoring; kinds 3 (profile mark) and 5 (unscored score pass): none
      const int slot = sp.kind[k] <= 2 ? sp.kind[k] : sp.kind[k] == 4 ? 3 : -1;
      if (e == hipSuccess && slot >= 0) {
        s->kernel_ms[slot] += ms;
        s->kernel_n[slot] += 1;
      }
    }
  }
  if (e == hipSuccess && s->t_step >= 0) {
    const TimedSpan &st = s->t_spans[s->t_step];
    e = hipEventElapsedTime(&s->step_ms, s->t_ev[st.ev], s->t_ev[st.ev + st.n]);
  }
  if (e != hipSuccess) return e;
  s->t_step = -1;
  s->t_spans.clear();
  s->t_ev_used = 0;
  return hipSuccess;
}

hipError_t begin_span(cgs_session s, int n, const int *kinds, TimedSpan **out) {
  hipError_t e = hipSuccess;
  if (s->t_ev_used + n + 1 > kTimeEvents) e = collect_times(s);
  if (e != hipSuccess) return e;
  TimedSpan sp{s->t_ev_used, n, {0, 0, 0}};
  for (int k = 0; k < n; ++k) sp.kind[k] = kinds[k];
  s->t_ev_used += (uint32_t)n + 1;
  s->t_spans.push_back(sp);
  *out = &s->t_spans.back();
  return hipEventRecord(s->t_ev[sp.ev], s->space->stream);
}

// Records the marker after kernel k of a span.
hipError_t mark_span(cgs_session s, const TimedSpan *sp, int k) {
  return hipEventRecord(s->t_ev[sp->ev + k + 1], s->space->stream);
}

// Waits for the draw numbered s->seq.  The draw publishes its result in
// pinned memory before its kernel ends, so the host polls that instead of
// sleeping on the stream; past kSpinLimit it waits for the stream, and a
// draw that still has not published is an error.
cgs_status wait_draw(cgs_session s, const DrawResult *res, uint64_t seq) {
  constexpr auto kSpinLimit = std::chrono::milliseconds(5);
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t it = 0;; ++it) {
    if (__atomic_load_n(&res->seq, __ATOMIC_ACQUIRE) == seq) return CGS_OK;
    if ((it & 1023u) == 1023u && std::chrono::steady_clock::now() - t0 > kSpinLimit) break;
#if defined(__x86_64__) && !defined(__HIP_DEVICE_COMPILE__)
    __builtin_ia32_pause();
#endif
  }
  HIP_TRY(hipStreamSynchronize(s->space->stream));
  if (__atomic_load_n(&res->seq, __ATOMIC_ACQUIRE) != seq)
    return fail(CGS_EDEVICE, "draw %llu did not publish its result", (unsigned long long)seq);
  return CGS_OK;
}

// Enqueues the recorded step: score pass, weight pass, and either its first
// draw (do_draw) or just the marking of its profiled configuration.
// Enqueues the recorded neighbourhood step: candidate scoring, compaction and
// weights, then either its first draw or the marking of its profile.
hipError_t launch_pending_nb(cgs_session s, bool do_draw, uint64_t u64) {
  cgs_space sp = s->space;
  cgs_model m = s->pending_model;
  const NbStep &st = s->pending_nbstep;
  const uint32_t nv = (uint32_t)sp->n_valid;
  const bool timed = s->params.timing > 0 && s->n_launched % (uint64_t)s->params.timing == 0;
  hipError_t e = hipSuccess;
  TimedSpan *span = nullptr;
  if (timed) {
    const int kinds[2] = {4, do_draw ? 2 : 3};
    e = begin_span(s, 2, kinds, &span);
    s->t_step = (int32_t)(s->t_spans.size() - 1);
  }
  if (e == hipSuccess)
    e = launch_nb_score(st, s->d_sub_off, s->d_sub_code, sp->d_mask, sp->d_rank, s->d_explored,
                        m->d_P, m->stride, s->d_nb_tmp_idx, s->d_nb_tmp_s, s->d_nb_acc,
                        sp->stream);
  if (e == hipSuccess)
    e = launch_nb_finish(st.total, s->d_nb_tmp_idx, s->d_nb_tmp_s, s->d_nb_acc, s->params.gamma,
                         s->params.w_min, s->d_nb_idx, s->d_nb_s, s->d_nb_q, s->d_nb_bsum,
                         s->d_nb_stats, sp->stream);
  if (e == hipSuccess && timed) e = mark_span(s, span, 0);
  if (e == hipSuccess) {
    if (do_draw)
      e = launch_nb_draw(s->d_nb_q, s->d_nb_idx, s->d_nb_stats, s->d_nb_bsum, s->d_explored,
                         st.profile, 1, nv, u64, sp->d_idx, s->d_res, ++s->seq, sp->stream);
    else
      e = launch_mark_one(s->d_explored, st.profile, nv, sp->stream);
  }
  if (e == hipSuccess && timed) e = mark_span(s, span, 1);
  if (e != hipSuccess) return e;
  ++s->n_launched;
  s->step_timed = timed;
  s->ran_in_batch = false;
  s->last_nb = true;
  s->pending = false;
  s->pending_nb = false;
  return hipSuccess;
}

// Enqueues one full step: score pass, weight pass, and either its first
// draw (do_draw; result in d_res under sequence number seq) or just the
// marking of its profiled configuration.  The profile is `prof` or, with
// d_prof_in, the word the previous step's draw left in device memory
// (`scored` then tells whether the step has counters to score); with
// d_prof_out the draw leaves its pick there.  Advances the accumulator set.
hipError_t launch_full_step(cgs_session s, cgs_model m, const ActiveCounters &act, uint32_t prof,
                            const uint32_t *d_prof_in, uint32_t *d_prof_out, bool scored,
                            bool do_draw, uint64_t u64, DrawResult *d_res, uint64_t seq) {
  cgs_space sp = s->space;
  const uint32_t nv = (uint32_t)sp->n_valid;
  StepAcc *acc = s->d_acc + s->parity * kAccSlots;
  StepAcc *acc_next = s->d_acc + (s->parity ^ 1) * kAccSlots;
  const bool timed = s->params.timing > 0 && s->n_launched % (uint64_t)s->params.timing == 0;
  hipError_t e = hipSuccess;
  TimedSpan *span = nullptr;
  if (timed) {
    // kind 5: a score pass that reads no prediction (no profile or no active
    // counter, e.g. the uniform start), kept out of the score-pass totals
    const int kinds[3] = {scored ? 0 : 5, 1, do_draw ? 2 : 3};
    e = begin_span(s, 3, kinds, &span);
    s->t_step = (int32_t)(s->t_spans.size() - 1);
  }
  if (e == hipSuccess)
    e = launch_score_pass(m->d_P, m->stride, prof, act, s->d_explored, nv, s->d_s, acc,
                          sp->stream, d_prof_in);
  if (e == hipSuccess && timed) e = mark_span(s, span, 0);
  if (e == hipSuccess)
    e = launch_weight_pass(s->d_s, s->d_explored, nv, prof, acc, acc_next, s->params.gamma,
                           s->params.w_min, s->block_log2, s->d_bsum, s->n_blocks, sp->stream,
                           d_prof_in);
  if (e == hipSuccess && timed) e = mark_span(s, span, 1);
  if (e == hipSuccess) {
    if (do_draw)
      e = launch_draw(s->d_s, s->d_explored, nv, prof, true, acc, s->params.gamma, s->params.w_min,
                      s->block_log2, s->d_bsum, s->n_blocks, u64, sp->d_idx, d_res, seq,
                      sp->stream, d_prof_in, d_prof_out);
    else
      e = launch_mark_one(s->d_explored, prof, nv, sp->stream);
  }
  if (e == hipSuccess && timed) e = mark_span(s, span, 2);
  if (e != hipSuccess) return e;
  ++s->n_launched;
  s->step_timed = timed;
  s->ran_in_batch = false;
  s->last_nb = false;
  s->cur_acc = s->parity;
  s->parity ^= 1;
  return hipSuccess;
}

hipError_t launch_pending(cgs_session s, bool do_draw, uint64_t u64) {
  if (s->pending_nb) return launch_pending_nb(s, do_draw, u64);
  const uint32_t prof = s->pending_profile;
  const bool scored = prof < (uint32_t)s->space->n_valid && s->pending_act.n > 0;
  const uint64_t seq = do_draw ? ++s->seq : s->seq;
  const hipError_t e = launch_full_step(s, s->pending_model, s->pending_act, prof, nullptr,
                                        nullptr, scored, do_draw, u64, s->d_res, seq);
  if (e != hipSuccess) return e;
  s->pending = false;
  return hipSuccess;
}

cgs_status flush_pending(cgs_session s) {
  if (s->pending) HIP_TRY(launch_pending(s, false, 0));
  return CGS_OK;
}

} // namespace

extern "C" cgs_status cgs_session_kernel_times(cgs_session s, double *total_ms, uint64_t *launches) {
  if (!s || !total_ms || !launches) return fail(CGS_EINVAL, "NULL argument");
  HIP_TRY(collect_times(s));
  for (int i = 0; i < 4; ++i) {
    total_ms[i] = s->kernel_ms[i];
    launches[i] = s->kernel_n[i];
  }
  return CGS_OK;
}

extern "C" cgs_status cgs_session_create(cgs_space sp, const cgs_params *params, cgs_session *out) {
  if (!out) return fail(CGS_EINVAL, "NULL out");
  *out = nullptr;
  if (!sp) return fail(CGS_EINVAL, "NULL space");
  cgs_params p;
  cgs_default_params(&p);
  if (params) p = *params;
  if (!std::isfinite(p.gamma) || p.gamma > 0.0f)
    return fail(CGS_EINVAL, "gamma must be finite and <= 0");
  if (!(p.w_min > 0.0f) || !(p.w_min <= 1.0f)) return fail(CGS_EINVAL, "w_min must be in (0, 1]");
  if (p.timing < 0) return fail(CGS_EINVAL, "timing must be >= 0");
  if (p.block_log2 != 0 && (p.block_log2 < 12 || p.block_log2 > 20))
    return fail(CGS_ERANGE, "block_log2 must be 0 or 12..20");
  cgs_session s = new (std::nothrow) cgs_session_s();
  if (!s) return fail(CGS_ENOMEM, "host allocation");
  s->space = sp;
  ++sp->refs;
  s->params = p;
  s->block_log2 = p.block_log2 ? p.block_log2 : auto_block_log2(sp->n_valid);
  s->n_blocks = (uint32_t)((sp->n_valid + (1ull << s->block_log2) - 1) >> s->block_log2);
  if (s->n_blocks > (1u << 20)) {
    destroy_session(s);
    return fail(CGS_ERANGE, "too many weight blocks; raise block_log2");
  }
  const uint64_t stride = (sp->n_valid + 63) & ~(uint64_t)63;
  const uint64_t n_words = (sp->n_valid + 31) / 32;
  hipError_t e = dalloc(&s->d_explored, n_words);
  if (e == hipSuccess) e = dalloc(&s->d_s, stride);
  if (e == hipSuccess) e = dalloc(&s->d_bsum, s->n_blocks);
  if (e == hipSuccess) e = dalloc(&s->d_acc, 2 * kAccSlots);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void **>(&s->h_res), sizeof(DrawResult),
                      hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess) {
    std::memset(s->h_res, 0, sizeof(DrawResult));
    e = hipHostGetDevicePointer(reinterpret_cast<void **>(&s->d_res), s->h_res, 0);
  }
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void **>(&s->h_acc), kAccSlots * sizeof(StepAcc), 0);
  if (e == hipSuccess) e = dalloc(&s->d_prof, 2);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void **>(&s->h_ring), kResultRing * sizeof(DrawResult),
                      hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess) {
    std::memset(s->h_ring, 0, kResultRing * sizeof(DrawResult));
    e = hipHostGetDevicePointer(reinterpret_cast<void **>(&s->d_ring), s->h_ring, 0);
  }
  if (e == hipSuccess && p.timing > 0) {
    s->t_ev.assign(kTimeEvents, nullptr);
    s->t_spans.reserve(kTimeEvents / 2);
    for (uint32_t i = 0; i < kTimeEvents && e == hipSuccess; ++i)
      e = hipEventCreateWithFlags(&s->t_ev[i], hipEventDisableSystemFence);
  }
  if (e == hipSuccess)
    e = hipMemsetAsync(s->d_explored, 0, std::max<uint64_t>(n_words, 1) * sizeof(uint32_t),
                       sp->stream);
  if (e == hipSuccess) e = hipMemsetAsync(s->d_s, 0, stride * sizeof(float), sp->stream);
  if (e == hipSuccess) e = launch_reset_acc(s->d_acc, 2 * kAccSlots, sp->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(sp->stream);
  if (e != hipSuccess) {
    destroy_session(s);
    return fail(e == hipErrorOutOfMemory ? CGS_ENOMEM : CGS_EDEVICE, "session buffers: %s",
                hipGetErrorString(e));
  }
  *out = s;
  return CGS_OK;
}

namespace {

// Counters entering a step's score: dpc from `delta` (each in [-1, 1]) or
// from the expert system on `measured` (24 Table 1 counters); none for the
// start of a search.
cgs_status step_counters(cgs_model m, bool no_profile, const float *delta, const double *measured,
                         const cgs_expert_params *expert, ActiveCounters *act) {
  const int C = m->n_counters;
  float dpc[CGS_MAX_COUNTERS] = {};
  if (no_profile) {
    // every score 0: uniform draw over unexplored configurations
  } else if (delta) {
    for (int c = 0; c < C; ++c) {
      if (!(delta[c] >= -1.0f && delta[c] <= 1.0f))
        return fail(CGS_EINVAL, "delta[%d] = %g outside [-1, 1]", c, (double)delta[c]);
      dpc[c] = delta[c];
    }
  } else {
    if (!measured) return fail(CGS_EINVAL, "need delta or measured counters");
    if (C != 24)
      return fail(CGS_EINVAL, "measured counters need a model of the 24 Table 1 counters");
    double b[18], d[24];
    const cgs_status st = cgs_expert_system(measured, expert, b, d, nullptr);
    if (st != CGS_OK) return fail(st, "expert system rejected the measured counters");
    for (int c = 0; c < 24; ++c) dpc[c] = (float)d[c];
  }
  *act = ActiveCounters{};
  for (int c = 0; c < C; ++c)
    if (dpc[c] != 0.0f) {
      act->ctr[act->n] = (uint32_t)c;
      act->delta[act->n] = dpc[c];
      ++act->n;
    }
  return CGS_OK;
}

// Subsets of 1..radius parameters in lexicographic order with the offset of
// each subset's first neighbour; subsets containing a parameter with a
// single value have no neighbours and are left out.
cgs_status build_subsets(cgs_session s, int radius, uint32_t *n_subsets, uint32_t *total) {
  const std::vector<int32_t> &r = s->space->radix;
  const int P = (int)r.size();
  std::vector<uint32_t> off{0}, code;
  uint64_t run = 0;
  auto add = [&](int n, int j0, int j1, int j2) {
    uint64_t c = (uint64_t)(r[j0] - 1);
    if (n > 1) c *= (uint64_t)(r[j1] - 1);
    if (n > 2) c *= (uint64_t)(r[j2] - 1);
    if (c == 0) return;
    code.push_back((uint32_t)j0 | (uint32_t)(n > 1 ? j1 : 0) << 8 |
                   (uint32_t)(n > 2 ? j2 : 0) << 16 | (uint32_t)n << 24);
    run += c;
    off.push_back((uint32_t)std::min<uint64_t>(run, 0xffffffffull));
  };
  for (int j = 0; j < P; ++j) add(1, j, 0, 0);
  if (radius >= 2)
    for (int j = 0; j < P; ++j)
      for (int k = j + 1; k < P; ++k) add(2, j, k, 0);
  if (radius >= 3)
    for (int j = 0; j < P; ++j)
      for (int k = j + 1; k < P; ++k)
        for (int l = k + 1; l < P; ++l) add(3, j, k, l);
  if (run > kNbMaxCandidates)
    return fail(CGS_ERANGE, "radius %d gives %llu neighbours, more than %u", radius,
                (unsigned long long)run, kNbMaxCandidates);
  if (run == 0) return fail(CGS_EEMPTY, "the neighbourhood of radius %d is empty", radius);
  const uint32_t n = (uint32_t)code.size();
  dfree(s->d_sub_off);
  dfree(s->d_sub_code);
  s->nb_radius = 0;
  hipError_t e = dalloc(&s->d_sub_off, n + 1);
  if (e == hipSuccess) e = dalloc(&s->d_sub_code, n);
  hipStream_t st = s->space->stream;
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_sub_off, off.data(), (n + 1) * sizeof(uint32_t), hipMemcpyHostToDevice,
                       st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->d_sub_code, code.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice,
                       st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? CGS_ENOMEM : CGS_EDEVICE, "subset table: %s",
                hipGetErrorString(e));
  s->nb_radius = radius;
  *n_subsets = n;
  *total = (uint32_t)run;
  return CGS_OK;
}

// Candidate buffers of restricted steps, allocated on first use.
cgs_status ensure_nb_buffers(cgs_session s) {
  if (s->d_nb_stats) return CGS_OK;
  hipError_t e = dalloc(&s->d_nb_tmp_idx, kNbMaxCandidates);
  if (e == hipSuccess) e = dalloc(&s->d_nb_tmp_s, kNbMaxCandidates);
  if (e == hipSuccess) e = dalloc(&s->d_nb_idx, kNbMaxCandidates);
  if (e == hipSuccess) e = dalloc(&s->d_nb_s, kNbMaxCandidates);
  if (e == hipSuccess) e = dalloc(&s->d_nb_q, kNbMaxCandidates);
  if (e == hipSuccess) e = dalloc(&s->d_nb_bsum, kNbBlocks);
  if (e == hipSuccess) e = dalloc(&s->d_nb_acc, kAccSlots);
  if (e == hipSuccess) e = launch_reset_acc(s->d_nb_acc, kAccSlots, s->space->stream);
  if (e == hipSuccess) e = dalloc(&s->d_nb_stats, 1);
  if (e == hipSuccess) e = hipStreamSynchronize(s->space->stream);
  if (e != hipSuccess) {
    dfree(s->d_nb_stats);
    s->d_nb_stats = nullptr;
    return fail(e == hipErrorOutOfMemory ? CGS_ENOMEM : CGS_EDEVICE, "neighbourhood buffers: %s",
                hipGetErrorString(e));
  }
  return CGS_OK;
}

} // namespace

extern "C" cgs_status cgs_search_step(cgs_session s, cgs_model m, uint64_t profile_raw,
                                      const float *delta, const double *measured,
                                      const cgs_expert_params *expert) {
  if (!s || !m) return fail(CGS_EINVAL, "NULL session or model");
  cgs_space sp = s->space;
  if (m->space != sp) return fail(CGS_EINVAL, "model and session belong to different spaces");
  const bool no_profile = profile_raw == CGS_NO_PROFILE;
  const int64_t prof = no_profile ? 0 : valid_index_of(sp, profile_raw);
  if (prof < 0)
    return fail(CGS_EINVAL, "profile %llu is not a valid configuration",
                (unsigned long long)profile_raw);
  if (sp->n_valid == 0) return fail(CGS_EEMPTY, "the space has no valid configuration");
  ActiveCounters act{};
  cgs_status st = step_counters(m, no_profile, delta, measured, expert, &act);
  if (st != CGS_OK) return st;
  // a step recorded but never drawn from still marks its profile and scores
  st = flush_pending(s);
  if (st != CGS_OK) return st;
  s->pending = true;
  s->pending_nb = false;
  s->pending_model = m;
  s->pending_profile = no_profile ? kNoProfile : (uint32_t)prof;
  s->pending_act = act;
  s->stepped = true;
  s->n_active = act.n;
  s->last_total = 0;
  return CGS_OK;
}

// n_steps steps of the counter-guided search, each the work of one
// cgs_search_step with measured counters plus one cgs_sample_next, with
// the same results.  Every step's counter changes come from the measured
// counters alone, so the expert system runs for all steps first and the
// steps are enqueued ahead of their picks (up to kResultRing - 1 ahead of
// the last pick read): step k reads its profiled configuration from the
// device word the draw of step k - 1 wrote, and its draw's result lands in
// ring slot k.  The host reads the picks in order as they are published.
extern "C" cgs_status cgs_search_run(cgs_session s, cgs_model m, int n_steps,
                                     const double *measured, const cgs_expert_params *expert,
                                     const uint64_t *u64, uint64_t *raw_out, uint64_t *valid_out,
                                     double *step_us) {
  if (!s || !m || !u64 || !raw_out || (n_steps > 0 && (!measured || !expert)))
    return fail(CGS_EINVAL, "NULL argument");
  if (n_steps < 0) return fail(CGS_EINVAL, "negative n_steps");
  for (int i = 0; i <= n_steps; ++i) {
    raw_out[i] = CGS_NO_PROFILE;
    if (valid_out) valid_out[i] = CGS_NO_PROFILE;
  }
  cgs_space sp = s->space;
  if (m->space != sp) return fail(CGS_EINVAL, "model and session belong to different spaces");
  if (sp->n_valid == 0) return fail(CGS_EEMPTY, "the space has no valid configuration");
  std::vector<ActiveCounters> acts((size_t)n_steps + 1);
  cgs_status st = step_counters(m, true, nullptr, nullptr, nullptr, &acts[0]);
  for (int i = 0; i < n_steps && st == CGS_OK; ++i)
    st = step_counters(m, false, nullptr, measured + (size_t)i * 24, expert + i, &acts[i + 1]);
  if (st != CGS_OK) return st;
  st = flush_pending(s);
  if (st != CGS_OK) return st;
  const uint64_t seq0 = s->seq;
  // step k: profile from d_prof[k & 1] (none for the start), pick to
  // d_prof[(k + 1) & 1], result in ring slot k % kResultRing
  auto launch = [&](int k) {
    const uint32_t *in = k == 0 ? nullptr : s->d_prof + (k & 1);
    return launch_full_step(s, m, acts[k], kNoProfile, in, s->d_prof + ((k + 1) & 1),
                            k > 0 && acts[k].n > 0, true, u64[k], s->d_ring + k % kResultRing,
                            seq0 + (uint64_t)k + 1);
  };
  // leaves the session as after the last launched step: no further draw
  // is pending, the stream has finished everything this call enqueued
  int launched = 0;
  auto finish = [&](cgs_status r) {
    s->seq = seq0 + (uint64_t)launched;
    s->stepped = s->stepped || launched > 0;
    const hipError_t e = hipStreamSynchronize(sp->stream);
    if (r == CGS_OK && e != hipSuccess)
      return fail(CGS_EDEVICE, "search run: %s", hipGetErrorString(e));
    return r;
  };
  auto t_prev = std::chrono::steady_clock::now();
  for (int k = 0; k <= n_steps; ++k) {
    while (launched <= n_steps && launched < k + (int)kResultRing - 1) {
      const hipError_t e = launch(launched);
      if (e != hipSuccess)
        return finish(fail(CGS_EDEVICE, "search run step %d: %s", launched, hipGetErrorString(e)));
      ++launched;
    }
    const DrawResult *slot = s->h_ring + k % kResultRing;
    const cgs_status ws = wait_draw(s, slot, seq0 + (uint64_t)k + 1);
    if (ws != CGS_OK) return finish(ws);
    const auto t = std::chrono::steady_clock::now();
    DrawResult r;
    std::memcpy(&r, const_cast<const DrawResult *>(static_cast<volatile const DrawResult *>(slot)),
                sizeof r);
    s->last_total = r.total;
    s->n_active = acts[k].n;
    if (r.total == 0) return finish(fail(CGS_EEMPTY, "no unexplored valid configuration is left"));
    if (r.valid == kNoPick)
      return finish(fail(CGS_EDEVICE, "draw found no configuration although Q = %llu",
                         (unsigned long long)r.total));
    raw_out[k] = r.raw;
    if (valid_out) valid_out[k] = r.valid;
    if (k > 0 && step_us) step_us[k - 1] = std::chrono::duration<double, std::micro>(t - t_prev).count();
    t_prev = t;
  }
  return finish(CGS_OK);
}

extern "C" void cgs_default_online_opts(cgs_online_opts *o) {
  if (!o) return;
  o->retrain_every = 20;
  o->train_steps = 500;
  o->batch = 256;
  o->reserved = 0;
  o->lr = 1e-3f;
  o->beta1 = 0.9f;
  o->beta2 = 0.999f;
  o->eps = 1e-8f;
  o->threshold = 0.05;
}

// cgs_model_rmse(mlp, tree, sample) for a perceptron whose full-space
// predictions are stale: the inference kernel evaluates only the sampled
// configurations (each configuration's result does not depend on which
// others share its launch, so these are the values a full evaluation
// would give) and the same sums are formed in the same order.
cgs_status mlp_sample_rmse(cgs_model mlp, cgs_model tree, const uint32_t *sample, uint64_t n,
                           double *rmse) {
  cgs_space sp = mlp->space;
  if (n == 0 || n > 0xffffffffull) return fail(CGS_ERANGE, "need 1 .. 2^32-1 samples");
  std::vector<uint32_t> raw(n);
  for (uint64_t i = 0; i < n; ++i) {
    if (sample[i] >= sp->n_valid)
      return fail(CGS_EINVAL, "sample %llu outside the valid list", (unsigned long long)i);
    raw[i] = sp->h_idx[sample[i]];
  }
  const int C = mlp->n_counters;
  const uint64_t stride = (n + 63) & ~(uint64_t)63;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((n + 255) / 256, 1024);
  uint32_t *d_s = nullptr, *d_raw = nullptr;
  float *d_p = nullptr;
  double *d_part = nullptr;
  std::vector<double> part(grid);
  hipError_t e = dalloc(&d_s, n);
  if (e == hipSuccess) e = dalloc(&d_raw, n);
  if (e == hipSuccess) e = dalloc(&d_p, (size_t)C * stride);
  if (e == hipSuccess) e = dalloc(&d_part, grid);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_s, sample, n * sizeof(uint32_t), hipMemcpyHostToDevice, sp->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_raw, raw.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, sp->stream);
  if (e == hipSuccess) {
    MlpFwdArgs a = mlp_args(mlp);
    a.idx = d_raw;
    a.n = (uint32_t)n;
    a.P = d_p;
    a.stride = stride;
    e = launch_mlp_forward(a, false, sp->stream);
  }
  if (e == hipSuccess)
    e = launch_sq_diff_dense(d_p, tree->d_P, stride, tree->stride, C, d_s, (uint32_t)n, d_part,
                             grid, sp->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(part.data(), d_part, grid * sizeof(double), hipMemcpyDeviceToHost,
                       sp->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(sp->stream);
  dfree(d_s);
  dfree(d_raw);
  dfree(d_p);
  dfree(d_part);
  if (e != hipSuccess) return fail(CGS_EDEVICE, "rmse: %s", hipGetErrorString(e));
  double sum = 0.0;
  for (double v : part) sum += v;
  *rmse = std::sqrt(sum / ((double)n * C));
  return CGS_OK;
}

// The online policy around the library's own calls: per window one
// cgs_model_rmse (and, after the first window, one cgs_mlp_train), per step
// one cgs_search_step and one cgs_sample_next.  Targets of the collected pairs
// are gathered from the tree once per window.
extern "C" cgs_status cgs_online_run(cgs_session s, cgs_model tree, cgs_model mlp, int n_steps,
                                     const float *delta, const uint64_t *u64, const float *noise,
                                     uint64_t n_seed, const uint32_t *seed_cfg,
                                     const float *seed_targets, uint64_t n_val,
                                     const uint32_t *val_sample, const uint64_t *batch_u64,
                                     const cgs_online_opts *opts, uint64_t *raw_out,
                                     uint64_t *valid_out, double *window_rmse,
                                     int32_t *window_mlp, double *step_us, double *retrain_ms) {
  if (!s || !tree || !mlp || !u64 || !noise || !val_sample || !opts || !raw_out ||
      !window_rmse || !window_mlp || (n_seed && (!seed_cfg || !seed_targets)))
    return fail(CGS_EINVAL, "NULL argument");
  if (n_steps < 0) return fail(CGS_EINVAL, "negative n_steps");
  if (n_steps > 0 && !delta) return fail(CGS_EINVAL, "NULL delta");
  if (mlp->kind != 1) return fail(CGS_EINVAL, "the surrogate is not a perceptron model");
  if (tree->space != s->space || mlp->space != s->space)
    return fail(CGS_EINVAL, "models and session belong to different spaces");
  if (tree->n_counters != mlp->n_counters) return fail(CGS_EINVAL, "models differ in counters");
  const int W = opts->retrain_every;
  if (W < 1) return fail(CGS_EINVAL, "retrain_every %d < 1", W);
  if (opts->train_steps < 0 || opts->batch < 1 || opts->batch > 4096)
    return fail(CGS_ERANGE, "train_steps %d / batch %d outside 0.. / 1..4096", opts->train_steps,
                opts->batch);
  if (opts->train_steps > 0 && n_steps >= W && !batch_u64)
    return fail(CGS_EINVAL, "NULL batch_u64");
  if (!std::isfinite(opts->threshold)) return fail(CGS_EINVAL, "threshold must be finite");
  const int C = tree->n_counters;
  const int n_windows = 1 + n_steps / W;
  for (int i = 0; i <= n_steps; ++i) {
    raw_out[i] = CGS_NO_PROFILE;
    if (valid_out) valid_out[i] = CGS_NO_PROFILE;
  }
  for (int w = 0; w < n_windows; ++w) {
    window_rmse[w] = NAN;
    window_mlp[w] = -1;
  }
  std::vector<uint32_t> cfg(seed_cfg, seed_cfg + n_seed);
  std::vector<float> tgt(seed_targets, seed_targets + n_seed * (uint64_t)C);
  std::vector<uint32_t> fresh;     // valid indices of picks whose targets are not gathered yet
  std::vector<int> fresh_step;     // and the step that picked them (row of noise)
  std::vector<float> pred;
  std::vector<int32_t> rows;
  auto gather_fresh = [&]() -> cgs_status {
    if (fresh.empty()) return CGS_OK;
    pred.resize(fresh.size() * (size_t)C);
    const cgs_status st = cgs_model_gather_predictions(tree, fresh.data(), fresh.size(), pred.data());
    if (st != CGS_OK) return st;
    for (size_t k = 0; k < fresh.size(); ++k)
      for (int c = 0; c < C; ++c)
        tgt.push_back(pred[k * C + c] + noise[(size_t)fresh_step[k] * C + c]);
    fresh.clear();
    fresh_step.clear();
    return CGS_OK;
  };
  // The surrogate's full-space predictions are refreshed only for windows
  // that score with it (and once before returning): a retrained network that
  // fails the RMSE check is never evaluated beyond the validation sample.
  auto rmse_of_mlp = [&](double *r) {
    return mlp->p_stale ? mlp_sample_rmse(mlp, tree, val_sample, n_val, r)
                        : cgs_model_rmse(mlp, tree, val_sample, n_val, r);
  };
  auto refresh = [&]() -> cgs_status {
    if (!mlp->p_stale) return CGS_OK;
    mlp->p_stale = false;
    return evaluate_model(mlp);
  };
  auto done = [&](cgs_status st) {
    const cgs_status r = refresh();
    return st != CGS_OK ? st : r;
  };
  double rmse = 0.0;
  cgs_status st = rmse_of_mlp(&rmse);
  if (st != CGS_OK) return done(st);
  bool use_mlp = rmse <= opts->threshold;
  window_rmse[0] = rmse;
  window_mlp[0] = use_mlp;
  st = cgs_search_step(s, tree, CGS_NO_PROFILE, nullptr, nullptr, nullptr);
  uint64_t raw = 0, valid = 0;
  if (st == CGS_OK) st = cgs_sample_next(s, u64[0], &raw, &valid);
  if (st != CGS_OK) return done(st);
  raw_out[0] = raw;
  if (valid_out) valid_out[0] = valid;
  cfg.push_back((uint32_t)raw);
  fresh.push_back((uint32_t)valid);
  fresh_step.push_back(0);
  for (int i = 1; i <= n_steps; ++i) {
    if (i % W == 0) {
      const int w = i / W;
      const auto t0 = std::chrono::steady_clock::now();
      st = gather_fresh();
      if (st != CGS_OK) return done(st);
      if (opts->train_steps > 0) {
        // row of each batch entry: floor(u * n_pairs / 2^64), one u per entry
        const uint64_t np = cfg.size(), per = (uint64_t)opts->train_steps * opts->batch;
        const uint64_t *u = batch_u64 + (uint64_t)(w - 1) * per;
        rows.resize(per);
        for (uint64_t k = 0; k < per; ++k)
          rows[k] = (int32_t)(((unsigned __int128)u[k] * np) >> 64);
        const cgs_train_opts to{opts->lr,    opts->beta1, opts->beta2,
                                opts->eps,   opts->batch, opts->train_steps};
        st = mlp_train_run(mlp, cfg.data(), tgt.data(), np, rows.data(), &to, nullptr, false);
        if (st != CGS_OK) return done(st);
      }
      st = rmse_of_mlp(&rmse);
      if (st != CGS_OK) return done(st);
      use_mlp = rmse <= opts->threshold;
      window_rmse[w] = rmse;
      window_mlp[w] = use_mlp;
      if (use_mlp) st = refresh();
      if (st != CGS_OK) return done(st);
      if (retrain_ms)
        retrain_ms[w - 1] =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    const auto t0 = std::chrono::steady_clock::now();
    st = cgs_search_step(s, use_mlp ? mlp : tree, raw, delta + (size_t)(i - 1) * C, nullptr,
                         nullptr);
    if (st == CGS_OK) st = cgs_sample_next(s, u64[i], &raw, &valid);
    if (st != CGS_OK) return done(st);
    if (step_us)
      step_us[i - 1] =
          std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
    raw_out[i] = raw;
    if (valid_out) valid_out[i] = valid;
    cfg.push_back((uint32_t)raw);
    fresh.push_back((uint32_t)valid);
    fresh_step.push_back(i);
  }
  return done(CGS_OK);
}

extern "C" cgs_status cgs_search_step_neighbourhood(cgs_session s, cgs_model m,
                                                    uint64_t profile_raw, int radius,
                                                    const float *delta, const double *measured,
                                                    const cgs_expert_params *expert) {
  if (!s || !m) return fail(CGS_EINVAL, "NULL session or model");
  cgs_space sp = s->space;
  if (m->space != sp) return fail(CGS_EINVAL, "model and session belong to different spaces");
  if (radius < 1 || radius > CGS_MAX_RADIUS)
    return fail(CGS_EINVAL, "radius %d outside 1..%d", radius, CGS_MAX_RADIUS);
  if (profile_raw == CGS_NO_PROFILE)
    return fail(CGS_EINVAL, "a restricted step needs a profiled configuration");
  const int64_t prof = valid_index_of(sp, profile_raw);
  if (prof < 0)
    return fail(CGS_EINVAL, "profile %llu is not a valid configuration",
                (unsigned long long)profile_raw);
  ActiveCounters act{};
  cgs_status st = step_counters(m, false, delta, measured, expert, &act);
  if (st != CGS_OK) return st;
  st = flush_pending(s);
  if (st != CGS_OK) return st;
  st = ensure_nb_buffers(s);
  if (st != CGS_OK) return st;
  NbStep &nb = s->pending_nbstep;
  if (s->nb_radius != radius) {
    st = build_subsets(s, radius, &nb.n_subsets, &nb.total);
    if (st != CGS_OK) return st;
  }
  const int P = sp->n_params;
  uint64_t k = profile_raw, stride = 1;
  for (int j = P - 1; j >= 0; --j) {
    const uint32_t r = (uint32_t)sp->radix[j];
    nb.radix[j] = (uint8_t)r;
    nb.pdig[j] = (uint8_t)(k % r);
    k /= r;
    nb.stride[j] = (uint32_t)stride;
    stride *= r;
  }
  nb.profile_raw = (uint32_t)profile_raw;
  nb.profile = (uint32_t)prof;
  nb.act = act;
  s->pending = true;
  s->pending_nb = true;
  s->pending_model = m;
  s->pending_profile = (uint32_t)prof;
  s->pending_act = act;
  s->stepped = true;
  s->n_active = act.n;
  s->last_total = 0;
  return CGS_OK;
}

extern "C" cgs_status cgs_session_copy_neighbourhood(cgs_session s, uint64_t capacity,
                                                     uint32_t *valid_idx, float *scores,
                                                     uint32_t *q, uint64_t *count) {
  if (!s || !count) return fail(CGS_EINVAL, "NULL argument");
  const cgs_status st = flush_pending(s);
  if (st != CGS_OK) return st;
  if (!s->last_nb) return fail(CGS_ESTATE, "the last step was not restricted to a neighbourhood");
  cgs_space sp = s->space;
  NbStats stats{};
  HIP_TRY(hipMemcpyAsync(&stats, s->d_nb_stats, sizeof stats, hipMemcpyDeviceToHost, sp->stream));
  HIP_TRY(hipStreamSynchronize(sp->stream));
  *count = stats.count;
  if (stats.count > capacity)
    return fail(CGS_ERANGE, "%u candidates, capacity %llu", stats.count,
                (unsigned long long)capacity);
  if (stats.count == 0) return CGS_OK;
  if (valid_idx)
    HIP_TRY(hipMemcpyAsync(valid_idx, s->d_nb_idx, stats.count * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, sp->stream));
  if (scores)
    HIP_TRY(hipMemcpyAsync(scores, s->d_nb_s, stats.count * sizeof(float), hipMemcpyDeviceToHost,
                           sp->stream));
  if (q)
    HIP_TRY(hipMemcpyAsync(q, s->d_nb_q, stats.count * sizeof(uint32_t), hipMemcpyDeviceToHost,
                           sp->stream));
  HIP_TRY(hipStreamSynchronize(sp->stream));
  return CGS_OK;
}

extern "C" cgs_status cgs_sample_next(cgs_session s, uint64_t u64, uint64_t *raw_out,
                                      uint64_t *valid_out) {
  if (!s) return fail(CGS_EINVAL, "NULL session");
  if (!s->stepped) return fail(CGS_ESTATE, "cgs_sample_next before any cgs_search_step");
  cgs_space sp = s->space;
  if (sp->n_valid == 0) return fail(CGS_EEMPTY, "the space has no valid configuration");
  if (s->pending) {
    HIP_TRY(launch_pending(s, true, u64));
  } else {
    TimedSpan *span = nullptr;
    if (s->step_timed) {
      const int kinds[1] = {2};
      HIP_TRY(begin_span(s, 1, kinds, &span));
    }
    if (s->last_nb)
      HIP_TRY(launch_nb_draw(s->d_nb_q, s->d_nb_idx, s->d_nb_stats, s->d_nb_bsum, s->d_explored,
                             kNoProfile, 0, (uint32_t)sp->n_valid, u64, sp->d_idx, s->d_res,
                             ++s->seq, sp->stream));
    else
      HIP_TRY(launch_draw(s->d_s, s->d_explored, (uint32_t)sp->n_valid, kNoProfile, false,
                          s->d_acc + s->cur_acc * kAccSlots, s->params.gamma, s->params.w_min,
                          s->block_log2, s->d_bsum, s->n_blocks, u64, sp->d_idx, s->d_res,
                          ++s->seq, sp->stream));
    if (span) HIP_TRY(mark_span(s, span, 0));
  }
  const cgs_status ws = wait_draw(s, s->h_res, s->seq);
  if (ws != CGS_OK) return ws;
  DrawResult r;
  std::memcpy(&r, const_cast<const DrawResult *>(static_cast<volatile DrawResult *>(s->h_res)),
              sizeof r);
  s->last_total = r.total;
  if (r.total == 0) return fail(CGS_EEMPTY, "no unexplored valid configuration is left");
  if (r.valid == kNoPick)
    return fail(CGS_EDEVICE, "draw found no configuration although Q = %llu",
                (unsigned long long)r.total);
  if (raw_out) *raw_out = r.raw;
  if (valid_out) *valid_out = r.valid;
  return CGS_OK;
}

extern "C" cgs_status cgs_session_step_info(cgs_session s, cgs_step_info *out) {
  if (!s || !out) return fail(CGS_EINVAL, "NULL argument");
  if (!s->stepped) return fail(CGS_ESTATE, "no step yet");
  const cgs_status st = flush_pending(s);
  if (st != CGS_OK) return st;
  cgs_space sp = s->space;
  StepAccSums a{0xffffffffu, 0u, 0u};
  if (s->last_nb) {
    // a restricted step: its candidates
    NbStats stats{};
    HIP_TRY(hipMemcpyAsync(&stats, s->d_nb_stats, sizeof stats, hipMemcpyDeviceToHost,
                           sp->stream));
    HIP_TRY(hipStreamSynchronize(sp->stream));
    a = StepAccSums{stats.min_key, stats.max_key, stats.count};
  } else {
    HIP_TRY(hipMemcpyAsync(s->h_acc, s->d_acc + s->cur_acc * kAccSlots,
                           kAccSlots * sizeof(StepAcc), hipMemcpyDeviceToHost, sp->stream));
    HIP_TRY(hipStreamSynchronize(sp->stream));
    for (int i = 0; i < kAccSlots; ++i) {
      a.min_key = std::min(a.min_key, s->h_acc[i].min_key);
      a.max_key = std::max(a.max_key, s->h_acc[i].max_key);
      a.n_unexplored += s->h_acc[i].n_unexplored;
    }
  }
  auto key_to_float = [](uint32_t k) {
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    float f;
    std::memcpy(&f, &u, sizeof f);
    return f;
  };
  out->n_unexplored = a.n_unexplored;
  out->total_weight = s->last_total;
  out->s_min = a.n_unexplored ? key_to_float(a.min_key) : 0.0f;
  out->s_max = a.n_unexplored ? key_to_float(a.max_key) : 0.0f;
  float ms = 0.0f;
  if (s->ran_in_batch) {
    ms = s->batch_ms;
  } else if (s->params.timing > 0) {
    HIP_TRY(collect_times(s));
    ms = s->step_ms;
  }
  out->device_ms = ms;
  out->n_active = s->n_active;
  return CGS_OK;
}

extern "C" cgs_status cgs_mark_explored(cgs_session s, uint64_t raw) {
  if (!s) return fail(CGS_EINVAL, "NULL session");
  const int64_t l = valid_index_of(s->space, raw);
  if (l < 0) return fail(CGS_EINVAL, "raw index %llu is not valid", (unsigned long long)raw);
  const cgs_status st = flush_pending(s);
  if (st != CGS_OK) return st;
  uint32_t word = 0;
  cgs_space sp = s->space;
  HIP_TRY(hipMemcpyAsync(&word, s->d_explored + (l >> 5), sizeof(uint32_t), hipMemcpyDeviceToHost,
                         sp->stream));
  HIP_TRY(hipStreamSynchronize(sp->stream));
  word |= 1u << (l & 31);
  HIP_TRY(hipMemcpyAsync(s->d_explored + (l >> 5), &word, sizeof(uint32_t), hipMemcpyHostToDevice,
                         sp->stream));
  HIP_TRY(hipStreamSynchronize(sp->stream));
  return CGS_OK;
}

extern "C" cgs_status cgs_session_copy_scores(cgs_session s, uint64_t first, uint64_t count,
                                              float *dst) {
  if (!s || (!dst && count)) return fail(CGS_EINVAL, "NULL argument");
  cgs_space sp = s->space;
  if (first > sp->n_valid || count > sp->n_valid - first)
    return fail(CGS_ERANGE, "range outside the valid list");
  const cgs_status st = flush_pending(s);
  if (st != CGS_OK) return st;
  if (s->last_nb) return fail(CGS_ESTATE, "the last step was restricted to a neighbourhood");
  if (count == 0) return CGS_OK;
  HIP_TRY(hipMemcpyAsync(dst, s->d_s + first, count * sizeof(float), hipMemcpyDeviceToHost,
                         sp->stream));
  HIP_TRY(hipStreamSynchronize(sp->stream));
  return CGS_OK;
}

extern "C" cgs_status cgs_session_copy_weights(cgs_session s, uint64_t first, uint64_t count,
                                               uint32_t *dst) {
  if (!s || (!dst && count)) return fail(CGS_EINVAL, "NULL argument");
  if (!s->stepped) return fail(CGS_ESTATE, "no step yet");
  cgs_space sp = s->space;
  if (first > sp->n_valid || count > sp->n_valid - first)
    return fail(CGS_ERANGE, "range outside the valid list");
  const cgs_status st = flush_pending(s);
  if (st != CGS_OK) return st;
  if (s->last_nb) return fail(CGS_ESTATE, "the last step was restricted to a neighbourhood");
  if (count == 0) return CGS_OK;
  uint32_t *d_q = nullptr;
  HIP_TRY(dalloc(&d_q, count));
  hipError_t e = launch_copy_weights(s->d_s, s->d_explored, (uint32_t)sp->n_valid,
                                     s->d_acc + s->cur_acc * kAccSlots, s->params.gamma,
                                     s->params.w_min, (uint32_t)first, (uint32_t)count, d_q,
                                     sp->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dst, d_q, count * sizeof(uint32_t), hipMemcpyDeviceToHost, sp->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(sp->stream);
  dfree(d_q);
  if (e != hipSuccess) return fail(CGS_EDEVICE, "weights: %s", hipGetErrorString(e));
  return CGS_OK;
}

extern "C" cgs_status cgs_session_copy_explored(cgs_session s, uint32_t *dst, uint64_t n_words) {
  if (!s || !dst) return fail(CGS_EINVAL, "NULL argument");
  cgs_space sp = s->space;
  if (n_words != (sp->n_valid + 31) / 32) return fail(CGS_EINVAL, "wrong number of words");
  const cgs_status st = flush_pending(s);
  if (st != CGS_OK) return st;
  if (n_words == 0) return CGS_OK;
  HIP_TRY(hipMemcpyAsync(dst, s->d_explored, n_words * sizeof(uint32_t), hipMemcpyDeviceToHost,
                         sp->stream));
  HIP_TRY(hipStreamSynchronize(sp->stream));
  return CGS_OK;
}

extern "C" void cgs_session_destroy(cgs_session s) { destroy_session(s); }

// ------------------------------------------------------------------ batch
struct cgs_batch_s {
  int n = 0;
  std::vector<cgs_session> sess;
  std::vector<cgs_model> models;
  hipStream_t stream = nullptr;
  BatchSess *d_sess = nullptr;
  BatchStep *d_step = nullptr;
  BatchStep *h_step = nullptr;  // pinned
  DrawResult *h_res = nullptr;  // pinned, mapped
  DrawResult *d_res = nullptr;  // device view of h_res
  uint16_t *d_tile_sess = nullptr, *d_blk_sess = nullptr;
  uint32_t total_tiles = 0, total_blocks = 0;
  uint64_t total_valid = 0;
  int total_counters = 0;
  cgs_batch_schedule sched{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float last_ms = 0.0f;
  uint64_t seq = 0; // sequence number of the last batch step's draws
};

namespace {

void drop_graph(cgs_batch b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

void destroy_batch(cgs_batch b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  dfree(b->d_sess);
  dfree(b->d_step);
  dfree(b->d_tile_sess);
  dfree(b->d_blk_sess);
  if (b->h_step) (void)hipHostFree(b->h_step);
  if (b->h_res) (void)hipHostFree(b->h_res);
  if (b->e0) (void)hipEventDestroy(b->e0);
  if (b->e1) (void)hipEventDestroy(b->e1);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

// Enqueues one batched step (copy of the step records, score, weight, draw).
hipError_t enqueue_batch(cgs_batch b, bool draw) {
  hipError_t e = hipMemcpyAsync(b->d_step, b->h_step, (size_t)b->n * sizeof(BatchStep),
                                hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = launch_batch_score(b->d_sess, b->d_step, b->d_tile_sess, b->total_tiles,
                           (uint32_t)b->sched.score_grid, b->sched.variant, b->stream);
  if (e == hipSuccess)
    e = launch_batch_weight(b->d_sess, b->d_step, b->d_blk_sess, b->total_blocks,
                            (uint32_t)b->sched.weight_grid, b->stream);
  if (e == hipSuccess && draw) e = launch_batch_draw(b->d_sess, b->d_step, (uint32_t)b->n, b->stream);
  return e;
}

hipError_t capture_graph(cgs_batch b) {
  drop_graph(b);
  hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  const hipError_t ek = enqueue_batch(b, true);
  e = hipStreamEndCapture(b->stream, &b->graph);
  if (ek != hipSuccess) return ek;
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  return e;
}

cgs_batch_schedule default_schedule(cgs_batch b) {
  cgs_batch_schedule s{};
  s.score_grid = (int32_t)std::min<uint32_t>(std::max<uint32_t>(b->total_tiles, 1), 2048);
  s.weight_grid = (int32_t)std::min<uint32_t>(std::max<uint32_t>(b->total_blocks, 1), 2048);
  s.use_graph = 1;
  return s;
}

std::string batch_key(cgs_batch b) {
  char buf[160];
  snprintf(buf, sizeof buf, "gfx950 n=%d tiles=%u blocks=%u counters=%d", b->n, b->total_tiles,
           b->total_blocks, b->total_counters);
  return buf;
}

} // namespace

extern "C" cgs_status cgs_batch_create(int n, const cgs_session *sessions, const cgs_model *models,
                                       const cgs_batch_schedule *sched, cgs_batch *out) {
  if (!out) return fail(CGS_EINVAL, "NULL out");
  *out = nullptr;
  if (n < 1 || n > 65535 || !sessions || !models) return fail(CGS_EINVAL, "need 1..65535 sessions");
  std::vector<BatchSess> desc(n);
  uint64_t tiles = 0, blocks = 0, valid = 0;
  int counters = 0;
  for (int i = 0; i < n; ++i) {
    cgs_session s = sessions[i];
    cgs_model m = models[i];
    if (!s || !m) return fail(CGS_EINVAL, "NULL session or model %d", i);
    if (m->space != s->space) return fail(CGS_EINVAL, "model %d predicts another space", i);
    const cgs_status st = flush_pending(s);
    if (st != CGS_OK) return st;
    HIP_TRY(hipStreamSynchronize(s->space->stream));
    BatchSess &d = desc[i];
    d.P = m->d_P;
    d.stride = m->stride;
    d.explored = s->d_explored;
    d.s = s->d_s;
    d.bsum = s->d_bsum;
    d.acc = s->d_acc;
    d.idx = s->space->d_idx;
    d.n_valid = (uint32_t)s->space->n_valid;
    d.n_blocks = s->n_blocks;
    d.block_log2 = s->block_log2;
    d.tile0 = (uint32_t)tiles;
    d.blk0 = (uint32_t)blocks;
    d.gamma = s->params.gamma;
    d.w_min = s->params.w_min;
    tiles += (d.n_valid + kBatchTile - 1) / kBatchTile;
    blocks += d.n_blocks;
    valid += d.n_valid;
    counters += m->n_counters;
  }
  if (tiles > 0xffffffffull || blocks > 0xffffffffull)
    return fail(CGS_ERANGE, "batch too large");
  cgs_batch b = new (std::nothrow) cgs_batch_s();
  if (!b) return fail(CGS_ENOMEM, "host allocation");
  b->n = n;
  b->sess.assign(sessions, sessions + n);
  b->models.assign(models, models + n);
  b->total_tiles = (uint32_t)tiles;
  b->total_blocks = (uint32_t)blocks;
  b->total_valid = valid;
  b->total_counters = counters;
  std::vector<uint16_t> tile_sess(std::max<uint64_t>(tiles, 1)), blk_sess(std::max<uint64_t>(blocks, 1));
  for (int i = 0; i < n; ++i) {
    const uint32_t nt = (desc[i].n_valid + kBatchTile - 1) / kBatchTile;
    for (uint32_t t = 0; t < nt; ++t) tile_sess[desc[i].tile0 + t] = (uint16_t)i;
    for (uint32_t t = 0; t < desc[i].n_blocks; ++t) blk_sess[desc[i].blk0 + t] = (uint16_t)i;
  }
  hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = dalloc(&b->d_sess, n);
  if (e == hipSuccess) e = dalloc(&b->d_step, n);
  if (e == hipSuccess) e = dalloc(&b->d_tile_sess, tile_sess.size());
  if (e == hipSuccess) e = dalloc(&b->d_blk_sess, blk_sess.size());
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void **>(&b->h_step), (size_t)n * sizeof(BatchStep), 0);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void **>(&b->h_res), (size_t)n * sizeof(DrawResult),
                      hipHostMallocMapped);
  if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void **>(&b->d_res), b->h_res, 0);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->e0, hipEventDisableSystemFence);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->e1, hipEventDisableSystemFence);
  if (e == hipSuccess) {
    for (int i = 0; i < n; ++i) desc[i].res = b->d_res + i;
    e = hipMemcpyAsync(b->d_sess, desc.data(), (size_t)n * sizeof(BatchSess), hipMemcpyHostToDevice,
                       b->stream);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_tile_sess, tile_sess.data(), tile_sess.size() * sizeof(uint16_t),
                       hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_blk_sess, blk_sess.data(), blk_sess.size() * sizeof(uint16_t),
                       hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    destroy_batch(b);
    return fail(e == hipErrorOutOfMemory ? CGS_ENOMEM : CGS_EDEVICE, "batch buffers: %s",
                hipGetErrorString(e));
  }
  b->sched = sched ? *sched : default_schedule(b);
  if (b->sched.score_grid < 1 || b->sched.weight_grid < 1 || b->sched.variant < 0 ||
      b->sched.variant >= kBatchScoreVariants) {
    destroy_batch(b);
    return fail(CGS_EINVAL, "schedule: grids must be >= 1, variant 0..%d", kBatchScoreVariants - 1);
  }
  if (b->sched.score_grid < 1 || b->sched.weight_grid < 1) {
    const cgs_batch_schedule d = default_schedule(b);
    if (b->sched.score_grid < 1) b->sched.score_grid = d.score_grid;
    if (b->sched.weight_grid < 1) b->sched.weight_grid = d.weight_grid;
  }
  *out = b;
  return CGS_OK;
}

extern "C" cgs_status cgs_batch_set_schedule(cgs_batch b, const cgs_batch_schedule *s) {
  if (!b || !s) return fail(CGS_EINVAL, "NULL argument");
  if (s->score_grid < 1 || s->weight_grid < 1) return fail(CGS_EINVAL, "grids must be >= 1");
  if (s->variant < 0 || s->variant >= kBatchScoreVariants)
    return fail(CGS_EINVAL, "variant %d outside 0..%d", s->variant, kBatchScoreVariants - 1);
  b->sched = *s;
  drop_graph(b);
  return CGS_OK;
}

extern "C" cgs_status cgs_batch_step(cgs_batch b, const uint64_t *profile_raw, const float *deltas,
                                     const uint64_t *u64, uint64_t *raw_out, uint64_t *valid_out,
                                     int32_t *status_out) {
  if (!b || !profile_raw || !u64) return fail(CGS_EINVAL, "NULL argument");
  size_t doff = 0;
  for (int i = 0; i < b->n; ++i) {
    cgs_session s = b->sess[i];
    cgs_model m = b->models[i];
    if (s->pending) {
      const cgs_status st = flush_pending(s);
      if (st != CGS_OK) return st;
      HIP_TRY(hipStreamSynchronize(s->space->stream));
    }
    BatchStep &st = b->h_step[i];
    const int C = m->n_counters;
    st.n_act = 0;
    if (profile_raw[i] == CGS_NO_PROFILE || s->space->n_valid == 0) {
      st.profile = kNoProfile;
    } else {
      const int64_t l = valid_index_of(s->space, profile_raw[i]);
      if (l < 0) return fail(CGS_EINVAL, "session %d: profile is not a valid configuration", i);
      st.profile = (uint32_t)l;
      if (!deltas) return fail(CGS_EINVAL, "deltas needed for profiled sessions");
      for (int c = 0; c < C; ++c) {
        const float d = deltas[doff + c];
        if (!(d >= -1.0f && d <= 1.0f))
          return fail(CGS_EINVAL, "session %d: delta[%d] outside [-1, 1]", i, c);
        if (d != 0.0f) {
          st.ctr[st.n_act] = (uint32_t)c;
          st.delta[st.n_act] = d;
          ++st.n_act;
        }
      }
    }
    doff += (size_t)C;
    st.parity = s->parity;
    st.draw = 1;
    st.u64 = u64[i];
    st.seq = b->seq + 1;
  }
  HIP_TRY(hipEventRecord(b->e0, b->stream));
  if (b->sched.use_graph) {
    if (!b->exec) HIP_TRY(capture_graph(b));
    HIP_TRY(hipGraphLaunch(b->exec, b->stream));
  } else {
    HIP_TRY(enqueue_batch(b, true));
  }
  HIP_TRY(hipEventRecord(b->e1, b->stream));
  ++b->seq;
  HIP_TRY(hipStreamSynchronize(b->stream));
  HIP_TRY(hipEventElapsedTime(&b->last_ms, b->e0, b->e1));
  for (int i = 0; i < b->n; ++i) {
    cgs_session s = b->sess[i];
    // the session now looks as if it had run this step itself
    s->cur_acc = s->parity;
    s->parity ^= 1;
    s->stepped = true;
    s->pending = false;
    s->ran_in_batch = true;
    s->batch_ms = b->last_ms;
    s->n_active = b->h_step[i].n_act;
    DrawResult r;
    std::memcpy(&r, const_cast<const DrawResult *>(static_cast<volatile DrawResult *>(b->h_res + i)),
                sizeof r);
    s->last_total = r.total;
    int32_t status = CGS_OK;
    if (r.total == 0) status = CGS_EEMPTY;
    else if (r.valid == kNoPick) return fail(CGS_EDEVICE, "session %d: no pick although Q > 0", i);
    if (status_out) status_out[i] = status;
    if (raw_out) raw_out[i] = status == CGS_OK ? r.raw : kNoPick;
    if (valid_out) valid_out[i] = status == CGS_OK ? r.valid : kNoPick;
  }
  return CGS_OK;
}

extern "C" cgs_status cgs_batch_step_time(cgs_batch b, float *ms) {
  if (!b || !ms) return fail(CGS_EINVAL, "NULL argument");
  *ms = b->last_ms;
  return CGS_OK;
}

extern "C" cgs_status cgs_batch_autotune(cgs_batch b, const char *cache_path,
                                         cgs_batch_schedule *chosen) {
  if (!b) return fail(CGS_EINVAL, "NULL batch");
  const std::string key = batch_key(b);
  if (cache_path) {
    if (FILE *f = fopen(cache_path, "r")) {
      char line[256];
      while (fgets(line, sizeof line, f)) {
        const char *sep = strstr(line, " -> ");
        if (!sep || std::string(line, sep - line) != key) continue;
        int sg = 0, wg = 0, ug = 1, va = 0;
        const int got = sscanf(sep + 4, "%d %d %d %d", &sg, &wg, &ug, &va);
        if (got >= 3 && sg > 0 && wg > 0 && va >= 0 && va < kBatchScoreVariants) {
          b->sched = cgs_batch_schedule{sg, wg, ug, va};
          drop_graph(b);
          fclose(f);
          if (chosen) *chosen = b->sched;
          return CGS_OK;
        }
      }
      fclose(f);
    }
  }
  // timing records: profile 0, every counter active, no draw; accumulator
  // set = the one the sessions' next step will not use
  for (int i = 0; i < b->n; ++i) {
    cgs_session s = b->sess[i];
    BatchStep &st = b->h_step[i];
    st.profile = s->space->n_valid > 0 ? 0u : kNoProfile;
    st.n_act = b->models[i]->n_counters;
    for (int c = 0; c < st.n_act; ++c) {
      st.ctr[c] = (uint32_t)c;
      st.delta[c] = (c & 1) ? -0.5f : 0.5f;
    }
    st.parity = s->parity ^ 1;
    st.draw = 0;
    st.u64 = 0;
    st.seq = 0;
  }
  HIP_TRY(hipMemcpyAsync(b->d_step, b->h_step, (size_t)b->n * sizeof(BatchStep),
                         hipMemcpyHostToDevice, b->stream));
  // the median of 5 timed runs after one warm-up run, HIP events around
  // the launches on the batch's stream
  auto time_runs = [&](auto &&launch, float &med) -> hipError_t {
    float t[6];
    for (int rep = 0; rep < 6; ++rep) {
      hipError_t e = hipEventRecord(b->e0, b->stream);
      if (e == hipSuccess) e = launch();
      if (e == hipSuccess) e = hipEventRecord(b->e1, b->stream);
      if (e == hipSuccess) e = hipEventSynchronize(b->e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&t[rep], b->e0, b->e1);
      if (e != hipSuccess) return e;
    }
    std::sort(t + 1, t + 6);
    med = t[3];
    return hipSuccess;
  };
  // grid sizes: powers of two up to the work items, and one workgroup per
  // item (no striding)
  const int cand[] = {128, 256, 512, 1024, 2048, 4096, 8192};
  auto grids = [&](uint32_t items) {
    std::vector<int> gs;
    for (int g : cand)
      if ((uint32_t)g < items || g == cand[0]) gs.push_back(g);
    if (items > (uint32_t)cand[0]) gs.push_back((int)std::min<uint32_t>(items, 1u << 20));
    return gs;
  };
  cgs_batch_schedule best = default_schedule(b);
  float best_s = 1e30f, best_w = 1e30f;
  // score pass: every variant at every grid size
  for (int v = 0; v < kBatchScoreVariants; ++v) {
    for (int g : grids(b->total_tiles)) {
      float t = 0.0f;
      HIP_TRY(time_runs(
          [&] {
            return launch_batch_score(b->d_sess, b->d_step, b->d_tile_sess, b->total_tiles,
                                      (uint32_t)g, v, b->stream);
          },
          t));
      if (t < best_s) {
        best_s = t;
        best.score_grid = g;
        best.variant = v;
      }
    }
  }
  for (int g : grids(b->total_blocks)) {
    float t = 0.0f;
    HIP_TRY(time_runs(
        [&] {
          return launch_batch_weight(b->d_sess, b->d_step, b->d_blk_sess, b->total_blocks,
                                     (uint32_t)g, b->stream);
        },
        t));
    if (t < best_w) {
      best_w = t;
      best.weight_grid = g;
    }
  }
  // graph or plain launches: the step's copy, score and weight passes (no
  // draw) either way
  float t_plain = 0.0f, t_graph = 1e30f;
  auto step_launches = [&]() -> hipError_t {
    hipError_t e = hipMemcpyAsync(b->d_step, b->h_step, (size_t)b->n * sizeof(BatchStep),
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
      e = launch_batch_score(b->d_sess, b->d_step, b->d_tile_sess, b->total_tiles,
                             (uint32_t)best.score_grid, best.variant, b->stream);
    if (e == hipSuccess)
      e = launch_batch_weight(b->d_sess, b->d_step, b->d_blk_sess, b->total_blocks,
                              (uint32_t)best.weight_grid, b->stream);
    return e;
  };
  HIP_TRY(time_runs(step_launches, t_plain));
  {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      const hipError_t ek = step_launches();
      e = hipStreamEndCapture(b->stream, &g);
      if (e == hipSuccess) e = ek;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e == hipSuccess) e = time_runs([&] { return hipGraphLaunch(ge, b->stream); }, t_graph);
    if (ge) hipGraphExecDestroy(ge);
    if (g) hipGraphDestroy(g);
    HIP_TRY(e);
  }
  best.use_graph = t_graph <= t_plain ? 1 : 0;
  b->sched = best;
  drop_graph(b);
  // the sessions' last-step results were overwritten
  for (cgs_session s : b->sess) s->stepped = false;
  if (cache_path) {
    if (FILE *f = fopen(cache_path, "a")) {
      fprintf(f, "%s -> %d %d %d %d\n", key.c_str(), best.score_grid, best.weight_grid,
              best.use_graph, best.variant);
      fclose(f);
    }
  }
  if (chosen) *chosen = best;
  return CGS_OK;
}

extern "C" cgs_status cgs_batch_draw(cgs_batch b, const uint64_t *u64, uint64_t *raw_out,
                                     uint64_t *valid_out, int32_t *status_out) {
  if (!b || !u64) return fail(CGS_EINVAL, "NULL argument");
  for (int i = 0; i < b->n; ++i) {
    cgs_session s = b->sess[i];
    // the session must still hold the weights of the batch's last step
    if (!s->stepped || !s->ran_in_batch || s->pending || s->cur_acc != b->h_step[i].parity)
      return fail(CGS_ESTATE, "session %d: no batch step to draw from", i);
    BatchStep &st = b->h_step[i];
    st.draw = 1;
    st.u64 = u64[i];
    st.seq = b->seq + 1;
  }
  HIP_TRY(hipMemcpyAsync(b->d_step, b->h_step, (size_t)b->n * sizeof(BatchStep),
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(launch_batch_draw(b->d_sess, b->d_step, (uint32_t)b->n, b->stream));
  ++b->seq;
  HIP_TRY(hipStreamSynchronize(b->stream));
  for (int i = 0; i < b->n; ++i) {
    DrawResult r;
    std::memcpy(&r, const_cast<const DrawResult *>(static_cast<volatile DrawResult *>(b->h_res + i)),
                sizeof r);
    b->sess[i]->last_total = r.total;
    int32_t status = CGS_OK;
    if (r.total == 0) status = CGS_EEMPTY;
    else if (r.valid == kNoPick) return fail(CGS_EDEVICE, "session %d: no pick although Q > 0", i);
    if (status_out) status_out[i] = status;
    if (raw_out) raw_out[i] = status == CGS_OK ? r.raw : kNoPick;
    if (valid_out) valid_out[i] = status == CGS_OK ? r.valid : kNoPick;
  }
  return CGS_OK;
}

// Alg. 1 for every session of a batch at once.  Each run follows exactly the
// steps of cgs_tuning_run with its own random numbers; the runs advance in
// lockstep (one batch step, then batched draws), and a run that has ended
// keeps stepping with no profile while its results are ignored.
extern "C" cgs_status cgs_tuning_run_batch(cgs_batch b, const float *runtime,
                                           const double *counters,
                                           const cgs_expert_params *expert,
                                           const uint64_t *uniforms, uint64_t n_uniforms,
                                           const cgs_tuning_opts *opts, uint64_t capacity,
                                           uint64_t *tested, uint8_t *profiled,
                                           uint64_t *n_tests, uint64_t *tests_to_well) {
  if (!b || !runtime || !counters || !uniforms || !opts || !n_tests || !tests_to_well ||
      (capacity && !tested))
    return fail(CGS_EINVAL, "NULL argument");
  const int n = b->n;
  cgs_space sp = b->sess[0]->space;
  for (int i = 0; i < n; ++i) {
    n_tests[i] = 0;
    tests_to_well[i] = 0;
    if (b->sess[i]->space != sp) return fail(CGS_EINVAL, "the runs must share one space");
    if (b->models[i]->n_counters != 24)
      return fail(CGS_EINVAL, "the loop needs models of the 24 counters");
  }
  if (opts->draws < 1) return fail(CGS_ERANGE, "draws %d < 1", opts->draws);
  if (opts->max_tests < 1 || opts->max_tests > capacity)
    return fail(CGS_ERANGE, "max_tests must be 1..capacity");
  const uint64_t nv = sp->n_valid;
  if (nv == 0) return fail(CGS_EEMPTY, "the space has no valid configuration");
  float rmin = runtime[0];
  for (uint64_t l = 1; l < nv; ++l) rmin = std::min(rmin, runtime[l]);
  const double thresh = opts->well_factor * (double)rmin;

  struct Run {
    uint64_t u = 0, c = 0, nt = 0, found = 0, next_c = 0;
    float best = INFINITY;
    bool active = true, drawing = false, stop = false, next = false;
  };
  std::vector<Run> run(n);
  std::vector<uint64_t> prof(n), u64(n), valid(n);
  std::vector<int32_t> status(n);
  std::vector<float> deltas((size_t)n * 24);
  auto test = [&](int i, uint64_t l, bool p) {
    Run &r = run[i];
    tested[(uint64_t)i * capacity + r.nt] = l;
    if (profiled) profiled[(uint64_t)i * capacity + r.nt] = p ? 1 : 0;
    ++r.nt;
    if (!r.found && (double)runtime[l] <= thresh) r.found = r.nt;
    return (opts->stop_at_well && r.found) || r.nt >= opts->max_tests;
  };
  auto take_uniform = [&](int i, uint64_t *out) -> cgs_status { // run i's next number
    Run &r = run[i];
    if (r.u >= n_uniforms)
      return fail(CGS_ERANGE, "run %d needs more than %llu random numbers", i,
                  (unsigned long long)n_uniforms);
    *out = uniforms[(uint64_t)i * n_uniforms + r.u++];
    return CGS_OK;
  };
  auto finish = [&]() {
    for (int i = 0; i < n; ++i) {
      n_tests[i] = run[i].nt;
      tests_to_well[i] = run[i].found;
    }
  };

  // Slot j of the current batch runs run[map[j]]; per-slot arrays below.
  // Once half of a batch's runs have ended, the live ones move to a new,
  // smaller batch (built from the same sessions and models) between
  // iterations, so finished runs stop costing score passes.
  cgs_batch cur = b, own = nullptr;
  std::vector<int> map(n);
  for (int i = 0; i < n; ++i) map[i] = i;
  auto release = [&](cgs_status st) {
    if (own) cgs_batch_destroy(own);
    if (st == CGS_OK) finish();
    return st;
  };

  // uniform start: the first draw of every run
  for (int i = 0; i < n; ++i) {
    prof[i] = CGS_NO_PROFILE;
    const cgs_status st = take_uniform(i, &u64[i]);
    if (st != CGS_OK) return st;
  }
  cgs_status st = cgs_batch_step(b, prof.data(), nullptr, u64.data(), nullptr, valid.data(),
                                 status.data());
  if (st != CGS_OK) return st;
  int n_active = 0;
  for (int i = 0; i < n; ++i) {
    run[i].active = status[i] == CGS_OK;
    run[i].c = valid[i];
    n_active += run[i].active;
  }
  while (n_active > 0) {
    const int m = cur->n;
    // profile the current configurations
    for (int j = 0; j < m; ++j) {
      const int i = map[j];
      Run &r = run[i];
      prof[j] = CGS_NO_PROFILE;
      u64[j] = 0;
      std::fill(deltas.begin() + (size_t)j * 24, deltas.begin() + (size_t)j * 24 + 24, 0.0f);
      if (!r.active) continue;
      if (test(i, r.c, true)) {
        r.active = false;
        --n_active;
        continue;
      }
      double bn[18], d[24];
      st = cgs_expert_system(counters + r.c * 24, expert, bn, d, nullptr);
      if (st != CGS_OK) return release(fail(st, "run %d: expert system rejected the counters", i));
      for (int c = 0; c < 24; ++c) deltas[(size_t)j * 24 + c] = (float)d[c];
      prof[j] = sp->h_idx[r.c];
      st = take_uniform(i, &u64[j]);
      if (st != CGS_OK) return release(st);
      r.best = INFINITY;
      r.next = false;
      r.stop = false;
      r.drawing = true;
    }
    if (n_active == 0) break;
    // the scored step and its first draw, then the further draws
    st = cgs_batch_step(cur, prof.data(), deltas.data(), u64.data(), nullptr, valid.data(),
                        status.data());
    for (int k = 0; st == CGS_OK; ++k) {
      bool more = false;
      for (int j = 0; j < m; ++j) {
        Run &r = run[map[j]];
        if (!r.active || !r.drawing) continue;
        if (status[j] != CGS_OK) { // no configuration left
          r.drawing = false;
          continue;
        }
        const uint64_t l = valid[j];
        if (test(map[j], l, false)) {
          r.stop = true;
          r.drawing = false;
          continue;
        }
        if (runtime[l] <= r.best) {
          r.best = runtime[l];
          r.next_c = l;
          r.next = true;
        }
        if (k + 1 < opts->draws) more = true;
        else r.drawing = false;
      }
      if (!more) break;
      for (int j = 0; j < m; ++j) {
        const int i = map[j];
        u64[j] = 0;
        if (run[i].active && run[i].drawing) {
          st = take_uniform(i, &u64[j]);
          if (st != CGS_OK) return release(st);
        }
      }
      st = cgs_batch_draw(cur, u64.data(), nullptr, valid.data(), status.data());
    }
    if (st != CGS_OK) return release(st);
    for (int j = 0; j < m; ++j) {
      Run &r = run[map[j]];
      if (!r.active) continue;
      if (r.stop || !r.next) {
        r.active = false;
        --n_active;
      } else {
        r.c = r.next_c;
      }
    }
    if (n_active > 0 && 2 * n_active <= m && m >= 4) {
      std::vector<cgs_session> ss;
      std::vector<cgs_model> ms;
      std::vector<int> keep;
      for (int j = 0; j < m; ++j)
        if (run[map[j]].active) {
          keep.push_back(map[j]);
          ss.push_back(cur->sess[j]);
          ms.push_back(cur->models[j]);
        }
      cgs_batch nb = nullptr;
      st = cgs_batch_create((int)ss.size(), ss.data(), ms.data(), nullptr, &nb);
      if (st != CGS_OK) return release(st);
      if (own) cgs_batch_destroy(own);
      own = cur = nb;
      map = keep;
    }
  }
  return release(CGS_OK);
}

extern "C" void cgs_batch_destroy(cgs_batch b) { destroy_batch(b); }

// ------------------------------------------------------- standalone sampler
namespace {

// n_draws draws with removal over the weights d_q[n] (a device working copy,
// zeroed where picked) with block sums d_bsum[n_blocks] (2^lg weights per
// block); the draws of cgs_sample_weights and cgs_sample_weights_noalloc.
cgs_status sample_resident(cgs_space sp, uint32_t *d_q, uint64_t n, int lg, uint64_t *d_bsum,
                           uint32_t n_blocks, const uint64_t *u64, int n_draws, int64_t *picks) {
  hipError_t e = launch_array_block_sums(d_q, (uint32_t)n, lg, d_bsum, sp->stream);
  for (int i = 0; i < n_draws && e == hipSuccess; ++i) {
    e = launch_array_draw(d_q, (uint32_t)n, lg, d_bsum, n_blocks, u64[i], sp->d_res, sp->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(sp->stream);
    if (e == hipSuccess) {
      if (sp->h_res->total == 0) break;
      if (sp->h_res->valid == kNoPick) return fail(CGS_EDEVICE, "draw found no index although Q > 0");
      picks[i] = (int64_t)sp->h_res->valid;
    }
  }
  if (e != hipSuccess) return fail(CGS_EDEVICE, "sampler: %s", hipGetErrorString(e));
  return CGS_OK;
}

cgs_status sample_args(cgs_space sp, const uint32_t *q, uint64_t n, const uint64_t *u64,
                       int n_draws, int64_t *picks) {
  if (!sp || (!q && n) || (!u64 && n_draws) || (!picks && n_draws))
    return fail(CGS_EINVAL, "NULL argument");
  if (n > 0xffffffffull) return fail(CGS_ERANGE, "more than 2^32 - 1 weights");
  if (n_draws < 0) return fail(CGS_EINVAL, "negative n_draws");
  for (int i = 0; i < n_draws; ++i) picks[i] = -1;
  return CGS_OK;
}

} // namespace

extern "C" cgs_status cgs_sample_weights(cgs_space sp, const uint32_t *q, uint64_t n,
                                         const uint64_t *u64, int n_draws, int64_t *picks) {
  const cgs_status st = sample_args(sp, q, n, u64, n_draws, picks);
  if (st != CGS_OK || n == 0 || n_draws == 0) return st;
  const int lg = auto_block_log2(n);
  const uint32_t n_blocks = (uint32_t)((n + (1ull << lg) - 1) >> lg);
  uint32_t *d_q = nullptr;
  uint64_t *d_bsum = nullptr;
  HIP_TRY(dalloc(&d_q, n));
  hipError_t e = dalloc(&d_bsum, n_blocks);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_q, q, n * sizeof(uint32_t), hipMemcpyHostToDevice, sp->stream);
  cgs_status r = e == hipSuccess ? sample_resident(sp, d_q, n, lg, d_bsum, n_blocks, u64, n_draws, picks)
                                 : fail(CGS_EDEVICE, "sampler: %s", hipGetErrorString(e));
  dfree(d_q);
  dfree(d_bsum);
  return r;
}

// ------------------------------------------- the sampler without allocation
// Device memory of cgs_sample_weights_noalloc: the working copy of the
// weights (a draw zeroes what it picks) from byte 0, the block sums from
// byte kNoAllocBsumOffset.  Every GPU the library runs on holds its own
// copy of the array until the process ends.  Host code never hands the
// array's name to a kernel or a copy (on the host it is only a stand-in for
// the symbol); it uses the device address hipGetSymbolAddress gives for
// the stream's device, fetched once per device.
constexpr uint64_t kNoAllocMaxWeights = 1ull << 22;
constexpr uint64_t kNoAllocBsumOffset = kNoAllocMaxWeights * sizeof(uint32_t);
constexpr uint64_t kNoAllocMaxBlocks = 1024; // 2^22 weights in blocks of 2^12
constexpr uint64_t kNoAllocBytes = kNoAllocBsumOffset + kNoAllocMaxBlocks * sizeof(uint64_t);
static_assert(kNoAllocBsumOffset % 256 == 0, "block sums stay 256-byte aligned");

static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on device dev (looked up on first use
// with dev current; the caller's current device is restored).
hipError_t scratch_on(int dev, uint8_t **out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess && prev != dev) e = hipSetDevice(dev);
    void *ptr = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (prev >= 0 && prev != dev) {
      const hipError_t e2 = hipSetDevice(prev);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<uint8_t *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

} // namespace

extern "C" cgs_status cgs_sample_weights_noalloc(cgs_space sp, const uint32_t *q, uint64_t n,
                                                 const uint64_t *u64, int n_draws,
                                                 int64_t *picks) {
  const cgs_status st = sample_args(sp, q, n, u64, n_draws, picks);
  if (st != CGS_OK) return st;
  if (n > kNoAllocMaxWeights)
    return fail(CGS_ERANGE, "cgs_sample_weights_noalloc takes at most %llu weights, got %llu",
                (unsigned long long)kNoAllocMaxWeights, (unsigned long long)n);
  if (n == 0 || n_draws == 0) return CGS_OK;
  const int lg = auto_block_log2(n);
  const uint32_t n_blocks = (uint32_t)((n + (1ull << lg) - 1) >> lg);
  if (n_blocks > kNoAllocMaxBlocks)
    return fail(CGS_ERANGE, "%u weight blocks exceed the %llu the array holds", n_blocks,
                (unsigned long long)kNoAllocMaxBlocks);
  int dev = -1;
  hipError_t e = hipStreamGetDevice(sp->stream, &dev);
  uint8_t *base = nullptr;
  if (e == hipSuccess) e = scratch_on(dev, &base);
  if (e != hipSuccess) return fail(CGS_EDEVICE, "sampler scratch: %s", hipGetErrorString(e));
  uint32_t *d_q = reinterpret_cast<uint32_t *>(base);
  uint64_t *d_bsum = reinterpret_cast<uint64_t *>(base + kNoAllocBsumOffset);
  // every weight and block sum the draws read is written here first
  e = hipMemcpyAsync(d_q, q, n * sizeof(uint32_t), hipMemcpyHostToDevice, sp->stream);
  if (e != hipSuccess) return fail(CGS_EDEVICE, "sampler: %s", hipGetErrorString(e));
  return sample_resident(sp, d_q, n, lg, d_bsum, n_blocks, u64, n_draws, picks);
}
