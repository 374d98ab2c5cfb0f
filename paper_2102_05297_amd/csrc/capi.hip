// Host runtime of libcgs: argument validation, device buffers, kernel
// sequencing and the extern "C" entry points declared in include/cgs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cgs.h"
#include "internal.h"

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
  std::vector<uint32_t> h_idx; // valid raw indices, for raw -> valid lookups
  // scratch for the standalone sampler
  DrawResult *d_res = nullptr;
  DrawResult *h_res = nullptr;
};

struct cgs_model_s {
  cgs_space space = nullptr;
  int kind = 0; // 0 = forest
  int n_counters = 0;
  int n_trees = 0, depth = 0;
  uint16_t *d_nodes = nullptr;
  float *d_leaves = nullptr;
  float *d_P = nullptr;
  uint64_t stride = 0;
  float eval_ms = 0.0f;
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
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;
  // timing mode: [0] before score, [1] after score, [2] after weights + first
  // draw, [3] before a further draw, [4] after it
  hipEvent_t ev_k[5] = {};
  bool step_times_pending = false;
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
  int n_active = 0;
  uint64_t last_total = 0;
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
namespace {

FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  const uint64_t m = ((((uint64_t)1 << l) - d) << 32) / d + 1;
  const uint32_t sh1 = l < 1 ? l : 1, sh2 = l > 1 ? l - 1 : 0;
  return FastDiv{(uint32_t)m, sh1 | (sh2 << 8)};
}

void destroy_space(cgs_space sp) {
  if (!sp) return;
  if (--sp->refs > 0) return;
  if (sp->stream) (void)hipStreamSynchronize(sp->stream);
  dfree(sp->d_desc);
  dfree(sp->d_mask);
  dfree(sp->d_idx);
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
                           d_total, nullptr, 0, sp->stream);
  uint64_t n_valid = 0;
  if (e == hipSuccess)
    e = hipMemcpyAsync(&n_valid, d_total, sizeof(uint64_t), hipMemcpyDeviceToHost, sp->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(sp->stream);
  if (e == hipSuccess) e = dalloc(&sp->d_idx, n_valid);
  if (e == hipSuccess && n_valid > 0)
    e = launch_enumeration(sp->d_desc, (uint32_t)n_raw, sp->d_mask, d_tile_count, d_tile_off,
                           d_total, sp->d_idx, 1, sp->stream);
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

void destroy_model(cgs_model m) {
  if (!m) return;
  if (m->space && m->space->stream) (void)hipStreamSynchronize(m->space->stream);
  dfree(m->d_nodes);
  dfree(m->d_leaves);
  dfree(m->d_P);
  destroy_space(m->space);
  delete m;
}

cgs_status evaluate_model(cgs_model m) {
  cgs_space sp = m->space;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, sp->stream));
  hipError_t e = launch_forest_eval(sp->d_desc, sp->d_idx, (uint32_t)sp->n_valid, m->d_nodes,
                                    m->d_leaves, m->n_trees, m->depth, m->n_counters, m->d_P,
                                    m->stride, nullptr, 0, 0, sp->stream);
  if (e == hipSuccess) e = hipEventRecord(e1, sp->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(CGS_EDEVICE, "forest evaluation: %s", hipGetErrorString(e));
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
    if (!std::isfinite(leaves[i])) return fail(CGS_EINVAL, "leaf value %zu is not finite", i);

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
  if (s->h_res) (void)hipHostFree(s->h_res);
  if (s->h_acc) (void)hipHostFree(s->h_acc);
  if (s->ev_begin) (void)hipEventDestroy(s->ev_begin);
  if (s->ev_end) (void)hipEventDestroy(s->ev_end);
  for (hipEvent_t &ev : s->ev_k)
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

// Adds the score / weight times of the last launched step.
hipError_t collect_step_times(cgs_session s) {
  hipError_t e = hipEventSynchronize(s->ev_k[2]);
  float ms[2] = {0, 0};
  for (int i = 0; i < 2 && e == hipSuccess; ++i)
    e = hipEventElapsedTime(&ms[i], s->ev_k[i], s->ev_k[i + 1]);
  if (e != hipSuccess) return e;
  s->kernel_ms[0] += ms[0];
  s->kernel_ms[1] += ms[1];
  s->kernel_n[0] += 1;
  s->kernel_n[1] += 1;
  s->step_times_pending = false;
  return hipSuccess;
}

// Enqueues the recorded step: score pass, weight pass, and either its first
// draw (do_draw) or just the marking of its profiled configuration.
hipError_t launch_pending(cgs_session s, bool do_draw, uint64_t u64) {
  cgs_space sp = s->space;
  cgs_model m = s->pending_model;
  const uint32_t nv = (uint32_t)sp->n_valid;
  const bool timing = s->params.timing != 0;
  hipError_t e = hipSuccess;
  if (timing && s->step_times_pending) e = collect_step_times(s);
  StepAcc *acc = s->d_acc + s->parity * kAccSlots;
  StepAcc *acc_next = s->d_acc + (s->parity ^ 1) * kAccSlots;
  const uint32_t prof = s->pending_profile;
  if (e == hipSuccess) e = hipEventRecord(s->ev_begin, sp->stream);
  if (e == hipSuccess && timing) e = hipEventRecord(s->ev_k[0], sp->stream);
  if (e == hipSuccess)
    e = launch_score_pass(m->d_P, m->stride, prof, s->pending_act, s->d_explored, nv, s->d_s, acc,
                          sp->stream);
  if (e == hipSuccess && timing) e = hipEventRecord(s->ev_k[1], sp->stream);
  if (e == hipSuccess)
    e = launch_weight_pass(s->d_s, s->d_explored, nv, prof, acc, acc_next, s->params.gamma,
                           s->params.w_min, s->block_log2, s->d_bsum, s->n_blocks, sp->stream);
  if (e == hipSuccess && timing) e = hipEventRecord(s->ev_k[2], sp->stream);
  if (e == hipSuccess && do_draw && timing) e = hipEventRecord(s->ev_k[3], sp->stream);
  if (e == hipSuccess) {
    if (do_draw)
      e = launch_draw(s->d_s, s->d_explored, nv, prof, true, acc, s->params.gamma, s->params.w_min,
                      s->block_log2, s->d_bsum, s->n_blocks, u64, sp->d_idx, s->d_res,
                      sp->stream);
    else
      e = launch_mark_one(s->d_explored, prof, nv, sp->stream);
  }
  if (e == hipSuccess && do_draw && timing) e = hipEventRecord(s->ev_k[4], sp->stream);
  if (e == hipSuccess) e = hipEventRecord(s->ev_end, sp->stream);
  if (e != hipSuccess) return e;
  s->step_times_pending = timing;
  s->cur_acc = s->parity;
  s->parity ^= 1;
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
  if (s->params.timing && s->step_times_pending) HIP_TRY(collect_step_times(s));
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
    e = hipHostMalloc(reinterpret_cast<void **>(&s->h_res), sizeof(DrawResult), hipHostMallocMapped);
  if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void **>(&s->d_res), s->h_res, 0);
  if (e == hipSuccess)
    e = hipHostMalloc(reinterpret_cast<void **>(&s->h_acc), kAccSlots * sizeof(StepAcc), 0);
  if (e == hipSuccess) e = hipEventCreate(&s->ev_begin);
  if (e == hipSuccess) e = hipEventCreate(&s->ev_end);
  for (int i = 0; i < 5 && e == hipSuccess && p.timing; ++i) e = hipEventCreate(&s->ev_k[i]);
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

extern "C" cgs_status cgs_search_step(cgs_session s, cgs_model m, uint64_t profile_raw,
                                      const float *delta, const double *measured,
                                      const cgs_expert_params *expert) {
  if (!s || !m) return fail(CGS_EINVAL, "NULL session or model");
  cgs_space sp = s->space;
  if (m->space != sp) return fail(CGS_EINVAL, "model and session belong to different spaces");
  const int C = m->n_counters;
  const bool no_profile = profile_raw == CGS_NO_PROFILE;
  const int64_t prof = no_profile ? 0 : valid_index_of(sp, profile_raw);
  if (prof < 0)
    return fail(CGS_EINVAL, "profile %llu is not a valid configuration",
                (unsigned long long)profile_raw);
  if (sp->n_valid == 0) return fail(CGS_EEMPTY, "the space has no valid configuration");
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
  // a step recorded but never drawn from still marks its profile and scores
  const cgs_status st = flush_pending(s);
  if (st != CGS_OK) return st;
  ActiveCounters act{};
  for (int c = 0; c < C; ++c)
    if (dpc[c] != 0.0f) {
      act.ctr[act.n] = (uint32_t)c;
      act.delta[act.n] = dpc[c];
      ++act.n;
    }
  s->pending = true;
  s->pending_model = m;
  s->pending_profile = no_profile ? kNoProfile : (uint32_t)prof;
  s->pending_act = act;
  s->stepped = true;
  s->n_active = act.n;
  s->last_total = 0;
  return CGS_OK;
}

extern "C" cgs_status cgs_sample_next(cgs_session s, uint64_t u64, uint64_t *raw_out,
                                      uint64_t *valid_out) {
  if (!s) return fail(CGS_EINVAL, "NULL session");
  if (!s->stepped) return fail(CGS_ESTATE, "cgs_sample_next before any cgs_search_step");
  cgs_space sp = s->space;
  if (sp->n_valid == 0) return fail(CGS_EEMPTY, "the space has no valid configuration");
  const bool timing = s->params.timing != 0;
  if (s->pending) {
    HIP_TRY(launch_pending(s, true, u64));
  } else {
    if (timing) HIP_TRY(hipEventRecord(s->ev_k[3], sp->stream));
    HIP_TRY(launch_draw(s->d_s, s->d_explored, (uint32_t)sp->n_valid, kNoProfile, false,
                        s->d_acc + s->cur_acc * kAccSlots, s->params.gamma, s->params.w_min,
                        s->block_log2, s->d_bsum, s->n_blocks, u64, sp->d_idx, s->d_res,
                        sp->stream));
    if (timing) HIP_TRY(hipEventRecord(s->ev_k[4], sp->stream));
    HIP_TRY(hipEventRecord(s->ev_end, sp->stream));
  }
  HIP_TRY(hipStreamSynchronize(sp->stream));
  if (timing) {
    if (s->step_times_pending) HIP_TRY(collect_step_times(s));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, s->ev_k[3], s->ev_k[4]));
    s->kernel_ms[2] += ms;
    s->kernel_n[2] += 1;
  }
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
  HIP_TRY(hipMemcpyAsync(s->h_acc, s->d_acc + s->cur_acc * kAccSlots, kAccSlots * sizeof(StepAcc),
                         hipMemcpyDeviceToHost, sp->stream));
  HIP_TRY(hipStreamSynchronize(sp->stream));
  StepAccSums a{0xffffffffu, 0u, 0u};
  for (int i = 0; i < kAccSlots; ++i) {
    a.min_key = std::min(a.min_key, s->h_acc[i].min_key);
    a.max_key = std::max(a.max_key, s->h_acc[i].max_key);
    a.n_unexplored += s->h_acc[i].n_unexplored;
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
  HIP_TRY(hipEventElapsedTime(&ms, s->ev_begin, s->ev_end));
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

// ------------------------------------------------------- standalone sampler
extern "C" cgs_status cgs_sample_weights(cgs_space sp, const uint32_t *q, uint64_t n,
                                         const uint64_t *u64, int n_draws, int64_t *picks) {
  if (!sp || (!q && n) || (!u64 && n_draws) || (!picks && n_draws))
    return fail(CGS_EINVAL, "NULL argument");
  if (n > 0xffffffffull) return fail(CGS_ERANGE, "more than 2^32 - 1 weights");
  if (n_draws < 0) return fail(CGS_EINVAL, "negative n_draws");
  for (int i = 0; i < n_draws; ++i) picks[i] = -1;
  if (n == 0 || n_draws == 0) return CGS_OK;
  const int lg = auto_block_log2(n);
  const uint32_t n_blocks = (uint32_t)((n + (1ull << lg) - 1) >> lg);
  uint32_t *d_q = nullptr;
  uint64_t *d_bsum = nullptr;
  HIP_TRY(dalloc(&d_q, n));
  hipError_t e = dalloc(&d_bsum, n_blocks);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_q, q, n * sizeof(uint32_t), hipMemcpyHostToDevice, sp->stream);
  if (e == hipSuccess) e = launch_array_block_sums(d_q, (uint32_t)n, lg, d_bsum, sp->stream);
  for (int i = 0; i < n_draws && e == hipSuccess; ++i) {
    e = launch_array_draw(d_q, (uint32_t)n, lg, d_bsum, n_blocks, u64[i], sp->d_res, sp->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(sp->stream);
    if (e == hipSuccess) {
      if (sp->h_res->total == 0) break;
      if (sp->h_res->valid == kNoPick) {
        dfree(d_q);
        dfree(d_bsum);
        return fail(CGS_EDEVICE, "draw found no index although Q > 0");
      }
      picks[i] = (int64_t)sp->h_res->valid;
    }
  }
  dfree(d_q);
  dfree(d_bsum);
  if (e != hipSuccess) return fail(CGS_EDEVICE, "sampler: %s", hipGetErrorString(e));
  return CGS_OK;
}
