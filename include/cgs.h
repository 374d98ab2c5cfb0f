/*
 * cgs.h - counter-guided search sweep on one AMD Instinct MI355X (gfx950).
 *
 * C ABI of the data-parallel hot path of the profile-based autotuning
 * searcher of Filipovic et al., "Using hardware performance counters to
 * speed up autotuning convergence on GPUs":
 *
 *   space    the tuning space: cross product of per-parameter value sets,
 *            pruned by a-priori constraints (Sect. 1; the array TS of Alg. 1)
 *   model    a problem-specific model predicting each configuration's
 *            counter vector (Sect. 3.4: decision tree; here also a forest and
 *            a multilayer-perceptron surrogate)
 *   session  the state of one search: explored configurations, scores,
 *            weights (Sect. 3.6 and Alg. 1)
 *   step     score every unexplored configuration against the profiled one
 *            (Sect. 3.6, score and score-normalisation equations)
 *   sample   draw the next configuration with probability proportional to
 *            its normalised score, then zero that score (Sect. 3.7, Alg. 1)
 *
 * Conventions, for every entry point:
 *   - Pointers named *_host are caller-owned host arrays, read (or written)
 *     before the call returns; the library keeps no reference to them.
 *   - Handles own their device memory (hipMalloc on the current device) and
 *     free it in *_destroy.  *_destroy accepts NULL.  Models and sessions
 *     hold a reference to their space, so handles may be destroyed in any
 *     order.
 *   - Work runs on the HIP stream given at space creation (NULL: the library
 *     creates one, default priority).  Every handle derived from a space uses
 *     that stream.  Calls that return device results to the host
 *     synchronise that stream; others only enqueue.
 *   - A handle is not thread-safe: one host thread at a time.
 *   - No C++ exception crosses this ABI.  A non-zero status comes with a
 *     message from cgs_last_error() (thread-local, valid until the next call
 *     on that thread).
 *   - Configurations are named by their raw index k in the mixed-radix
 *     numbering of the cross product, parameter 0 most significant, or by
 *     their valid index l: the position of k in the ascending list of valid
 *     raw indices.
 */
#ifndef CGS_H
#define CGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cgs_space_s *cgs_space;
typedef struct cgs_model_s *cgs_model;
typedef struct cgs_session_s *cgs_session;

typedef enum {
  CGS_OK = 0,
  CGS_EINVAL = -1,  /* malformed argument                                 */
  CGS_ENOMEM = -2,  /* device or host allocation failed                   */
  CGS_EDEVICE = -3, /* HIP runtime error (message names the call)         */
  CGS_EEMPTY = -4,  /* no unexplored valid configuration is left          */
  CGS_ESTATE = -5,  /* call out of order (e.g. sample before any step)    */
  CGS_ERANGE = -6   /* a size exceeds a documented limit                  */
} cgs_status;

/* Limits (CGS_ERANGE beyond them). */
#define CGS_MAX_PARAMS 32           /* tuning parameters per space             */
#define CGS_MAX_RADIX 16            /* values per parameter                    */
#define CGS_MAX_ABS_VALUE (1 << 20) /* |parameter value| must stay below this  */
#define CGS_MAX_CONSTRAINTS 32
#define CGS_MAX_COUNTERS 64         /* counters per model                      */
#define CGS_MAX_TREES 64
#define CGS_MAX_DEPTH 14
#define CGS_MAX_RADIUS 3            /* neighbourhood radius of a restricted step */
#define CGS_MAX_NEIGHBOURS 65536    /* neighbours of one restricted step        */
/* raw space size: at most 2^32 - 1 configurations */

/* Constraint kinds, over parameter values v[] of one configuration.
 * A divisibility test by a zero value fails. */
enum {
  CGS_DIV = 0,      /* v[a] % v[b] == 0          */
  CGS_DIV2 = 1,     /* v[a] % (v[b] * v[c]) == 0 */
  CGS_PROD_LE = 2,  /* v[a] * v[b] <= bound      */
  CGS_PROD3_LE = 3, /* v[a] * v[b] * v[c] <= bound */
  CGS_PROD_GE = 4,  /* v[a] * v[b] >= bound      */
  CGS_LE = 5        /* v[a] <= v[b]              */
};

typedef struct {
  int32_t kind;  /* CGS_DIV ... CGS_LE                     */
  int32_t a, b, c; /* parameter indices (unused ones: 0)  */
  int64_t bound;
} cgs_constraint;

/* Search constants; cgs_default_params() gives the paper's values
 * (Sect. 3.6: cut-off gamma = -0.25, weights in [1e-4, 256]). */
typedef struct {
  float gamma;       /* scores <= gamma get weight w_min                    */
  float w_min;       /* smallest weight of an unexplored configuration      */
  int32_t block_log2; /* configurations per weight block = 2^block_log2,
                          12..20; 0 = automatic                              */
  int32_t timing;     /* k > 0: time the kernels of every k-th step (steps
                         0, k, 2k, ... in launch order, with any further
                         draws of those steps) with HIP events; each timed
                         step pays a few microseconds for its event markers
                         (cgs_session_kernel_times); 0: no timing           */
} cgs_params;

/* Expert-system settings (Sect. 3.5). */
typedef struct {
  double inst_reaction; /* 0.7, or 0.5 for problems known to be compute-bound */
  int32_t volta;        /* counters from a Volta-or-newer GPU: L2_U is a
                           percentage and issue utilisation saturates at 50  */
  int32_t reserved;
  double cores;         /* CUDA cores of the profiled GPU                     */
  double threads;       /* threads of the profiled launch                     */
} cgs_expert_params;

/* Results of the last search step.  Filled by cgs_session_step_info(). */
typedef struct {
  uint64_t n_unexplored; /* valid configurations not yet explored          */
  uint64_t total_weight; /* Q: sum of quantised weights at the last draw   */
  float s_min, s_max;    /* extreme scores over unexplored configurations */
  float device_ms;       /* device time from the score pass to the end of the
                            first draw of the last timed step (hipEvents); the
                            batch step's time for a step run in a batch; 0
                            without timing                                  */
  int32_t n_active;      /* counters that entered the score               */
} cgs_step_info;

/* ---------------------------------------------------------------- misc */
const char *cgs_last_error(void);
int cgs_version(void);
void cgs_default_params(cgs_params *out);
void cgs_default_expert_params(cgs_expert_params *out);
/* Wait for all work enqueued on the space's stream. */
cgs_status cgs_synchronize(cgs_space space);

/* ------------------------------------------------------------- space */
/* Enumerate the tuning space (Sect. 1; TS of Alg. 1): decode every raw index
 * k < prod(radix) to digits, look the digits up in the value tables,
 * evaluate every constraint, and keep the valid ones in ascending k.
 *   radix[n_params]   values per parameter, 1..CGS_MAX_RADIX
 *   values[sum radix] value tables, concatenated in parameter order, each
 *                     strictly ascending, |v| < CGS_MAX_ABS_VALUE
 *   cons[n_cons]      constraints (may be NULL when n_cons == 0)
 *   hip_stream        hipStream_t to use, or NULL
 * Synchronises once (to size the valid list).  An empty valid set is not an
 * error (n_valid = 0; every later step reports CGS_EEMPTY). */
cgs_status cgs_space_create(int n_params, const int32_t *radix, const int64_t *values,
                            int n_cons, const cgs_constraint *cons, void *hip_stream,
                            cgs_space *out);
cgs_status cgs_space_info(cgs_space space, uint64_t *n_raw, uint64_t *n_valid);
/* Digits of raw index k (host arithmetic).  digits_host[n_params]. */
cgs_status cgs_space_decode(cgs_space space, uint64_t raw_index, int32_t *digits_host);
/* Valid index of raw index k, or -1 when k is not a valid configuration. */
cgs_status cgs_space_valid_index(cgs_space space, uint64_t raw_index, int64_t *valid_index);
/* Copy valid raw indices [first, first+count) (uint32, ascending). */
cgs_status cgs_space_copy_valid(cgs_space space, uint64_t first, uint64_t count,
                                uint32_t *dst_host);
/* Copy the validity bitmask: bit (k % 32) of word k / 32 is set when raw
 * index k is valid; ceil(n_raw / 32) words. */
cgs_status cgs_space_copy_mask(cgs_space space, uint32_t *dst_host, uint64_t n_words);
void cgs_space_destroy(cgs_space space);

/* ------------------------------------------------------------- model */
/* Load a regression forest and predict every valid configuration
 * (Sect. 3.4.2).  Trees are complete binary trees of depth `depth` in heap
 * order (children of node i: 2i+1, 2i+2); internal node i of tree t goes left
 * when digit[feat[t][i]] <= thr[t][i].  The prediction is the mean of the
 * trees' leaf vectors: sum over t ascending in float32, then one division by
 * n_trees.
 *   feat, thr [n_trees][2^depth - 1]   uint8
 *   leaves    [n_trees][2^depth][n_counters]  float32, finite and >= 0
 *             (counters are non-negative: the score equation divides by
 *             the sum of two predictions; CGS_EINVAL otherwise)
 * The predictions of all valid configurations are kept on the device
 * (n_counters * n_valid floats) and reused by every search step. */
cgs_status cgs_model_load_forest(cgs_space space, int n_trees, int depth, int n_counters,
                                 const uint8_t *feat, const uint8_t *thr, const float *leaves,
                                 cgs_model *out);
/* n_counters and the device time of the last full model evaluation. */
cgs_status cgs_model_info(cgs_model model, int *n_counters, float *eval_ms);
/* Re-run the full-space model evaluation (same result; for timing). */
cgs_status cgs_model_refresh(cgs_model model);
/* Predictions of valid configurations [first, first+count): dst[count][C]. */
cgs_status cgs_model_copy_predictions(cgs_model model, uint64_t first, uint64_t count,
                                      float *dst_host);
/* Predictions of the valid configurations listed in valid_idx_host[n] (any
 * order, repeats allowed): dst[n][C].  An index outside the valid list is
 * CGS_EINVAL. */
cgs_status cgs_model_gather_predictions(cgs_model model, const uint32_t *valid_idx_host, uint64_t n,
                                        float *dst_host);
/* Root-mean-square difference of two models' predictions (same space, same
 * counters) over valid indices sample_host[n]: sqrt(mean over the sampled
 * configurations and the counters of (Pa - Pb)^2), summed in float64. */
cgs_status cgs_model_rmse(cgs_model a, cgs_model b, const uint32_t *sample_host, uint64_t n,
                          double *rmse);
/* Forest only: leaf reached in each tree by valid configurations
 * [first, first+count): dst[n_trees][count] uint16. */
cgs_status cgs_model_copy_leaf_ids(cgs_model model, uint64_t first, uint64_t count,
                                   uint16_t *dst_host);
void cgs_model_destroy(cgs_model model);

/* Regression-tree fitting (Sect. 3.4.2): grow one multi-output regression
 * tree from measured (configuration, counter) pairs on the device, choose
 * its depth on a held-out half, and load it like cgs_model_load_forest.
 *
 *   points_host[n]        valid indices of the measured configurations
 *                         (repeats allowed); n >= 2, n * n_counters < 2^31
 *   targets_host[n][C]    their measured counters, finite and >= 0
 *   keys_host[n]          one random 64-bit number per point: the training
 *                         half is the ceil(n/2) points first in the order of
 *                         (key >> 32, point index), the rest is the test half
 *   max_depth             0..CGS_MAX_DEPTH; min_leaf >= 1
 *
 * Counter c is quantised to integers q = rint(y * 2^s_c), s_c = 22 - e_c,
 * with 2^(e_c - 1) <= max |y_c| < 2^e_c (e_c = 0 when all are 0), so every
 * node sum is exact.  Growth is greedy, level by level: a node with at least
 * max(2, 2 min_leaf) training points takes the binary split (parameter j,
 * digit <= t) with both sides >= min_leaf that maximises
 * sum_c (S_L^2/n_L + S_R^2/n_R) (float64, c ascending; ties to the lower j,
 * then t), if that exceeds its own sum_c S^2/n; otherwise it stays whole
 * ("always left": parameter 0, threshold 255).  Node values are
 * rint(S/n).  The candidate trees are the grown tree cut at depths
 * 0..max_depth; on the test half each has exact error sums A_d = sum |e|,
 * B_d = sum e^2 (e = node value - q, all points and counters); the model
 * is the cut with the lowest A_d, then B_d, then depth, with leaf values
 * float32(value * 2^-s_c).  The model's predictions of every valid
 * configuration are computed as for a loaded forest.
 *
 * CGS_EINVAL for a point outside the valid list or a negative or non-finite target,
 * CGS_ERANGE for sizes outside the limits.  Synchronises; `report` may be
 * NULL. */
typedef struct {
  int32_t depth;                           /* selected cut depth              */
  int32_t max_depth, min_leaf, n_counters;
  uint64_t n_train, n_test;
  uint32_t n_split;                        /* nodes of the grown tree that split */
  float fit_ms;                            /* device time of the fit          */
  int32_t scale_log2[CGS_MAX_COUNTERS];    /* s_c                             */
  uint64_t abs_err[CGS_MAX_DEPTH + 1];     /* A_d                             */
  uint64_t sq_err[CGS_MAX_DEPTH + 1][2];   /* B_d = [1] * 2^64 + [0]          */
} cgs_tree_fit_report;

cgs_status cgs_model_fit_tree(cgs_space space, uint64_t n, int n_counters,
                              const uint32_t *points_host, const float *targets_host,
                              const uint64_t *keys_host, int max_depth, int min_leaf,
                              cgs_model *out, cgs_tree_fit_report *report);
/* Least-squares polynomial counter models (Sect. 3.4.1).  Parameters with
 * two values are binary: their digits select one of 2^B subspaces (bit i =
 * digit of the i-th binary parameter).  Parameters with three or more values
 * are non-binary, with feature x_j = (2 v - v_max - v_min) / (v_max - v_min).
 * In every subspace each counter is a polynomial over the basis: the product
 * of x_j over every set of non-binary parameters of size <= order (sets by
 * size, then lexicographically; the empty set is the constant term), then x_j^2
 * for every non-binary j.  Its coefficients solve
 * (F^T F + lam I) beta = F^T Y over the subspace's training points, float64,
 * lam = 1e-9 trace(F^T F) / T (keeps rank-deficient designs defined); a
 * subspace without training points has beta = 0.  Predictions of every valid
 * configuration are evaluated in float32, clamped at 0 (a polynomial can go
 * negative where counters cannot; a prediction of exactly 0 drops the
 * counter from the score of that configuration) and kept like a forest's. */
#define CGS_POLY_MAX_TERMS 176
#define CGS_POLY_MAX_ORDER 4
#define CGS_POLY_MAX_BINARY 16

/* The design the paper measures: valid configurations whose every non-binary
 * digit is 0, R_j - 1 or the digit whose value is nearest to the middle of the
 * value range (the lower one on a tie), as ascending valid indices.  *count is
 * always set; CGS_ERANGE (with the first `capacity` written) when it exceeds
 * capacity. */
cgs_status cgs_poly_design(cgs_space space, uint64_t capacity, uint32_t *valid_idx_host,
                           uint64_t *count);

typedef struct {
  int32_t n_subspaces, n_terms, order, n_counters;
  uint64_t n_points;
  float fit_ms;        /* device time of features, Gram matrices and solves */
  float eval_ms;       /* device time of the evaluation of every valid configuration */
  int32_t pivot_clamped; /* 1 when a Cholesky pivot was not positive (then clamped) */
  int32_t reserved;
} cgs_poly_fit_report;

/* Fit the polynomials on measured pairs: points_host[n] valid indices
 * (1 <= n < 2^31, repeats allowed), targets_host[n][n_counters] finite;
 * order 0..CGS_POLY_MAX_ORDER.  CGS_ERANGE when the basis exceeds
 * CGS_POLY_MAX_TERMS terms or the space has more than CGS_POLY_MAX_BINARY binary
 * parameters; CGS_EINVAL for an index outside the valid list or a non-finite
 * target.  Synchronises; `report` may be NULL. */
cgs_status cgs_model_fit_poly(cgs_space space, uint64_t n, int n_counters,
                              const uint32_t *points_host, const float *targets_host, int order,
                              cgs_model *out, cgs_poly_fit_report *report);
/* Polynomial models only: subspaces and terms, then the float64 coefficients
 * beta_host[n_subspaces][n_terms][n_counters]. */
cgs_status cgs_poly_shape(cgs_model model, int *n_subspaces, int *n_terms);
cgs_status cgs_poly_copy_coefficients(cgs_model model, double *beta_host);

/* A model whose predictions the caller gives: pred_host[n_valid][n_counters]
 * (finite and >= 0, else CGS_EINVAL), e.g. counters measured on every configuration, the setting of
 * Sect. 4.3 where the search reads measured counters instead of a model's. */
cgs_status cgs_model_load_predictions(cgs_space space, int n_counters, const float *pred_host,
                                      cgs_model *out);

/* The searcher's outer loop, Alg. 1 (Sect. 3.7), on tables of measured
 * runtimes and counters (the paper's simulated autotuning, Sect. 4.1).  A
 * uniform draw gives the first configuration; each iteration profiles the
 * current one (one test: its runtime and Table 1 counters are looked up),
 * runs the expert system and a scored step with the model, then `draws`
 * weighted draws, each one test; the fastest of them (the later on a tie) is
 * profiled next.  The run stops at the first test whose runtime is within
 * well_factor of the table's best (when stop_at_well), after max_tests
 * tests, or when no configuration is left.
 *   runtime_host[n_valid]       float32 runtimes
 *   counters_host[n_valid][24]  Table 1 counters, pre-Volta scales
 *   expert                      expert-system settings (cores, threads)
 *   uniforms_host[n_uniforms]   one 64-bit random number per draw
 *   tested_host[capacity]       valid indices in test order; profiled_host
 *                               (may be NULL) 1 for profiled runs
 *   *n_tests, *tests_to_well    tests made; position (1-based) of the first
 *                               well-performing test, 0 if none
 * The model must predict the 24 counters; the session should be fresh.
 * CGS_ERANGE when the random numbers run out.  An iteration's draws (up to
 * 33) are made in one go, since they depend only on the step's weights and
 * the random numbers: the tests are those of drawing one at a time, but
 * draws after the test that ends the run are made too, so the session's
 * explored set may then hold up to draws - 1 configurations more. */
typedef struct {
  int32_t draws;          /* runs without counters per profiled run (n), 5 by default */
  int32_t stop_at_well;   /* 1: stop at the first well-performing test */
  uint64_t max_tests;     /* 1..capacity */
  double well_factor;     /* 1.1: within 1.1x of the best runtime */
} cgs_tuning_opts;

void cgs_default_tuning_opts(cgs_tuning_opts *out);
cgs_status cgs_tuning_run(cgs_session session, cgs_model model, const float *runtime_host,
                          const double *counters_host, const cgs_expert_params *expert,
                          const uint64_t *uniforms_host, uint64_t n_uniforms,
                          const cgs_tuning_opts *opts, uint64_t capacity, uint64_t *tested_host,
                          uint8_t *profiled_host, uint64_t *n_tests, uint64_t *tests_to_well);

/* Forest models only: number of trees and depth, then the trees in the
 * layout of cgs_model_load_forest (feat, thr [n_trees][2^depth - 1],
 * leaves [n_trees][2^depth][n_counters]). */
cgs_status cgs_model_forest_shape(cgs_model model, int *n_trees, int *depth);
cgs_status cgs_model_copy_forest(cgs_model model, uint8_t *feat_host, uint8_t *thr_host,
                                 float *leaves_host);

/* Multilayer-perceptron surrogate of the counter model (an extension: it
 * stands in for the trees of Sect. 3.4).  Features x_j = digit_j / 8 of
 * every parameter; z1 = W1 x + b1, h1 = gelu(z1), z2 = W2 h1 + b2,
 * h2 = gelu(z2), y = W3 h2 + b3; predictions max(y, 0).  bf16 weights and
 * activations, fp32 accumulation (MFMA), fp32 master weights.
 *   n_in    must equal the space's n_params (<= 32)
 *   hidden  64, 128, 256 or 512
 *   n_out   1..64 counters */
typedef struct {
  int32_t n_in, hidden, n_out, reserved;
} cgs_mlp_desc;

/* Adam settings (Kingma & Ba): lr, beta1, beta2, eps; batch rows per step
 * (1..4096) and number of steps. */
typedef struct {
  float lr, beta1, beta2, eps;
  int32_t batch, steps;
} cgs_train_opts;

/* Number of fp32 parameters: H*F + H + H*H + H + C*H + C, stored in that
 * order: W1 [H][F], b1 [H], W2 [H][H], b2 [H], W3 [C][H], b3 [C]. */
uint64_t cgs_mlp_param_count(const cgs_mlp_desc *desc);

/* Load a perceptron with the given fp32 parameters (layout above) and
 * predict every valid configuration; Adam moments start at zero. */
cgs_status cgs_model_load_mlp(cgs_space space, const cgs_mlp_desc *desc, const float *params_host,
                              cgs_model *out);
/* opts.steps Adam steps on (configuration, counter) pairs: cfg_raw_host[n]
 * raw indices (< n_raw), targets_host[n][n_out]; batch_idx_host
 * [steps][batch] rows of the pairs used by each step.  Loss: mean squared
 * error over the batch and the counters; loss_host[steps] receives it (may be
 * NULL).  Afterwards the predictions of every valid configuration are
 * recomputed.  Synchronises. */
cgs_status cgs_mlp_train(cgs_model model, const uint32_t *cfg_raw_host, const float *targets_host,
                         uint64_t n, const int32_t *batch_idx_host, const cgs_train_opts *opts,
                         float *loss_host);
/* Loss gradient of every parameter (layout above) on n <= 4096 pairs, without
 * updating; grads_host[cgs_mlp_param_count], loss_host (may be NULL). */
cgs_status cgs_mlp_gradients(cgs_model model, const uint32_t *cfg_raw_host,
                             const float *targets_host, uint32_t n, float *grads_host,
                             float *loss_host);
/* Unclamped outputs y of n <= 4096 raw configurations: y_host[n][n_out]. */
cgs_status cgs_mlp_forward(cgs_model model, const uint32_t *cfg_raw_host, uint32_t n,
                           float *y_host);
/* fp32 master parameters (layout above). */
cgs_status cgs_mlp_copy_params(cgs_model model, float *params_host, uint64_t n);

/* ----------------------------------------------------------- session */
/* profile_raw value meaning "nothing profiled yet": the step gives every
 * unexplored configuration score 0 (weight 1), so the next draw is the
 * uniform random start of Alg. 1. */
#define CGS_NO_PROFILE UINT64_MAX

/* A search over `space` with nothing explored.  params: NULL = defaults. */
cgs_status cgs_session_create(cgs_space space, const cgs_params *params, cgs_session *out);

/* One scoring pass of Alg. 1 (Sect. 3.6): mark the profiled configuration
 * explored, score every unexplored valid configuration c against it with
 *   s(c) = sum_{p: dpc_p != 0, a_p != 0, x_p != 0} dpc_p (x_p - a_p) / (a_p + x_p)
 * (x = model prediction of c, a = model prediction of the profiled
 * configuration; float32, counters ascending, every operation rounded), find
 * s_min / s_max over unexplored configurations, normalise
 *   s > 0: (1 + s/s_max)^8;  gamma < s <= 0: max(w_min, (1 - s/s_min)^8)
 *   (1 when s == 0);  s <= gamma: w_min;  explored: 0
 * and quantise to integer weights q = rint(w * 2^23).
 *   profile_raw   raw index of the profiled configuration (must be valid),
 *                 or CGS_NO_PROFILE (delta and measured are then ignored)
 *   delta_host    [n_counters] required counter changes in [-1, 1], or NULL
 *   measured_host [24] Table 1 counters of the profiled run, used when
 *                 delta_host is NULL: the expert system derives the changes
 *                 (cgs_expert_system); the model must have 24 counters
 *   expert        NULL = defaults
 * Records the step; its kernels are enqueued together with its first draw
 * (cgs_sample_next), or when one of its results is read.  Recording a new
 * step before drawing from the previous one still executes the previous one
 * (its profile is marked explored). */
cgs_status cgs_search_step(cgs_session session, cgs_model model, uint64_t profile_raw,
                           const float *delta_host, const double *measured_host,
                           const cgs_expert_params *expert);

/* Restricted step (Sect. 3.7, footnote to the scoring line of Alg. 1: for
 * huge spaces only the neighbourhood of the profiled configuration need be
 * scored).  Candidates: the valid, unexplored configurations whose parameter
 * values differ from the profiled configuration's in 1..radius positions,
 * in the order: distance, then the set of changed parameters
 * (lexicographic), then their new digits (lexicographic, the profile's own
 * digit skipped).  The step scores only the candidates (the score equation,
 * same float32 chain as cgs_search_step), normalises over them (s_min /
 * s_max over the candidates) and quantises the same way; draws
 * (cgs_sample_next) pick among the candidates in candidate order.
 *   profile_raw   must be a valid configuration (no CGS_NO_PROFILE)
 *   radius        1..CGS_MAX_RADIUS
 *   delta_host, measured_host, expert: as for cgs_search_step
 * CGS_ERANGE when the neighbourhood has more than CGS_MAX_NEIGHBOURS
 * configurations (valid or not), CGS_EEMPTY when it has none.  Records the
 * step like cgs_search_step; cgs_session_copy_scores and
 * cgs_session_copy_weights then answer CGS_ESTATE. */
cgs_status cgs_search_step_neighbourhood(cgs_session session, cgs_model model,
                                         uint64_t profile_raw, int radius,
                                         const float *delta_host, const double *measured_host,
                                         const cgs_expert_params *expert);

/* The last restricted step's candidates in candidate order: valid indices,
 * scores and quantised weights (weights of configurations drawn since are
 * 0).  Each output may be NULL; *count receives the number of candidates
 * (CGS_ERANGE when above capacity).  Synchronises.  CGS_ESTATE when the
 * last step was not restricted. */
cgs_status cgs_session_copy_neighbourhood(cgs_session session, uint64_t capacity,
                                          uint32_t *valid_idx_host, float *scores_host,
                                          uint32_t *q_host, uint64_t *count);

/* Draw one configuration (Alg. 1): r = floor(u64 * Q / 2^64) with Q the sum
 * of weights; pick l with sum_{i<l} q_i <= r < sum_{i<=l} q_i (valid-index
 * order, or candidate order after a restricted step); mark it explored and
 * zero its weight for further draws of this step.  Synchronises.
 * CGS_EEMPTY when Q == 0.
 * No tie flag: the weights are integers fixed by the float32 operation
 * order documented at cgs_search_step and the prefix sums are exact, so the
 * pick is a deterministic function of the model's predictions and u64 (a
 * reference evaluating the same float32 order reproduces it exactly).
 *   raw_out / valid_out may be NULL. */
cgs_status cgs_sample_next(cgs_session session, uint64_t u64, uint64_t *raw_out,
                           uint64_t *valid_out);

/* A whole search of Alg. 1 (Sect. 3.7) with one draw per step, driven by
 * host code in the library: the uniform start (cgs_search_step without a
 * profile, cgs_sample_next with u64_host[0]), then for i = 0..n_steps-1 a
 * step profiling the last pick with measured_host[i][24] and expert[i],
 * and a draw with u64_host[i + 1] -- the results of exactly those calls,
 * in that order.  The counter changes of every step follow from the
 * measured counters alone, so the library runs the expert system for all
 * steps first and enqueues the steps ahead of their picks (up to 255
 * ahead): each step's kernels read the configuration to profile from
 * device memory, where the previous draw left it, and the host collects
 * the picks as they are published.
 *   raw_out_host[n_steps + 1]     picks (raw indices); valid_out_host may
 *                                 be NULL; unmade picks stay 2^64 - 1
 *   step_us_host[n_steps]         wall time between the publication of
 *                                 each step's pick and the previous one,
 *                                 in microseconds (may be NULL)
 * Returns the first failing call's status (CGS_EEMPTY when the space runs
 * out); the steps enqueued after that one find no profile and draw
 * nothing.  The session's stream is idle on return. */
cgs_status cgs_search_run(cgs_session session, cgs_model model, int n_steps,
                          const double *measured_host, const cgs_expert_params *expert,
                          const uint64_t *u64_host, uint64_t *raw_out_host,
                          uint64_t *valid_out_host, double *step_us_host);

/* Online retraining of the perceptron surrogate with tree fallback (an
 * extension: the model of Sect. 3.4 stands in for measured counters; here a
 * perceptron stands in for the tree, and the tree judges it).  A search of
 * Alg. 1 with one draw per step, like cgs_search_run but with counter
 * changes given per step, that collects (configuration, counters) pairs as
 * it goes: each pick's counters as measured by a synthetic profiler, the
 * tree's prediction plus noise_host[i][C].  Steps are grouped in windows of
 * retrain_every steps.  Before step 0 and at every window start the
 * surrogate's RMSE against the tree over the valid indices val_sample_host
 * [n_val] (cgs_model_rmse) decides the model of the window: the surrogate
 * if RMSE <= threshold, else the tree.  At the start of window w >= 1 the
 * surrogate first takes train_steps Adam steps (cgs_mlp_train) on the seed
 * pairs seed_cfg_raw_host[n_seed] / seed_targets_host[n_seed][C] followed
 * by every pair collected so far, in pick order; entry b of Adam step k
 * uses pair floor(u * n_pairs / 2^64) with
 * u = batch_u64_host[(w - 1)][k][b].
 *   step 0          the uniform start (cgs_search_step without a profile on
 *                   the tree, cgs_sample_next with u64_host[0])
 *   step i >= 1     profile the last pick with changes delta_host[i - 1][C],
 *                   draw with u64_host[i]
 *   raw_out_host[n_steps + 1], valid_out_host (may be NULL): picks; unmade
 *                   picks stay 2^64 - 1
 *   window_rmse_host[W], window_mlp_host[W] (1: surrogate, 0: tree), for the
 *                   W = 1 + n_steps / retrain_every windows
 *   step_us_host[n_steps], retrain_ms_host[W - 1] (may be NULL): wall times
 *                   of each step with its draw, and of each retraining with
 *                   its RMSE check
 * A retrained surrogate is evaluated over every valid configuration only
 * when its window scores with it: its RMSE comes from the validation
 * configurations alone (the same values a full evaluation gives them), and
 * the full evaluation follows when the RMSE passes, and once before the
 * call returns, so the model's predictions are current afterwards.
 * tree: any model (normally a forest); mlp: a perceptron with the same
 * counters on the same space; the session should be fresh.  Returns the
 * first failing call's status (CGS_EEMPTY when the space runs out). */
typedef struct {
  int32_t retrain_every; /* steps per window (20)                          */
  int32_t train_steps;   /* Adam steps per retraining (500); 0: none        */
  int32_t batch;         /* pairs per Adam step, 1..4096 (256)              */
  int32_t reserved;
  float lr, beta1, beta2, eps; /* Adam (1e-3, 0.9, 0.999, 1e-8)            */
  double threshold;      /* largest RMSE at which the surrogate scores (0.05) */
} cgs_online_opts;

void cgs_default_online_opts(cgs_online_opts *out);
cgs_status cgs_online_run(cgs_session session, cgs_model tree, cgs_model mlp, int n_steps,
                          const float *delta_host, const uint64_t *u64_host,
                          const float *noise_host, uint64_t n_seed,
                          const uint32_t *seed_cfg_raw_host, const float *seed_targets_host,
                          uint64_t n_val, const uint32_t *val_sample_host,
                          const uint64_t *batch_u64_host, const cgs_online_opts *opts,
                          uint64_t *raw_out_host, uint64_t *valid_out_host,
                          double *window_rmse_host, int32_t *window_mlp_host,
                          double *step_us_host, double *retrain_ms_host);

/* Statistics of the last step (synchronises). */
cgs_status cgs_session_step_info(cgs_session session, cgs_step_info *out);

/* Device time per kernel kind, summed over the timed launches since session
 * creation (sessions created with params.timing > 0; zeros otherwise); slot
 * [3] is the scoring of restricted steps (candidates and weights):
 *   total_ms[4] / launches[4]: [0] score pass of scored steps (a profile and
 *   at least one counter with a non-zero change; the pass of an unscored
 *   step such as the uniform start reads no prediction and is not counted),
 *   [1] weight pass, [2] draws, [3] restricted scoring (one launch = one
 *   step).  Synchronises. */
cgs_status cgs_session_kernel_times(cgs_session session, double *total_ms, uint64_t *launches);

/* Mark raw index k explored (must be valid). */
cgs_status cgs_mark_explored(cgs_session session, uint64_t raw_index);
/* Copy scores of valid configurations [first, first+count) from the last step. */
cgs_status cgs_session_copy_scores(cgs_session session, uint64_t first, uint64_t count,
                                   float *dst_host);
/* Copy quantised weights q of valid configurations [first, first+count) as
 * the last step left them (explored: 0). */
cgs_status cgs_session_copy_weights(cgs_session session, uint64_t first, uint64_t count,
                                    uint32_t *dst_host);
/* Copy the explored bitmask over valid indices: ceil(n_valid / 32) words. */
cgs_status cgs_session_copy_explored(cgs_session session, uint32_t *dst_host, uint64_t n_words);
void cgs_session_destroy(cgs_session session);

/* ---------------------------------------------------------- batches */
/* Many independent searches stepped together (an extension: the paper tunes
 * one kernel at a time).  Each step scores, weighs and draws in every member
 * session with three launches that run over the concatenated per-session
 * tile lists, replayed from one captured hipGraph. */
typedef struct cgs_batch_s *cgs_batch;

typedef struct {
  int32_t score_grid;  /* workgroups of the score pass                     */
  int32_t weight_grid; /* workgroups of the weight pass                    */
  int32_t use_graph;   /* 1: replay the step from a captured hipGraph      */
  int32_t variant;     /* score-pass kernel: counter rows in flight x waves
                          per SIMD, 0 (8 rows, unconstrained), 1 (4, 4),
                          2 (16, 2), 3 (8, 4), 4 (4, 8)                   */
} cgs_batch_schedule;

/* sessions[i] searches its own space with models[i] (same space).  The batch
 * keeps pointers to both: destroy the batch first.  While stepping through
 * the batch, the sessions may still be read (copy_scores, step_info, ...) and
 * drawn from between batch steps.  sched NULL: defaults (grids capped at
 * 2048 workgroups, graph on). */
cgs_status cgs_batch_create(int n, const cgs_session *sessions, const cgs_model *models,
                            const cgs_batch_schedule *sched, cgs_batch *out);
/* One step in every session: profile_raw_host[n] (CGS_NO_PROFILE allowed),
 * deltas_host: session i's n_counters changes, concatenated in session
 * order (may be NULL when no session has a profile), u64_host[n] uniforms.
 * Outputs per session (may be NULL): raw / valid index of the pick and
 * CGS_OK or CGS_EEMPTY.  Synchronises. */
cgs_status cgs_batch_step(cgs_batch batch, const uint64_t *profile_raw_host,
                          const float *deltas_host, const uint64_t *u64_host,
                          uint64_t *raw_out_host, uint64_t *valid_out_host,
                          int32_t *status_out_host);
/* One more draw in every session from the weights of the batch's last step
 * (the further draws of an Alg. 1 iteration, Sect. 3.7): u64_host[n]
 * uniforms; outputs as for cgs_batch_step.  Each drawn configuration is
 * marked explored and its weight removed, as cgs_sample_next does.
 * CGS_ESTATE when a session has stepped on its own since the batch step.
 * Synchronises. */
cgs_status cgs_batch_draw(cgs_batch batch, const uint64_t *u64_host, uint64_t *raw_out_host,
                          uint64_t *valid_out_host, int32_t *status_out_host);
/* Device time of the last batch step (ms, HIP events around the launch). */
cgs_status cgs_batch_step_time(cgs_batch batch, float *ms);
/* Picks the schedule by timing candidates with HIP events (the median of 5
 * runs after a warm-up; score records with every counter active; no draw,
 * the explored sets are untouched; the sessions' last-step results become
 * unavailable until their next step): every score-pass variant at grid
 * sizes 128..8192 below the number of tiles and at one workgroup per tile,
 * then the weight-pass grid over blocks likewise, then graph replay against
 * plain launches of the step.  cache_path (may be NULL): a text file of
 * "<shape key> -> score_grid weight_grid use_graph variant" lines, read
 * first and appended to. */
cgs_status cgs_batch_autotune(cgs_batch batch, const char *cache_path,
                              cgs_batch_schedule *chosen);
cgs_status cgs_batch_set_schedule(cgs_batch batch, const cgs_batch_schedule *sched);
void cgs_batch_destroy(cgs_batch batch);

/* Alg. 1 for every session of a batch at once: run i uses session i (fresh)
 * and model i (24 counters, all on one space) and the random numbers
 * uniforms_host[i][n_uniforms]; every run makes exactly the tests
 * cgs_tuning_run would make with the same numbers.  Runs advance in
 * lockstep: one batch step (the scored step and first draw of every run),
 * then draws - 1 batched draws; a finished run steps unprofiled, its
 * results ignored, until half of the batch has finished: the live runs then
 * continue in a new batch of their sessions and models (freed on return).
 *   tested_host[n][capacity], profiled_host[n][capacity] (may be NULL),
 *   n_tests[n], tests_to_well[n]   as for cgs_tuning_run, per run
 * The options and outputs are those of cgs_tuning_run (above). */
cgs_status cgs_tuning_run_batch(cgs_batch batch, const float *runtime_host,
                                const double *counters_host, const cgs_expert_params *expert,
                                const uint64_t *uniforms_host, uint64_t n_uniforms,
                                const cgs_tuning_opts *opts, uint64_t capacity,
                                uint64_t *tested_host, uint8_t *profiled_host, uint64_t *n_tests,
                                uint64_t *tests_to_well);

/* ------------------------------------------------ standalone sampler */
/* The draw of Alg. 1 on caller-given integer weights: n_draws consecutive
 * draws with removal over q_host[n] (each < 2^32), uniforms u64_host[n_draws].
 * picks_host[i] = chosen index, or -1 once every weight is 0.  Uses the same
 * device scan and search as cgs_sample_next.  Synchronises. */
cgs_status cgs_sample_weights(cgs_space stream_owner, const uint32_t *q_host, uint64_t n,
                              const uint64_t *u64_host, int n_draws, int64_t *picks_host);

/* cgs_sample_weights for callers that cannot allocate device memory (code
 * under stream capture, tight serving loops, hosts that forbid hipMalloc):
 * the same arguments, draws and results, but the working copy of the
 * weights and the block sums live in one fixed array of device memory that
 * the library reserves per GPU (16 MiB + 8 KiB, held until the process
 * ends), so the call makes no hipMalloc or hipFree.
 *   n       at most 4,194,304 (2^22) weights; more returns CGS_ERANGE
 *           before any device work
 * The array is shared by every call on the same GPU and keeps the last
 * call's contents; each call rewrites all of it that it reads.  Calls that
 * overlap on one GPU (other threads, other streams) race on it: serialise
 * them.  Synchronises. */
cgs_status cgs_sample_weights_noalloc(cgs_space stream_owner, const uint32_t *q_host, uint64_t n,
                                      const uint64_t *u64_host, int n_draws,
                                      int64_t *picks_host);

/* -------------------------------------------------- expert system */
/* Bottleneck analysis and counter changes (Sect. 3.5), host float64.
 *   pc_host[24]       measured counters in Table 1 order
 *   b_host[18]        out: bottlenecks dram_read, dram_write, l2_read,
 *                     l2_write, tex, local, shr_load, shr_store, fp32, fp64,
 *                     int, misc, ldst, cont, bconv, issue, sm, paral
 *   delta_host[24]    out: required change per Table 1 counter
 *   delta_threads     out: required change of the thread count (may be NULL)
 * A ratio with a zero denominator is 0; bottlenecks are clipped to [0, 1]. */
cgs_status cgs_expert_system(const double *pc_host, const cgs_expert_params *expert,
                             double *b_host, double *delta_host, double *delta_threads);

#ifdef __cplusplus
}
#endif
#endif /* CGS_H */
