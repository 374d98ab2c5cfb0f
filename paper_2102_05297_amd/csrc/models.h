// Model-creation interfaces of libcgs (tree fitting, least-squares
// polynomials, prediction tables), shared by the host runtime and the
// kernels that build models.  The sweep's own types live in internal.h.
#pragma once

#include "internal.h"

namespace cgs {

// Predictions given per configuration, src[l][C], into the model layout
// P[c][stride].
hipError_t launch_rows_to_columns(const float *d_src, uint32_t n, int C, float *d_P,
                                  uint64_t stride, hipStream_t stream);

// The perceptron's training forward pass (features, then one GEMM per layer
// with the bias and GELU in its epilogue) into a.xout, z1out, h1out, z2out,
// h2out, yout; w1, w2, w3: the fp32 master weights ([H][F], [H][H], [C][H]).
// With `loss` set (training), the output layer's epilogue also forms the
// error d = Y - T against the targets and writes dY = scale * d (fp32 dyf and
// bf16 dyb, [n][Cp] like Y, padding columns untouched) and, per 32 x 32
// output tile, the sum of d^2 into partial[tile] (ceil(n/32) * ceil(C/32)
// tiles, row-major over the tiles).
struct LossArgs {
  const float *targets; // [rows][C]; output row i takes target row batch[i] (or i)
  const int32_t *batch;
  float scale;          // 2 / (n C)
  float *dyf;
  __bf16 *dyb;
  float *partial;
};
hipError_t launch_mlp_train_forward(const MlpFwdArgs &a, const float *w1, const float *w2,
                                   const float *w3, const LossArgs *loss, hipStream_t stream);
// Column sums dst[c] = sum over rows r < nrows of src[r * ld + c], c < ncols,
// in row order split over the waves of a workgroup; with loss_out set, also
// *loss_out = (partial[0] + ... + partial[n_partial - 1]) / loss_div.
struct ColSumJob {
  const float *src;
  int ld, nrows, ncols;
  float *dst;
  const float *partial;
  int n_partial;
  float *loss_out;
  float loss_div;
};
// One level of the backward pass as one launch: products g0 and g1 (bf16
// operands; epilogue 0: C = A B; 1: dZ = (A B) * gelu'(Z), fp32 and bf16)
// and the column sums cs; an empty product has M = 0, no sums ncols = 0.
hipError_t launch_bwd_group(const GemmArgs &g0, int epi0, const GemmArgs &g1, int epi1,
                            const ColSumJob &cs, hipStream_t stream);
// Bias gradients (column sums of dZ1, dZ2 [n][H] and dY [n][Cp]) and the
// mean squared error: loss_out = (partial[0] + ... + partial[n_partial - 1]) / (n C).
hipError_t launch_bias_grads(const float *dz1, const float *dz2, const float *dyf, int n, int H,
                             int C, int Cp, float *gb1, float *gb2, float *gb3,
                             const float *partial, int n_partial, float *loss_out,
                             hipStream_t stream);
// The bf16 weights from the fp32 masters theta[n]: the inference fragments
// w1p, w2p, w3p, and the transposed copies w2t[k][o] = W2[o][k] ([H][H]) and
// w3t[k][c] = W3[c][k] ([H][Cp], Cp = C rounded up to 32) that the backward
// products read.
hipError_t launch_pack_weights(const MlpShape &sh, const float *theta, size_t n, __bf16 *w1p,
                               __bf16 *w2p, __bf16 *w3p, __bf16 *w2t, __bf16 *w3t,
                               hipStream_t stream);
// One Adam step on theta (moments m, v; c1, c2 the bias corrections of this
// step), then the same packing of the updated weights.
hipError_t launch_adam_pack(const MlpShape &sh, float *theta, float *m, float *v,
                            const float *grad, size_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2, __bf16 *w1p, __bf16 *w2p, __bf16 *w3p,
                            __bf16 *w2t, __bf16 *w3t, hipStream_t stream);

// ---- regression-tree fitting (Sect. 3.4.2)
FastDiv make_fastdiv(uint32_t d);

struct TreeFitIn {
  const SpaceDev *d_space;
  const uint32_t *d_idx;    // valid raw indices of the space
  uint32_t n_valid;
  int n_params;
  const int32_t *radix;     // host [n_params]
  uint32_t n;               // measured points, 2 .. 2^31 - 1
  int n_counters;
  const uint32_t *d_points; // valid indices [n]
  const float *d_targets;   // [n][n_counters]
  const uint64_t *d_keys;   // [n]
  int max_depth, min_leaf;
};
struct TreeFitOut {
  uint32_t err; // bit 0: a point outside the valid list; bit 1: a non-finite target
  int32_t depth;
  uint32_t n_train, n_test, n_split;
  int32_t scale[CGS_MAX_COUNTERS];
  uint64_t abs_err[CGS_MAX_DEPTH + 1];
  uint64_t sq_lo32[CGS_MAX_DEPTH + 1], sq_hi32[CGS_MAX_DEPTH + 1]; // sum e^2 = hi 2^32 + lo
  float ms;
};
struct TreeFitWork;
// Runs the whole fit on `stream` and synchronises; *work holds the grown tree
// until tree_fit_release (also after an error, when non-null).
hipError_t tree_fit_run(const TreeFitIn &in, TreeFitOut &out, TreeFitWork **work,
                        hipStream_t stream);
// Writes the tree cut at `depth` in the evaluator's layout.
hipError_t tree_fit_emit(const TreeFitWork *work, int depth, uint16_t *d_nodes, float *d_leaves,
                         hipStream_t stream);
void tree_fit_release(TreeFitWork *work);

// ---- least-squares polynomial models per binary subspace (Sect. 3.4.1)
constexpr int kPolyMaxTerms = CGS_POLY_MAX_TERMS;   // the solve keeps the packed factor in LDS
constexpr int kPolyMaxOrder = CGS_POLY_MAX_ORDER;   // variables per basis term
constexpr int kPolyMaxBinary = CGS_POLY_MAX_BINARY; // at most 65,536 subspaces
// Term descriptor: bits 0..2 the number of factors, then 5 bits per factor
// (a parameter index); squares repeat their parameter.
struct PolyDev {
  int32_t P, k, B, T, C, S, order, pad;
  uint32_t bin_params[CGS_MAX_PARAMS]; // parameter of subspace bit i
  uint32_t terms[kPolyMaxTerms];
  double xv64[CGS_MAX_PARAMS * CGS_MAX_RADIX]; // feature of (parameter, digit)
  float xv32[CGS_MAX_PARAMS * CGS_MAX_RADIX];
};
size_t poly_solve_lds(int T, int C);
hipError_t launch_poly_design(const SpaceDev *d_space, const uint32_t *d_idx, uint32_t nv,
                              const uint32_t *d_allowed, uint64_t *d_tile_cnt,
                              uint64_t *d_tile_off, uint32_t *d_out, hipStream_t stream);
// Parts each subspace's Gram sums are split into (a partial Gram buffer
// of parts * S * (T + C)^2 doubles is needed when above 1).
uint32_t poly_gram_parts(int S, uint32_t n_pairs);
// d_list[d_off[s] .. d_off[s + 1]): the points (positions in d_pts) of
// subspace s in input order.  d_Gp: the partial Gram buffer, or NULL (no
// parts).
hipError_t launch_poly_fit(const PolyDev *d_pd, int T, int C, int S, const SpaceDev *d_space,
                           const uint32_t *d_idx, uint32_t nv, const uint32_t *d_pts,
                           const float *d_Y, uint32_t n, double *d_F, uint32_t *d_sub,
                           const uint32_t *d_list, const uint32_t *d_off,
                           const uint32_t *d_pairs, uint32_t n_pairs, double *d_G, double *d_Gp,
                           double *d_beta64, float *d_beta32, uint32_t *d_err,
                           hipStream_t stream);
hipError_t launch_poly_eval(const PolyDev *d_pd, int T, int C, int S, const SpaceDev *d_space,
                            const uint32_t *d_idx, uint32_t nv, const float *d_beta32, float *d_P,
                            uint64_t stride, hipStream_t stream);

} // namespace cgs
