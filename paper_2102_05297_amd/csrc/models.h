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

// The bf16 copies of the perceptron's weights, rewritten from the fp32
// masters at creation and by every Adam step (mlp.hip):
//   w1p, w2p, w3p: the inference kernel's packed A fragments (32x32x16);
//   w2t (H x H), w3t (H x Cp): W2^T and W3^T, the training backward's B
//   operands; w1n (H x 32), w2n (H x H), w3n (Cp x H): W1, W2, W3, the
//   training forward's B operands (W1's rows padded to 32 features, W3 to Cp
//   rows); all five in the 16x16x32 MFMA fragment order of mlp.hip.
// Padding is never written: the caller zeroes w1p, w3p, w3t, w1n and w3n.
struct MlpCopies {
  __bf16 *w1p, *w2p, *w3p, *w2t, *w3t, *w1n, *w2n, *w3n;
};

// One training step of the perceptron in two launches (mlp.hip), after
// launch_mlp_gather_rows has gathered the rows of a run of steps.
// launch_mlp_train_rows: per 16 rows of the batch, the forward pass, the
// loss terms (dY = scale (Y - T)) and the backward chain to dZ1; it writes
// the weight gradients' operands transposed, [feature][n_pad] bf16 (xt: 32
// feature rows, zero past F; h1t, h2t, dz2t, dz1t: H rows; dyt: Cp rows),
// the column sums of dY, dZ2 and dZ1 over each block of 16 rows
// (bp3[blk][Cp], bp2[blk][H], bp1[blk][H]) and each block's sum of squared
// errors (lossp[blk]).  Without train only the forward pass runs and Y goes
// to yout[n][Cp].  Rows past n are zeros.
struct TrainRowsArgs {
  const __bf16 *xin;        // the step's features [n_pad][K1] (launch_mlp_gather_rows)
  const float *tin;         // the step's targets [n][C], or null (forward only)
  bool train;               // tin set
  uint32_t n, n_pad;        // rows; a multiple of 32 >= n
  int H, C, K1;
  float scale;              // 2 / (n C)
  const __bf16 *w1n, *w2n, *w3n, *w2t, *w3t;
  const float *b1, *b2, *b3;
  float *yout;
  __bf16 *xt, *h1t, *h2t, *dyt, *dz2t, *dz1t;
  float *bp1, *bp2, *bp3, *lossp;
};
hipError_t launch_mlp_train_rows(const TrainRowsArgs &a, hipStream_t stream);
// The features (and targets) of `steps` steps of n rows: step s, row r is
// pair batch[s n + r] (pair r when batch is null); xg[s][n_pad][K1] bf16,
// zero rows past n; tg[s][n][C] when targets is set.
hipError_t launch_mlp_gather_rows(const SpaceDev *sp, const uint32_t *cfg_raw,
                                  const int32_t *batch, const float *targets, uint32_t steps,
                                  uint32_t n, uint32_t n_pad, int F, int K1, int C, __bf16 *xg,
                                  float *tg, hipStream_t stream);
// launch_mlp_grad_tiles: the weight gradients dW2 = dZ2^T H1, dW1 = dZ1^T X,
// dW3 = dY^T H2 by 32 x 32 tiles and the bias gradients (the blocks' column
// sums added in block order) from launch_mlp_train_rows's outputs; with grad
// set they are stored there (the layout of theta), otherwise one Adam step
// updates theta, m, v and every bf16 copy.  loss_out (if set) gets
// (lossp[0] + ... ) / loss_div.
struct GradTilesArgs {
  MlpShape sh;
  uint32_t n_pad;
  const __bf16 *xt, *h1t, *h2t, *dyt, *dz2t, *dz1t;
  const float *bp1, *bp2, *bp3, *lossp;
  float *loss_out;
  float loss_div;
  float *grad;
  float *theta, *m, *v;
  float lr, beta1, beta2, eps, c1, c2;
  MlpCopies cp;
};
hipError_t launch_mlp_grad_tiles(const GradTilesArgs &g, hipStream_t stream);
// launch_sq_diff with Pa holding the sampled configurations' predictions
// in sample order: Pa[c * stride_a + i] against Pb[c * stride_b + sample[i]].
hipError_t launch_sq_diff_dense(const float *Pa, const float *Pb, uint64_t stride_a,
                                uint64_t stride_b, int n_counters, const uint32_t *sample,
                                uint32_t n, double *partial, uint32_t grid, hipStream_t stream);
// Every bf16 copy (MlpCopies) from the fp32 masters theta[n].
hipError_t launch_pack_weights(const MlpShape &sh, const float *theta, size_t n,
                               const MlpCopies &cp, hipStream_t stream);

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
