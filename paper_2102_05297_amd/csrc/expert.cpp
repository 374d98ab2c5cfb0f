// Bottleneck analysis and required counter changes (Sect. 3.5), host float64.
//
// Counter order is Table 1's.  Each formula below is evaluated left to right
// exactly as the corresponding equation reads; the file is compiled without
// floating-point contraction so every operation is one IEEE rounding.
#include <algorithm>
#include <cmath>

#include "cgs.h"

namespace {

enum {
  DRAM_RT, DRAM_WT, L2_RT, L2_WT, TEX_RWT, LOC_O, SHR_LT, SHR_WT, INST_F32, INST_F64,
  INST_INT, INST_MISC, INST_LDST, INST_CONT, INST_BCONV, INST_EXE, INST_ISSUE_U, DRAM_U,
  L2_U, TEX_U, SHR_U, SM_E, WARP_E, WARP_NP_E
};

// A ratio whose denominator is zero is taken as zero.
inline double ratio(double n, double d) { return d != 0.0 ? n / d : 0.0; }
inline double clip01(double x) { return std::min(1.0, std::max(0.0, x)); }

// Reaction of an instruction-related bottleneck (FP32 reaction equation).
inline double react(double b, double r) { return b <= r ? 0.0 : -((b - r) / (1.0 - r)); }

} // namespace

extern "C" cgs_status cgs_expert_system(const double *pc, const cgs_expert_params *ep,
                                        double *b_out, double *delta_out,
                                        double *delta_threads) {
  if (!pc || !b_out || !delta_out) return CGS_EINVAL;
  cgs_expert_params def;
  cgs_default_expert_params(&def);
  const cgs_expert_params &e = ep ? *ep : def;
  if (!(e.inst_reaction >= 0.0 && e.inst_reaction < 1.0) || !(e.cores > 0.0)) return CGS_EINVAL;
  for (int i = 0; i < 24; ++i)
    if (!std::isfinite(pc[i])) return CGS_EINVAL;

  const double dram = pc[DRAM_U] / 10.0;
  const double l2 = pc[L2_U] / (e.volta ? 100.0 : 10.0);
  const double tex = pc[TEX_U] / 10.0;
  const double shr = pc[SHR_U] / 10.0;

  double b[18];
  // memory subsystems: utilisation weighted by the read / write share
  b[0] = ratio(pc[DRAM_RT], pc[DRAM_RT] + pc[DRAM_WT]) * dram;
  b[1] = ratio(pc[DRAM_WT], pc[DRAM_RT] + pc[DRAM_WT]) * dram;
  b[2] = ratio(pc[L2_RT], pc[L2_RT] + pc[L2_WT]) * l2;
  b[3] = ratio(pc[L2_WT], pc[L2_RT] + pc[L2_WT]) * l2;
  b[4] = tex;
  b[5] = pc[LOC_O] / 100.0 * std::max(std::max(dram, l2), tex);
  b[6] = ratio(pc[SHR_LT], pc[SHR_LT] + pc[SHR_WT]) * shr;
  b[7] = ratio(pc[SHR_WT], pc[SHR_LT] + pc[SHR_WT]) * shr;

  // instructions: shares of the efficiency-corrected instruction count
  const double ins_fitted =
      32.0 * pc[INST_EXE] * ratio(100.0, pc[WARP_E]) * ratio(100.0, pc[WARP_NP_E]);
  const double ins_util =
      e.volta ? std::min(1.0, pc[INST_ISSUE_U] / 50.0) : pc[INST_ISSUE_U] / 100.0;
  const int classes[7] = {INST_F32, INST_F64, INST_INT, INST_MISC, INST_LDST, INST_CONT, INST_BCONV};
  double util_max = 0.0;
  for (int i = 0; i < 7; ++i) {
    const double frac = ratio(pc[classes[i]], ins_fitted);
    b[8 + i] = frac * ins_util;
    util_max = i == 0 ? frac : std::max(util_max, frac);
  }
  b[15] = util_max * ((100.0 - pc[INST_ISSUE_U]) / 100.0);
  // parallelism
  b[16] = (100.0 - pc[SM_E]) / 100.0;
  b[17] = std::max(0.0, (e.cores * 5.0 - e.threads) / (e.cores * 5.0));
  for (int i = 0; i < 18; ++i) b_out[i] = clip01(b[i]);

  double *d = delta_out;
  for (int i = 0; i < 24; ++i) d[i] = 0.0;
  d[DRAM_RT] = -b_out[0];
  d[DRAM_WT] = -b_out[1];
  d[L2_RT] = -b_out[2];
  d[L2_WT] = -b_out[3];
  d[TEX_RWT] = -b_out[4];
  d[LOC_O] = -b_out[5];
  d[SHR_LT] = -b_out[6];
  d[SHR_WT] = -b_out[7];
  for (int i = 0; i < 7; ++i) d[classes[i]] = react(b_out[8 + i], e.inst_reaction);
  d[INST_ISSUE_U] = react(b_out[15], e.inst_reaction);
  d[SM_E] = b_out[16];
  if (delta_threads) *delta_threads = b_out[17];
  return CGS_OK;
}
