"""Bottleneck analysis and counter-change computation (oracle), Sect. 3.5.

Input: one measured counter vector in Table 1 order (24 values).  Output:
the bottleneck vector B (Sect. 3.5.1) and the required counter changes
dPC (Sect. 3.5.2), one per Table 1 counter.

Bottlenecks (float64, each clipped to the stated range [0, 1]):
  b_DRAM_read/write   DRAM read (write) share of DRAM transactions times
                      DRAM_U/10 (global-read / global-write equations);
                      L2 and shared memory analogous with L2_*, SHR_*
  b_tex               TEX_U/10
  b_local             LOC_O/100 times the largest of DRAM_U, L2_U, TEX_U /10
                      (local-memory equation)
  ins_fitted          32 * INST_EXE * 100/WARP_E * 100/WARP_NP_E
  ins_util            INST_ISSUE_U/100, or min(1, INST_ISSUE_U/50) on Volta+
  b_X                 INST_X / ins_fitted * ins_util for the seven
                      instruction classes (FP32 equation and its analogues)
  b_issue             max_X(INST_X / ins_fitted) * (100 - INST_ISSUE_U)/100
  b_sm                (100 - SM_E)/100
  b_paral             max(0, (5 cores - threads) / (5 cores))

Changes: memory counters get -b; instruction counters (and INST_ISSUE_U
from b_issue, "analogous") get -(b - r)/(1 - r) when b > r, else 0, with
r = inst_reaction (0.7, or 0.5 for compute-bound problems); SM_E gets +b_sm.
The thread-count change (+b_paral) has no model counter and is returned
separately.

Readings: a ratio whose denominator is 0 is 0; utilisation counters are on
the pre-Volta 0..10 scale except L2_U, which on Volta+ is a percentage and is
divided by 100 instead of 10; the operation order below is the order of the
equations, left to right.
"""
from __future__ import annotations

import numpy as np

(DRAM_RT, DRAM_WT, L2_RT, L2_WT, TEX_RWT, LOC_O, SHR_LT, SHR_WT, INST_F32, INST_F64,
 INST_INT, INST_MISC, INST_LDST, INST_CONT, INST_BCONV, INST_EXE, INST_ISSUE_U, DRAM_U,
 L2_U, TEX_U, SHR_U, SM_E, WARP_E, WARP_NP_E) = range(24)

INST_CLASSES = (INST_F32, INST_F64, INST_INT, INST_MISC, INST_LDST, INST_CONT, INST_BCONV)

# Order of the bottleneck vector returned by ``bottlenecks``.
B_NAMES = ("dram_read", "dram_write", "l2_read", "l2_write", "tex", "local", "shr_load",
           "shr_store", "fp32", "fp64", "int", "misc", "ldst", "cont", "bconv", "issue",
           "sm", "paral")


def _ratio(n: float, d: float) -> float:
    return n / d if d != 0.0 else 0.0


def _clip01(x: float) -> float:
    return min(1.0, max(0.0, x))


def bottlenecks(pc, volta: bool = False, cores: float = 1.0, threads: float = 0.0) -> np.ndarray:
    """Bottleneck vector B (18 entries, order ``B_NAMES``)."""
    c = [float(v) for v in pc]
    dram = c[DRAM_U] / 10.0
    l2 = c[L2_U] / (100.0 if volta else 10.0)
    tex = c[TEX_U] / 10.0
    shr = c[SHR_U] / 10.0

    b = []
    b.append(_ratio(c[DRAM_RT], c[DRAM_RT] + c[DRAM_WT]) * dram)
    b.append(_ratio(c[DRAM_WT], c[DRAM_RT] + c[DRAM_WT]) * dram)
    b.append(_ratio(c[L2_RT], c[L2_RT] + c[L2_WT]) * l2)
    b.append(_ratio(c[L2_WT], c[L2_RT] + c[L2_WT]) * l2)
    b.append(tex)
    b.append(c[LOC_O] / 100.0 * max(dram, l2, tex))
    b.append(_ratio(c[SHR_LT], c[SHR_LT] + c[SHR_WT]) * shr)
    b.append(_ratio(c[SHR_WT], c[SHR_LT] + c[SHR_WT]) * shr)

    ins_fitted = 32.0 * c[INST_EXE] * _ratio(100.0, c[WARP_E]) * _ratio(100.0, c[WARP_NP_E])
    if volta:
        ins_util = min(1.0, c[INST_ISSUE_U] / 50.0)
    else:
        ins_util = c[INST_ISSUE_U] / 100.0
    fracs = [_ratio(c[k], ins_fitted) for k in INST_CLASSES]
    for f in fracs:
        b.append(f * ins_util)
    b.append(max(fracs) * ((100.0 - c[INST_ISSUE_U]) / 100.0))
    b.append((100.0 - c[SM_E]) / 100.0)
    b.append(max(0.0, (cores * 5.0 - threads) / (cores * 5.0)))
    return np.array([_clip01(x) for x in b], dtype=np.float64)


def _react(b: float, r: float) -> float:
    """Reaction rule of the FP32 equation."""
    if b <= r:
        return 0.0
    return -((b - r) / (1.0 - r))


def delta_pc(B, inst_reaction: float = 0.7):
    """Counter changes dPC in Table 1 order (24 float64) and the thread change."""
    d = np.zeros(24, dtype=np.float64)
    d[DRAM_RT] = -B[0]
    d[DRAM_WT] = -B[1]
    d[L2_RT] = -B[2]
    d[L2_WT] = -B[3]
    d[TEX_RWT] = -B[4]
    d[LOC_O] = -B[5]
    d[SHR_LT] = -B[6]
    d[SHR_WT] = -B[7]
    for i, k in enumerate(INST_CLASSES):
        d[k] = _react(B[8 + i], inst_reaction)
    d[INST_ISSUE_U] = _react(B[15], inst_reaction)
    d[SM_E] = B[16]
    return d, float(B[17])


def expert_system(pc, volta=False, cores=1.0, threads=0.0, inst_reaction=0.7):
    """Counters -> (B, dPC float64, dPC rounded to float32, thread change)."""
    B = bottlenecks(pc, volta, cores, threads)
    d, d_threads = delta_pc(B, inst_reaction)
    return B, d, d.astype(np.float32), d_threads
