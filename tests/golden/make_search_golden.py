"""Writes c2_search.json: the oracle's trajectory of the 100-step search on
the 12-parameter space (2^24 raw configurations, forest of 16 depth-12 trees,
24 counters), computed by the oracle only.  Run from the repository root:

    python tests/golden/make_search_golden.py

Trajectory (Alg. 1 with one draw per scoring pass):
  step 0    nothing profiled: uniform draw with U[0]
  step i>0  profile = pick of step i-1; counter changes from the expert
            system on synthetic counters pcs[i-1] (threads thr[i-1], 1920
            cores, inst_reaction 0.7, pre-Volta scales); draw with U[i]
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import expert as E  # noqa: E402
from oracle import search as SR  # noqa: E402

N_STEPS = 100
CORES = 1920.0


def inputs():
    g = synth.rng(2, 3)
    U = synth.uniforms_u64(g, N_STEPS + 1)
    pcs = synth.profiler_counters(synth.rng(2, 4), N_STEPS)
    thr = synth.threads_launched(synth.rng(2, 5), N_STEPS)
    return U, pcs, thr


def main():
    t0 = time.time()
    spec = synth.space_c2()
    forest = synth.forest_c2(spec)
    prep = SR.prepare(spec, forest)
    print(f"prepared {len(prep.valid)} valid configurations in {time.time() - t0:.1f} s", flush=True)
    U, pcs, thr = inputs()
    explored = np.zeros(len(prep.valid), dtype=bool)
    steps = []
    prof = None
    for i in range(N_STEPS + 1):
        if i == 0:
            d32 = np.zeros(24, np.float32)
        else:
            _, _, d32, _ = E.expert_system(pcs[i - 1], False, CORES, float(thr[i - 1]), 0.7)
        n_unexplored = int((~explored).sum()) - (0 if prof is None or explored[prof] else 1)
        r = SR.step(prep, explored, prof, d32, [int(U[i])], with_fp64=(i in (1, 2)))
        rec = {
            "pick": int(r.picks[0]),
            "pick_raw": int(prep.valid[r.picks[0]]),
            "total": str(r.total),
            "s_min": float(np.float32(r.s_min)) if i > 0 else 0.0,
            "s_max": float(np.float32(r.s_max)) if i > 0 else 0.0,
            "n_unexplored": n_unexplored,
            "n_active": int((d32 != 0).sum()),
        }
        if i in (0, 1, 2, 50, 100):
            rec["sha256_q_u32le"] = hashlib.sha256(r.q.astype("<u4").tobytes()).hexdigest()
            rec["sha256_s32_le"] = hashlib.sha256(r.s32.astype("<f4").tobytes()).hexdigest()
        if i in (1, 2):
            rec["max_abs_s32_minus_s64"] = float(np.max(np.abs(r.s32.astype(np.float64) - r.s64)))
        steps.append(rec)
        prof = r.picks[0]
        print(i, rec["pick"], rec["total"], f"{time.time() - t0:.0f}s", flush=True)
    out = {
        "_source": "oracle only; see tests/golden/make_search_golden.py",
        "n_valid": int(len(prep.valid)),
        "cores": CORES,
        "steps": steps,
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_search.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
