"""Writes batch_large.json: the oracle's first steps of the two largest
batched sessions between 10^6 and 10^7 raw configurations (sessions 34 and
7 of the 64-session batch: 8,503,056 and 9,765,625 raw), with the batch's
own seeded inputs, computed by the oracle only.  Run from the repository
root:

    python tests/golden/make_batch_golden.py

Inputs are those of the 64-session batch workload (synth.rng(4, 3, 0)):
counter changes D[step][session][16] and uniforms U[step][session].  Per
session: the uniform start with U[0], then 3 scored steps, each profiling
the last pick; picks, totals and SHA-256 of the quantised weight vector as
the step leaves it after its draw (the pick's weight is 0).
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
from oracle import search as SR  # noqa: E402

SESSIONS = (34, 7)
N_SESS = 64
N_STEPS = 3
BATCH_STEPS = 10        # the batch workload's step count (shapes its input arrays)


def inputs():
    g = synth.rng(4, 3, 0)
    D = synth.deltas(g, BATCH_STEPS * N_SESS, 16).reshape(BATCH_STEPS, N_SESS, 16)
    U = synth.uniforms_u64(g, (BATCH_STEPS + 1) * N_SESS).reshape(BATCH_STEPS + 1, N_SESS)
    return D, U


def main():
    t0 = time.time()
    D, U = inputs()
    out = {"_source": "oracle only; see tests/golden/make_batch_golden.py", "sessions": {}}
    for s in SESSIONS:
        spec = synth.space_batch(s)
        prep = SR.prepare(spec, synth.forest_batch(s, spec))
        explored = np.zeros(len(prep.valid), dtype=bool)
        prof = None
        steps = []
        for k in range(N_STEPS + 1):
            d = D[k - 1][s] if k else np.zeros(16, np.float32)
            r = SR.step(prep, explored, prof, d, [int(U[k][s])], with_fp64=False)
            l = r.picks[0]
            q = r.q.copy()
            q[l] = 0
            steps.append({"pick": int(l), "pick_raw": int(prep.valid[l]), "total": str(r.total),
                          "sha256_q_after_draw_u32le":
                              hashlib.sha256(q.astype("<u4").tobytes()).hexdigest()})
            prof = l
            print(s, k, steps[-1], f"({time.time() - t0:.0f} s)", flush=True)
        out["sessions"][str(s)] = {"n_raw": int(spec.n_raw), "n_valid": int(len(prep.valid)),
                                   "steps": steps}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_large.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
