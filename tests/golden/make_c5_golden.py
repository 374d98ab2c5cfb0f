"""Writes c5_steps.json: the oracle's forest evaluation and first scored
steps on the 16-parameter space (2^14 * 3^8 = 107,495,424 raw
configurations), computed by the oracle only.  Run from the repository root:

    python tests/golden/make_c5_golden.py

Contents:
  * leaf ids (16 trees) and float32 predictions (32 counters) of the valid
    configurations in seeded runs of the valid list and its last 64, as
    SHA-256 of their little-endian bytes (sample order, leaf ids tree-major),
    with the first 8 configurations' values in plain;
  * a search of Alg. 1 with one draw per step: the uniform start (U[0]),
    then 3 scored steps, each profiling the last pick with counter changes
    that are non-zero for all 32 counters (so every prediction row enters
    the score): picks, totals, s_min / s_max, unexplored counts and SHA-256
    of the quantised weight vector and of the float32 scores of the unexplored
    configurations, before each draw.
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
from oracle import forest as F  # noqa: E402
from oracle import sampling as S  # noqa: E402
from oracle import score as SC  # noqa: E402
from oracle import space as SP  # noqa: E402

N_STEPS = 3
RUN = 512          # configurations per sampled run of the valid list
N_RUNS = 8
CHUNK = 1 << 21


def inputs(n_valid):
    """Seeded inputs of the golden (shared with the GPU test through synth)."""
    g = synth.rng(5, 20)
    U = synth.uniforms_u64(g, N_STEPS + 1)
    D = synth.deltas(g, N_STEPS, 32)
    D = np.where(D == 0, np.float32(0.5), D).astype(np.float32)   # every counter active
    starts = np.sort(synth.uniform_indices(synth.rng(5, 21), N_RUNS, n_valid - RUN))
    return U, D, starts


def main():
    t0 = time.time()
    spec = synth.space_c5()
    forest = synth.forest_c5(spec)
    valid = SP.enumerate_valid(spec.radix, spec.values, spec.constraints)
    nv = len(valid)
    print(f"{nv} valid configurations ({time.time() - t0:.0f} s)", flush=True)
    C = forest.leaves.shape[2]
    P32 = np.empty((nv, C), dtype=np.float32)
    U, D, starts = inputs(nv)
    sample = np.concatenate([np.arange(s, s + RUN) for s in starts] +
                            [np.arange(nv - 64, nv)])
    ids_sample = np.empty((forest.feat.shape[0], len(sample)), dtype=np.int64)
    for c0 in range(0, nv, CHUNK):
        c1 = min(nv, c0 + CHUNK)
        digits = SP.digits_of(valid[c0:c1].astype(np.int64), spec.radix)
        ids = F.leaf_ids(forest.feat, forest.thr, forest.depth, digits)
        P32[c0:c1] = F.predict_fp32(forest.leaves, ids)
        inside = (sample >= c0) & (sample < c1)
        ids_sample[:, inside] = ids[:, sample[inside] - c0]
        print(f"  forest {c1}/{nv} ({time.time() - t0:.0f} s)", flush=True)
    out = {
        "_source": "oracle only; see tests/golden/make_c5_golden.py",
        "n_valid": int(nv),
        "sample_starts": [int(s) for s in starts],
        "sample_run": RUN,
        "sha256_leaf_ids_u16le": hashlib.sha256(ids_sample.astype("<u2").tobytes()).hexdigest(),
        "sha256_predictions_f32le": hashlib.sha256(P32[sample].astype("<f4").tobytes()).hexdigest(),
        "leaf_ids_first8": ids_sample[:, :8].astype(int).tolist(),
        "predictions_first8": [[float(v) for v in row] for row in P32[sample[:8]]],
        "steps": [],
    }
    explored = np.zeros(nv, dtype=bool)
    prof = None
    for i in range(N_STEPS + 1):
        if prof is None:
            s32 = np.zeros(nv, dtype=np.float32)
        else:
            explored[prof] = True
            s32 = np.empty(nv, dtype=np.float32)
            for c0 in range(0, nv, CHUNK):
                c1 = min(nv, c0 + CHUNK)
                s32[c0:c1] = SC.score_fp32(P32[prof], P32[c0:c1], D[i - 1])
        w32, s_min, s_max = SC.weights_fp32(s32, explored)
        q = SC.quantize(w32)
        total = int(q.sum(dtype=np.uint64))
        l = S.pick(q, int(U[i]))
        out["steps"].append({
            "pick": int(l),
            "pick_raw": int(valid[l]),
            "total": str(total),
            "s_min": float(s_min) if prof is not None else 0.0,
            "s_max": float(s_max) if prof is not None else 0.0,
            "n_unexplored": int((~explored).sum()),
            "sha256_q_u32le": hashlib.sha256(q.astype("<u4").tobytes()).hexdigest(),
            "sha256_s32_unexplored_le":
                hashlib.sha256(s32[~explored].astype("<f4").tobytes()).hexdigest(),
        })
        explored[l] = True
        prof = l
        print(i, out["steps"][-1], f"({time.time() - t0:.0f} s)", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_steps.json")
    with open(path, "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
