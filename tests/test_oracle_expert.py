"""Oracle pins: bottleneck analysis and reaction (Sect. 3.5)."""
import json
import os

import numpy as np
import pytest

from oracle import expert as E
from oracle import forest as F
from oracle import score as SC
from oracle import search as SR
from oracle import space as SP

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "expert_hand_computed.json")


def _cases():
    g = json.load(open(GOLDEN))
    return g, g["cases"]


@pytest.mark.parametrize("idx", range(6))
def test_hand_computed_cases(idx):
    g, cases = _cases()
    case = cases[idx]
    pc = np.zeros(24)
    for k, v in case["pc"].items():
        pc[g["counters"].index(k)] = v
    B, d64, d32, dthr = E.expert_system(pc, case["volta"], case["cores"], case["threads"],
                                        case["inst_reaction"])
    expB = np.zeros(18)
    for k, v in case["B"].items():
        expB[g["bottlenecks"].index(k)] = v
    expD = np.zeros(24)
    for k, v in case["delta"].items():
        expD[g["counters"].index(k)] = v
    assert np.allclose(B, expB, rtol=0, atol=1e-12), (B, expB)
    assert np.allclose(d64, expD, rtol=0, atol=1e-12), (d64, expD)
    assert abs(dthr - case["delta_threads"]) < 1e-12
    assert (d32 == d64.astype(np.float32)).all()


def test_ranges():
    import synth
    pcs = synth.profiler_counters(synth.rng(77), 200)
    thr = synth.threads_launched(synth.rng(78), 200)
    for i in range(200):
        B, d, _, _ = E.expert_system(pcs[i], cores=2048.0, threads=thr[i])
        assert (B >= 0).all() and (B <= 1).all()
        assert (d >= -1).all() and (d <= 1).all()
        # only memory, instruction, issue and SM_E counters ever get a change
        untouched = [E.INST_EXE, E.DRAM_U, E.L2_U, E.TEX_U, E.SHR_U, E.WARP_E, E.WARP_NP_E]
        assert (d[untouched] == 0).all()


def test_section2_example_direction():
    """Sect. 2.2: texture cache at 9/10 and FP units at 3/10 with Z_ITERATIONS = 1;
    raising Z_ITERATIONS lowers texture traffic and FP instructions.  The
    searcher must favour larger Z_ITERATIONS."""
    radix = [6]                                 # Z_ITERATIONS in {1,2,4,8,16,32}
    values = [[1, 2, 4, 8, 16, 32]]
    # one-parameter tree, depth 3: leaves 0..5 reached by digits 0..5
    feat = np.zeros((1, 7), dtype=np.uint8)
    thr = np.array([[2, 0, 4, 255, 1, 3, 5]], dtype=np.uint8)
    digits = np.arange(6)[:, None]
    ids = F.leaf_ids(feat, thr, 3, digits)[0]
    assert len(set(ids.tolist())) == 6
    C = 24
    leaves = np.full((1, 8, C), 0.5, dtype=np.float32)
    for d in range(6):
        z = values[0][d]
        leaves[0, ids[d], E.TEX_RWT] = 1.0 / z
        leaves[0, ids[d], E.INST_F32] = 1.0 / z ** 0.5
    pc = np.zeros(24)
    pc[E.TEX_U] = 9.0
    pc[E.INST_EXE] = 1000
    pc[E.WARP_E] = pc[E.WARP_NP_E] = 100
    pc[E.INST_F32] = 0.3 * 32000
    pc[E.INST_ISSUE_U] = 100
    pc[E.SM_E] = 100
    _, _, delta, _ = E.expert_system(pc, cores=1, threads=5)
    assert delta[E.TEX_RWT] == np.float32(-0.9)
    P32 = F.predict_fp32(leaves, ids[None, :])
    s = SC.score_fp32(P32[0], P32, delta)
    explored = np.zeros(6, dtype=bool)
    explored[0] = True
    w, _, _ = SC.weights_fp32(s, explored)
    assert (np.diff(w[1:]) > 0).all() and np.argmax(w) == 5
