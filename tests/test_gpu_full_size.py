"""Full-size workloads against stored oracle results (written by
tests/golden/make_c5_golden.py and make_batch_golden.py, oracle only):

* the 16-parameter space (107,495,424 raw, 26,986,176 valid) with its forest
  of 16 depth-12 trees over 32 counters: leaf ids and predictions of sampled
  runs of the valid list, then the uniform start and three scored steps with
  every counter active: picks, totals, s_min / s_max and the SHA-256 of the
  weight vector and of the unexplored configurations' scores, bit for bit;
* the two largest batched sessions between 10^6 and 10^7 raw configurations,
  stepped inside the whole 64-session batch: their picks, totals and weight
  vectors after each draw equal the oracle's."""
import hashlib

import numpy as np
import pytest

import synth
from tests.helpers import cgs, golden

pytestmark = pytest.mark.gpu


def _sha(a, fmt):
    return hashlib.sha256(np.ascontiguousarray(a).astype(fmt).tobytes()).hexdigest()


def test_large_space_forest_and_scored_steps():
    m = cgs()
    ref = golden("c5_steps.json")
    spec = synth.space_c5()
    sp = m.Space.from_spec(spec)
    assert sp.n_valid == ref["n_valid"]
    model = m.ForestModel.from_spec(sp, synth.forest_c5(spec))
    run = ref["sample_run"]
    starts = ref["sample_starts"] + [sp.n_valid - 64]
    ids, P = [], []
    for k, s0 in enumerate(starts):
        n = run if k < len(ref["sample_starts"]) else 64
        ids.append(model.copy_leaf_ids(s0, n))
        P.append(model.copy_predictions(s0, n))
    ids = np.concatenate(ids, axis=1)
    P = np.concatenate(P, axis=0)
    assert (ids[:, :8] == np.asarray(ref["leaf_ids_first8"])).all()
    assert (P[:8] == np.asarray(ref["predictions_first8"], dtype=np.float32)).all()
    assert _sha(ids, "<u2") == ref["sha256_leaf_ids_u16le"]
    assert _sha(P, "<f4") == ref["sha256_predictions_f32le"]
    # the golden's inputs (synth only)
    g = synth.rng(5, 20)
    U = synth.uniforms_u64(g, 4)
    D = synth.deltas(g, 3, 32)
    D = np.where(D == 0, np.float32(0.5), D).astype(np.float32)
    sess = m.Session(sp)
    raw = None
    for i, r in enumerate(ref["steps"]):
        print(f"large space: step {i}", flush=True)
        if i == 0:
            sess.search_step(model, m.NO_PROFILE)
        else:
            sess.search_step(model, raw, delta=D[i - 1])
        q = sess.copy_weights()
        assert _sha(q, "<u4") == r["sha256_q_u32le"], i
        s = sess.copy_scores()
        assert _sha(s[q > 0], "<f4") == r["sha256_s32_unexplored_le"], i
        raw, l = sess.sample_next(int(U[i]))
        assert (l, raw) == (r["pick"], r["pick_raw"]), i
        info = sess.step_info()
        assert info.total_weight == int(r["total"]) and info.n_unexplored == r["n_unexplored"]
        if i:
            assert info.s_min == np.float32(r["s_min"]) and info.s_max == np.float32(r["s_max"])
            assert info.n_active == 32


def test_large_batched_sessions_match_the_oracle():
    m = cgs()
    ref = golden("batch_large.json")
    n_sess, n_steps = 64, 10
    specs = [synth.space_batch(s) for s in range(n_sess)]
    spaces = [m.Space.from_spec(sp) for sp in specs]
    models = [m.ForestModel.from_spec(spc, synth.forest_batch(s, sp))
              for s, (sp, spc) in enumerate(zip(specs, spaces))]
    sessions = [m.Session(spc) for spc in spaces]
    batch = m.Batch(sessions, models)
    g = synth.rng(4, 3, 0)
    D = synth.deltas(g, n_steps * n_sess, 16).reshape(n_steps, n_sess, 16)
    U = synth.uniforms_u64(g, (n_steps + 1) * n_sess).reshape(n_steps + 1, n_sess)
    prof = [m.NO_PROFILE] * n_sess
    for k in range(4):
        print(f"batch: step {k}", flush=True)
        raw, val, st = batch.step(prof, D[k - 1] if k else None, U[k])
        assert (st == 0).all()
        for s, rs in ref["sessions"].items():
            s = int(s)
            r = rs["steps"][k]
            assert spaces[s].n_raw == rs["n_raw"] and spaces[s].n_valid == rs["n_valid"]
            assert (int(val[s]), int(raw[s])) == (r["pick"], r["pick_raw"]), (s, k)
            assert sessions[s].step_info().total_weight == int(r["total"]), (s, k)
            assert _sha(sessions[s].copy_weights(), "<u4") == r["sha256_q_after_draw_u32le"], (s, k)
        prof = [int(x) for x in raw]
