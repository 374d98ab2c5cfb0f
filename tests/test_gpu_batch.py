"""Batched sessions: one step over many independent searches gives, in every
session, the scores, weights and picks of the single-session step (which the
other tests pin to the oracle), and for small sessions the oracle's picks
directly."""
import numpy as np
import pytest

import synth
from oracle import search as SR
from tests.helpers import cgs

pytestmark = pytest.mark.gpu

SESSIONS = (3, 7, 11, 21, 40, 44, 52, 61, 63)   # 10^4 .. 10^6 raw configurations


def _build(m, ids, params=None):
    specs = [synth.space_batch(s) for s in ids]
    spaces = [m.Space.from_spec(sp) for sp in specs]
    models = [m.ForestModel.from_spec(spc, synth.forest_batch(s, sp))
              for s, sp, spc in zip(ids, specs, spaces)]
    sessions = [m.Session(spc, params) for spc in spaces]
    return specs, spaces, models, sessions


def _inputs(n_sess, n_steps, seed):
    g = synth.rng(4, 3, seed)
    return synth.deltas(g, n_steps * n_sess, 16).reshape(n_steps, n_sess, 16), \
        synth.uniforms_u64(g, (n_steps + 1) * n_sess).reshape(n_steps + 1, n_sess)


# (graph replay, score-pass variant: counter rows in flight x waves per SIMD)
@pytest.mark.parametrize("use_graph,variant", [(1, 0), (0, 0), (1, 2), (0, 4)])
def test_batch_equals_single_sessions(use_graph, variant):
    m = cgs()
    ids = SESSIONS
    _, spaces, models, sess_b = _build(m, ids)
    _, _, models_s, sess_s = _build(m, ids)
    sched = m.cgs_batch_schedule(512, 256, use_graph, variant)
    batch = m.Batch(sess_b, models, sched)
    D, U = _inputs(len(ids), 6, 1)
    prof_b = [m.NO_PROFILE] * len(ids)
    prof_s = [m.NO_PROFILE] * len(ids)
    for step in range(7):
        raw, val, st = batch.step(prof_b, D[step - 1] if step else None, U[step])
        assert (st == 0).all()
        for i in range(len(ids)):
            if step == 0:
                sess_s[i].search_step(models_s[i], m.NO_PROFILE)
            else:
                sess_s[i].search_step(models_s[i], prof_s[i], delta=D[step - 1][i])
            r = sess_s[i].sample_next(int(U[step][i]))
            assert (int(raw[i]), int(val[i])) == r, (step, i)
            if step in (1, 5):
                assert (sess_b[i].copy_scores() == sess_s[i].copy_scores()).all()
                assert (sess_b[i].copy_weights() == sess_s[i].copy_weights()).all()
                ib, is_ = sess_b[i].step_info(), sess_s[i].step_info()
                assert (ib.s_min, ib.s_max, ib.n_unexplored, ib.total_weight) == \
                    (is_.s_min, is_.s_max, is_.n_unexplored, is_.total_weight)
            prof_s[i] = r[0]
        prof_b = [int(x) for x in raw]
        assert batch.step_ms() > 0


def test_small_sessions_match_the_oracle():
    m = cgs()
    ids = [s for s in range(64) if synth.space_batch(s).n_raw <= 60000][:6]
    assert len(ids) >= 3
    specs, spaces, models, sessions = _build(m, ids)
    batch = m.Batch(sessions, models)
    preps = [SR.prepare(sp, synth.forest_batch(s, sp)) for s, sp in zip(ids, specs)]
    explored = [np.zeros(len(p.valid), dtype=bool) for p in preps]
    D, U = _inputs(len(ids), 5, 2)
    prof = [None] * len(ids)
    profiles = [m.NO_PROFILE] * len(ids)
    for step in range(6):
        raw, val, st = batch.step(profiles, D[step - 1] if step else None, U[step])
        for i in range(len(ids)):
            d = D[step - 1][i] if step else np.zeros(16, np.float32)
            ref = SR.step(preps[i], explored[i], prof[i], d, [int(U[step][i])], with_fp64=False)
            assert int(val[i]) == ref.picks[0], (step, i)
            prof[i] = ref.picks[0]
        profiles = [int(x) for x in raw]


def test_autotune_keeps_search_state_and_caches(tmp_path):
    m = cgs()
    ids = SESSIONS[:5]
    _, _, models, sess_b = _build(m, ids)
    _, _, models_s, sess_s = _build(m, ids)
    batch = m.Batch(sess_b, models)
    D, U = _inputs(len(ids), 3, 3)
    raw, _, _ = batch.step([m.NO_PROFILE] * len(ids), None, U[0])
    for i in range(len(ids)):
        sess_s[i].search_step(models_s[i], m.NO_PROFILE)
        sess_s[i].sample_next(int(U[0][i]))
    cache = str(tmp_path / "tune.txt")
    sched = batch.autotune(cache)
    assert sched.score_grid >= 1 and sched.weight_grid >= 1
    assert open(cache).read().count("->") == 1
    again = batch.autotune(cache)                    # served from the cache
    assert (again.score_grid, again.weight_grid) == (sched.score_grid, sched.weight_grid)
    assert open(cache).read().count("->") == 1
    prof = [int(x) for x in raw]
    for step in range(1, 3):
        raw, val, st = batch.step(prof, D[step - 1], U[step])
        for i in range(len(ids)):
            sess_s[i].search_step(models_s[i], prof[i], delta=D[step - 1][i])
            assert sess_s[i].sample_next(int(U[step][i])) == (int(raw[i]), int(val[i]))
        prof = [int(x) for x in raw]


def test_exhausted_session_reports_empty():
    m = cgs()
    spec = synth.Space([2, 2], [[1, 2], [1, 2]], [])
    big = synth.space_batch(3)
    spaces = [m.Space.from_spec(spec), m.Space.from_spec(big)]
    models = [m.ForestModel.from_spec(spaces[0], synth.random_forest(synth.rng(90), [2, 2], 1, 2, 16)),
              m.ForestModel.from_spec(spaces[1], synth.forest_batch(3, big))]
    sessions = [m.Session(s) for s in spaces]
    batch = m.Batch(sessions, models)
    U = synth.uniforms_u64(synth.rng(91), 12).reshape(6, 2)
    seen = set()
    prof = [m.NO_PROFILE, m.NO_PROFILE]
    for step in range(6):
        deltas = [np.full(16, 0.5, np.float32), np.full(16, -0.5, np.float32)]
        raw, val, st = batch.step(prof, deltas if step else None, U[step])
        if step < 4:
            assert st[0] == 0 and int(val[0]) not in seen
            seen.add(int(val[0]))
        else:
            assert st[0] == m.EEMPTY
        assert st[1] == 0
        prof = [int(raw[0]) if st[0] == 0 else m.NO_PROFILE, int(raw[1])]
