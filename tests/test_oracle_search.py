"""Oracle pins: one search step of Alg. 1 composed end to end."""
import numpy as np

import synth
from oracle import forest as F
from oracle import sampling as S
from oracle import score as SC
from oracle import search as SR
from oracle import space as SP


def _prep_c1():
    sp = synth.space_c1()
    return sp, SR.prepare(sp, synth.forest_c1(sp))


def test_zero_bottleneck_is_uniform_random_search():
    sp, prep = _prep_c1()
    n = len(prep.valid)
    explored = np.zeros(n, dtype=bool)
    explored[[3, 10, 11]] = True
    un = np.flatnonzero(~explored)
    for U in [0, 1 << 63, (1 << 64) - 1, 12345678901234567890]:
        ex = explored.copy()
        r = SR.step(prep, ex, 3, np.zeros(12, np.float32), [U], with_fp64=False)
        assert (r.q[~explored] == 1 << 23).all() and (r.q[explored] == 0).all()
        assert r.picks[0] == un[(U * len(un)) >> 64]
        assert ex[r.picks[0]]


def test_only_unexplored_config_is_drawn():
    sp, prep = _prep_c1()
    n = len(prep.valid)
    explored = np.ones(n, dtype=bool)
    explored[777] = False
    d = synth.deltas(synth.rng(11), 1, 12)[0]
    for U in synth.uniforms_u64(synth.rng(12), 5):
        ex = explored.copy()
        assert SR.step(prep, ex, 0, d, [int(U)], with_fp64=False).picks == [777]
    ex = np.ones(n, dtype=bool)
    assert SR.step(prep, ex, 0, d, [5], with_fp64=False).picks == [None]


def test_step_matches_scalar_composition():
    """Composition check against the scalar definitions on a few draws."""
    sp, prep = _prep_c1()
    g = synth.rng(13)
    d = synth.deltas(g, 1, 12)[0]
    U = [int(x) for x in synth.uniforms_u64(g, 3)]
    explored = np.zeros(len(prep.valid), dtype=bool)
    explored[[0, 5]] = True
    r = SR.step(prep, explored.copy(), 5, d, U)
    # scalar float64 scores
    for i in range(0, len(prep.valid), 211):
        assert abs(r.s64[i] - SC.score_one(prep.P64[5], prep.P64[i], d)) < 1e-14
    # the picks are those of the stated draw rule on the quantised weights
    q = r.q.copy()
    for U_k, l in zip(U, r.picks):
        assert l == S.pick_scalar(q.tolist(), U_k)
        q[l] = 0
    # the float32 and float64 weight chains agree closely
    w64 = SC.normalize_fp64(r.s64, np.isin(np.arange(len(q)), [0, 5]))
    un = w64 > 0
    assert np.max(np.abs(r.w32[un] - w64[un]) / np.maximum(w64[un], 1)) < 1e-5


def test_picks_favour_high_scores():
    """Weighted draws land in the top-scored part far more often than uniform."""
    sp, prep = _prep_c1()
    d = synth.deltas(synth.rng(14), 1, 12)[0]
    explored = np.zeros(len(prep.valid), dtype=bool)
    r = SR.step(prep, explored.copy(), 0, d, [0])
    top = r.s32 >= np.quantile(r.s32, 0.9)
    U = synth.uniforms_u64(synth.rng(15), 400)
    hits = sum(top[S.pick(r.q, int(u))] for u in U)
    assert hits / len(U) > 0.5
