"""Pins of the interval propagation (oracle/bounds.py) that carries a
model's prediction error bound through the score equation, the
normalisation, the quantisation and the draw (Sect. 3.6, Alg. 1).

The intervals must hold every float32 result the step can compute from
predictions inside the bounds: checked by brute force (the oracle's float32
chain on predictions sampled inside the bounds, corners included) and by
enumerating every integer weight vector of small boxes for the draw; plus
hand-worked cases and the degenerate case of exact predictions."""
import itertools

import numpy as np
import pytest

from oracle import bounds as B
from oracle import sampling as S
from oracle import score as SC

U = 2.0 ** -24


def test_single_counter_hand_cases():
    pad = (1 + 5) * U
    s_lo, s_hi = B.score_interval([1.0], [1.0], [[2.0], [0.0], [0.0]], [[4.0], [1.0], [0.0]],
                                  np.float32([1.0]))
    # x in [2, 4] against a = 1: t = (x - 1) / (x + 1) in [1/3, 3/5]
    assert np.isclose(s_lo[0], 1 / 3 - pad, rtol=0, atol=1e-15)
    assert np.isclose(s_hi[0], 3 / 5 + pad, rtol=0, atol=1e-15)
    # x in [0, 1]: 0 drops the term, x -> 0+ gives -1, x = 1 gives 0
    assert np.isclose(s_lo[1], -1 - pad, atol=1e-15) and np.isclose(s_hi[1], pad, atol=1e-15)
    # x == 0: exactly no term (and no rounding)
    assert s_lo[2] == 0.0 and s_hi[2] == 0.0
    # a negative change reverses the interval
    s_lo, s_hi = B.score_interval([1.0], [1.0], [[2.0]], [[4.0]], np.float32([-0.5]))
    assert np.isclose(s_lo[0], -0.3 - 0.5 * pad, atol=1e-15)
    assert np.isclose(s_hi[0], -1 / 6 + 0.5 * pad, atol=1e-15)
    # no change, or a profile predicted 0: the score is exactly 0
    for a, d in (([1.0], [0.0]), ([0.0], [1.0])):
        s_lo, s_hi = B.score_interval(a, a, [[2.0]], [[4.0]], np.float32(d))
        assert s_lo[0] == 0.0 and s_hi[0] == 0.0


def test_weight_spot_values():
    s = np.array([0.5, 0.0, -0.2, 0.25, -1.0])
    w_lo, w_hi = B.weight_interval(s, s, np.zeros(5, bool))
    want = [256.0, 1.0, (1 - 0.2) ** 8, 1.5 ** 8, float(np.float32(1e-4))]
    for lo, hi, w in zip(w_lo, w_hi, want):
        assert lo <= w <= hi and hi - lo <= 64 * U * w * 1.0001
    # explored configurations weigh exactly 0
    w_lo, w_hi = B.weight_interval(s, s, np.array([1, 0, 0, 0, 0], bool))
    assert w_lo[0] == 0.0 and w_hi[0] == 0.0


def test_draw_hand_cases():
    # exact weights 1, 2, 3 and r = floor(Q / 2) = 3: the third is picked
    assert B.feasible_picks([1, 2, 3], [1, 2, 3], 1 << 63) == (2, 2, True)
    # the second weight may be 3: Q in [6, 7], r = 3, so l = 1 or 2
    assert B.feasible_picks([1, 2, 3], [1, 3, 3], 1 << 63) == (1, 2, False)
    # U = 0 picks the first non-zero weight
    assert B.feasible_picks([0, 5, 1], [0, 5, 1], 0) == (1, 1, True)
    assert B.feasible_picks([0, 0], [0, 0], 123) == (None, None, True)


@pytest.mark.parametrize("seed", range(6))
def test_draw_range_holds_every_integer_weight_choice(seed):
    """Enumerate every integer q with q_lo <= q <= q_hi on small boxes: each
    resulting pick lies in the feasible range, and a certain range names the
    only pick."""
    g = np.random.default_rng(seed)
    for _ in range(40):
        n = int(g.integers(1, 5))
        q_lo = g.integers(0, 6, n).astype(np.uint64)
        q_hi = q_lo + g.integers(0, 3, n).astype(np.uint64)
        Uv = int(g.integers(0, 2 ** 63)) * 2 + int(g.integers(0, 2))
        first, last, certain = B.feasible_picks(q_lo, q_hi, Uv)
        seen = set()
        for q in itertools.product(*[range(int(a), int(b) + 1) for a, b in zip(q_lo, q_hi)]):
            seen.add(S.pick(np.array(q, np.uint64), Uv))
        seen.discard(None)
        for l in seen:
            assert first <= l <= last
        if certain and first is not None:
            assert seen == {first}


def _case(g, n, C):
    """Random prediction bounds with exact zeros, tiny values and wide
    intervals, a profile interval, changes and an explored set."""
    base = g.uniform(0.0, 2.0, (n, C))
    base[g.random((n, C)) < 0.1] = 0.0
    base[g.random((n, C)) < 0.05] *= 1e-6
    width = base * 10.0 ** g.uniform(-7, -2, (n, C))
    width[g.random((n, C)) < 0.05] = 0.0
    X_lo = np.maximum(base - width, 0.0)
    X_hi = base + width
    X_lo[g.random((n, C)) < 0.05] = 0.0     # a prediction that may be clamped to 0
    X_lo[0, g.integers(0, C)] = 0.0         # the profile's too
    a_lo, a_hi = X_lo[0], X_hi[0]
    d = g.uniform(-1, 1, C).astype(np.float32)
    d[g.random(C) < 0.2] = 0.0
    explored = g.random(n) < 0.1
    explored[0] = True                       # the profile itself
    return a_lo, a_hi, X_lo, X_hi, d, explored


def _sample(g, lo, hi):
    """float32 values inside [lo, hi]: random interior points, the corners
    (rounded inward) and 0 where 0 is inside."""
    lo32 = np.float32(lo)
    lo32 = np.where(lo32.astype(np.float64) < lo, np.nextafter(lo32, np.float32(np.inf)), lo32)
    hi32 = np.float32(hi)
    hi32 = np.where(hi32.astype(np.float64) > hi, np.nextafter(hi32, np.float32(-np.inf)), hi32)
    pick = g.integers(0, 3, np.shape(lo))
    mid = np.float32(lo + (hi - lo) * g.random(np.shape(lo)))
    mid = np.clip(mid, lo32, hi32)
    return np.where(pick == 0, lo32, np.where(pick == 1, hi32, mid)).astype(np.float32)


@pytest.mark.parametrize("seed", range(8))
def test_brute_force_float32_chain_stays_inside(seed):
    g = np.random.default_rng(100 + seed)
    n, C = 400, 7
    a_lo, a_hi, X_lo, X_hi, d, explored = _case(g, n, C)
    s_lo, s_hi = B.score_interval(a_lo, a_hi, X_lo, X_hi, d)
    w_lo, w_hi = B.weight_interval(s_lo, s_hi, explored)
    q_lo, q_hi = B.q_interval(w_lo, w_hi)
    Us = [int(x) * 2 + 1 for x in g.integers(0, 2 ** 63, 4)]
    ranges = []
    qq_lo, qq_hi = q_lo.copy(), q_hi.copy()
    for Uv in Us:
        r = B.feasible_picks(qq_lo, qq_hi, Uv)
        ranges.append(r)
        if not r[2] or r[0] is None:
            break
        qq_lo[r[0]] = qq_hi[r[0]] = 0        # removal of a certain pick
    for trial in range(60):
        a = _sample(g, a_lo, a_hi)
        X = _sample(g, X_lo, X_hi)
        s = SC.score_fp32(a, X, d)
        assert ((s >= s_lo) & (s <= s_hi)).all(), trial
        w, _, _ = SC.weights_fp32(s, explored)
        assert ((w >= w_lo) & (w <= w_hi)).all(), trial
        q = SC.quantize(w)
        assert ((q >= q_lo) & (q <= q_hi)).all(), trial
        picks = S.draws(q, Us[:len(ranges)])
        for l, (first, last, certain) in zip(picks, ranges):
            if first is None:
                assert l is None
                continue
            assert first <= l <= last
            if certain:
                assert l == first


def test_exact_predictions_give_narrow_intervals_and_certain_picks():
    """Degenerate prediction intervals (the float32 predictions themselves):
    the float32 chain lies inside intervals of rounding width, and at this
    size every draw is certain and equals the oracle's pick."""
    g = np.random.default_rng(7)
    n, C = 300, 6
    X = g.uniform(0.1, 1.0, (n, C)).astype(np.float32)
    d = g.uniform(-1, 1, C).astype(np.float32)
    explored = np.zeros(n, bool)
    explored[0] = True
    Xd = X.astype(np.float64)
    s_lo, s_hi = B.score_interval(Xd[0], Xd[0], Xd, Xd, d)
    s = SC.score_fp32(X[0], X, d)
    assert ((s >= s_lo) & (s <= s_hi)).all()
    assert (s_hi - s_lo).max() <= 2 * (C + 5) * U * np.abs(d).sum() * 1.0001
    w_lo, w_hi = B.weight_interval(s_lo, s_hi, explored)
    q_lo, q_hi = B.q_interval(w_lo, w_hi)
    q = SC.quantize(SC.weights_fp32(s, explored)[0])
    certain = 0
    for Uv in [int(x) * 2 for x in g.integers(0, 2 ** 63, 50)]:
        first, last, c = B.feasible_picks(q_lo, q_hi, int(Uv))
        l = S.pick(q, int(Uv))
        assert first <= l <= last
        certain += c
        if c:
            assert l == first
    assert certain >= 45


def test_weight_rounding_slack():
    """Exact float32 scores (degenerate score intervals): the float32
    normalisation rounds, and the weight interval still holds its result."""
    g = np.random.default_rng(11)
    for _ in range(20):
        s = np.float32(g.uniform(-1.5, 2.0, 5000))
        s[g.random(5000) < 0.05] = 0.0
        explored = g.random(5000) < 0.1
        w, _, _ = SC.weights_fp32(s, explored)
        w_lo, w_hi = B.weight_interval(s.astype(np.float64), s.astype(np.float64), explored)
        assert ((w >= w_lo) & (w <= w_hi)).all()
