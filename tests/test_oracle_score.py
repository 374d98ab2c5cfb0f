"""Oracle pins: score and score normalisation (Sect. 3.6)."""
import numpy as np
import pytest

from oracle import score as SC

U32 = 2.0 ** -24


def test_single_counter_hand_example():
    # profile a = 1, candidate x = 3, increase wanted (dpc = +1): (3 - 1) / (1 + 3) = +0.5
    assert SC.score_one([1.0], [3.0], [1.0]) == 0.5
    assert SC.score_fp64(np.array([1.0]), np.array([[3.0]]), np.array([1.0]))[0] == 0.5
    # decrease wanted: the same candidate scores -0.5
    assert SC.score_one([1.0], [3.0], [-1.0]) == -0.5


def test_two_counter_hand_example():
    # -1 * (3-1)/(1+3) + 0.5 * (1-4)/(4+1) = -0.5 - 0.3
    s = SC.score_one([1.0, 4.0], [3.0, 1.0], [-1.0, 0.5])
    assert abs(s + 0.8) < 1e-15
    # a candidate lowering counter 0 (wanted) and raising counter 1 (wanted) scores > 0
    s = SC.score_one([1.0, 4.0], [0.5, 6.0], [-1.0, 0.5])
    assert abs(s - (1.0 / 3.0 + 0.1)) < 1e-15


def test_pc_used_excludes_zero_predictions():
    # p0 both non-zero (t = 0), p1 a = 0 excluded, p2 x = 0 excluded
    a = np.array([2.0, 0.0, 1.0])
    X = np.array([[2.0, 5.0, 0.0]])
    d = np.array([1.0, 1.0, 1.0])
    assert SC.score_fp64(a, X, d)[0] == 0.0
    assert SC.score_fp32(a, X, d)[0] == 0.0
    # without the exclusion p1 would contribute -1 and p2 +1: use unequal deltas
    d2 = np.array([1.0, 3.0, 0.25])
    assert SC.score_fp64(a, X, d2)[0] == 0.0


def _random_case(seed, n=500, C=12):
    g = np.random.default_rng(seed)
    a = g.random(C).astype(np.float32)
    X = g.random((n, C)).astype(np.float32)
    X[g.random((n, C)) < 0.05] = 0.0
    d = (g.random(C) * 2 - 1).astype(np.float32)
    return a, X, d


@pytest.mark.parametrize("seed", range(4))
def test_invariants(seed):
    a, X, d = _random_case(seed)
    s = SC.score_fp64(a, X, d)
    # profiled configuration scores 0
    assert SC.score_fp64(a, a[None, :], d)[0] == 0.0
    # antisymmetric in dPC
    assert np.allclose(SC.score_fp64(a, X, -d), -s, rtol=0, atol=1e-15)
    # each term lies in [-|d_p|, |d_p|] for non-negative counters
    assert (np.abs(s) <= np.abs(d.astype(np.float64)).sum() + 1e-12).all()
    # swapping candidate and profile flips the sign
    for i in range(0, 50, 7):
        assert abs(SC.score_one(X[i], a, d) + SC.score_one(a, X[i], d)) < 1e-14
    # vectorised equals the scalar loop
    for i in range(0, len(X), 37):
        assert abs(s[i] - SC.score_one(a, X[i], d)) < 1e-14


@pytest.mark.parametrize("seed", range(4))
def test_fp32_chain_within_rounding_bound(seed):
    a, X, d = _random_case(seed)
    s64 = SC.score_fp64(a, X, d)
    s32 = SC.score_fp32(a, X, d).astype(np.float64)
    C = len(d)
    bound = (C + 4) * U32 * np.abs(d.astype(np.float64)).sum()
    assert (np.abs(s32 - s64) <= bound).all()


def test_zero_bottleneck_gives_zero_scores_and_unit_weights():
    a, X, _ = _random_case(9)
    d = np.zeros_like(a)
    s = SC.score_fp32(a, X, d)
    assert (s == 0).all()
    w, _, _ = SC.weights_fp32(s, np.zeros(len(s), dtype=bool))
    assert (w == 1.0).all()


def test_normalisation_spot_values():
    # s_max = 0.4, s_min = -0.3
    smin, smax = -0.3, 0.4
    assert SC.normalize_one(0.4, smin, smax) == 256.0
    assert SC.normalize_one(0.2, smin, smax) == 1.5 ** 8 == 25.62890625
    assert SC.normalize_one(0.0, smin, smax) == 1.0
    assert SC.normalize_one(-0.25, smin, smax) == 1e-4          # at gamma: cut off
    assert SC.normalize_one(-0.3, smin, smax) == 1e-4
    # above the cut-off, negative scores are scaled by s_min: (1 - (-0.1)/(-0.2))^8
    assert SC.normalize_one(-0.1, -0.2, smax) == 0.5 ** 8 == 0.00390625
    # s = s_min > gamma: (1 - 1)^8 = 0 -> clipped to 1e-4
    assert SC.normalize_one(-0.2, -0.2, smax) == 1e-4
    # no positive scores: s = 0 -> 1 even when s_min = 0
    assert SC.normalize_one(0.0, 0.0, 0.0) == 1.0


def test_normalisation_range_and_monotone():
    g = np.random.default_rng(3)
    s = np.sort(g.uniform(-0.6, 0.9, 2000))
    explored = np.zeros(len(s), dtype=bool)
    w = SC.normalize_fp64(s, explored)
    assert w.min() >= 1e-4 and w.max() == 256.0
    assert (np.diff(w) >= 0).all()
    explored[::3] = True
    w2 = SC.normalize_fp64(s, explored)
    assert (w2[explored] == 0).all()


def test_weights_fp32_match_fp64_definition():
    g = np.random.default_rng(5)
    s = g.uniform(-0.6, 0.9, 3000).astype(np.float32)
    s[::17] = 0.0
    explored = g.random(3000) < 0.1
    w32, smin, smax = SC.weights_fp32(s, explored)
    w64 = SC.normalize_fp64(s.astype(np.float64), explored)
    # y = 1 +- s/s_ext carries at most 2 roundings (|dy| <= 2u * max(y, 1)), the eighth
    # power multiplies that by 8 y^7, and the 3 squarings add 3u: |dw| <= 24u * max(w, 1)
    u = 2.0 ** -24
    assert (np.abs(w32.astype(np.float64) - w64) <= 24 * u * np.maximum(w64, 1.0)).all()
    assert float(smin) == s[~explored].min() and float(smax) == s[~explored].max()


def test_quantize_exact_values_and_half_even():
    w = np.array([1.0, 256.0, 1e-4, 0.0, 0.5 + 2.0 ** -24, 0.5 + 3 * 2.0 ** -24], dtype=np.float32)
    q = SC.quantize(w)
    assert q.tolist() == [1 << 23, 1 << 31, 839, 0, 1 << 22, (1 << 22) + 2]
