"""Oracle pins: weighted random draw with removal (Sect. 3.7, Alg. 1)."""
import numpy as np
import pytest
from scipy import stats

from oracle import sampling as S

TWO64 = 1 << 64


def test_equal_weights_closed_form():
    g = np.random.default_rng(1)
    for n in (1, 3, 16, 1000, 12345):
        q = np.full(n, 1 << 23, dtype=np.uint64)
        for U in [0, TWO64 - 1] + [int(x) for x in g.integers(0, 2 ** 63, 20)] * 2:
            assert S.pick(q, U) == (U * n) >> 64


def test_first_and_last_nonzero():
    q = np.array([0, 0, 5, 0, 7, 1, 0, 0], dtype=np.uint64)
    assert S.pick(q, 0) == 2
    assert S.pick(q, TWO64 - 1) == 5
    assert S.pick(np.zeros(4, dtype=np.uint64), 123) is None


def test_interval_rule_by_hand():
    # q = [3, 0, 5, 2]: cumulative [3, 3, 8, 10]; r = floor(U*10/2^64)
    q = np.array([3, 0, 5, 2], dtype=np.uint64)
    for r, expect in [(0, 0), (2, 0), (3, 2), (7, 2), (8, 3), (9, 3)]:
        U = -(-(r << 64) // 10)           # smallest U with floor(U*10/2^64) = r
        assert (U * 10) >> 64 == r
        assert S.pick(q, U) == expect
        assert S.pick_scalar(q.tolist(), U) == expect


def test_vectorised_matches_linear_scan():
    g = np.random.default_rng(2)
    for _ in range(50):
        n = int(g.integers(1, 60))
        q = g.integers(0, 2 ** 31, n, dtype=np.uint64)
        q[g.random(n) < 0.3] = 0
        U = int(g.integers(0, 2 ** 63)) * 2 + int(g.integers(0, 2))
        assert S.pick(q, U) == S.pick_scalar(q.tolist(), U)


def test_removal_never_repeats_and_exhausts():
    q = np.array([4, 0, 1, 9, 2], dtype=np.uint64)
    g = np.random.default_rng(3)
    U = [int(x) for x in g.integers(0, 2 ** 63, 6)]
    picks = S.draws(q, U)
    assert picks[-1] is None
    got = [p for p in picks if p is not None]
    assert sorted(got) == [0, 2, 3, 4] and len(set(got)) == 4


def test_chi_square_matches_weights():
    g = np.random.default_rng(4)
    q = g.integers(1, 1 << 20, 16, dtype=np.uint64)
    U = g.integers(0, np.iinfo(np.uint64).max, 100000, dtype=np.uint64, endpoint=True)
    counts = np.zeros(16)
    for u in U:
        counts[S.pick(q, int(u))] += 1
    expected = q.astype(np.float64) / q.astype(np.float64).sum() * len(U)
    p = stats.chisquare(counts, expected).pvalue
    assert p > 0.01
