"""Oracle pins: neighbourhood-restricted step (Sect. 3.7, footnote to the
scoring line of Alg. 1)."""
import itertools
import math

import numpy as np
import pytest

import synth
from oracle import neighbourhood as NB
from oracle import search as SR
from oracle import space as SP
from tests.helpers import random_small_space


def test_hand_example():
    """Radices (3, 2), profile digits (1, 0) = raw 2: changing parameter 0
    gives digits (0, 0) and (2, 0) = raw 0 and 4; changing parameter 1 gives
    (1, 1) = raw 3; radius 2 adds (0, 1) and (2, 1) = raw 1 and 5."""
    assert NB.ball([3, 2], [1, 0], 1).tolist() == [0, 4, 3]
    assert NB.ball([3, 2], [1, 0], 2).tolist() == [0, 4, 3, 1, 5]


@pytest.mark.parametrize("seed", range(8))
def test_ball_is_the_hamming_ball_in_candidate_order(seed):
    g = np.random.default_rng(seed)
    radix = [int(r) for r in g.integers(1, 5, g.integers(2, 6))]
    n = int(np.prod(radix))
    for radius in (1, 2, 3):
        prof = int(g.integers(0, n))
        pd = SP.decode(prof, radix)
        brute = []
        for k, d in enumerate(itertools.product(*[range(r) for r in radix])):
            diff = [j for j in range(len(radix)) if d[j] != pd[j]]
            if 1 <= len(diff) <= radius:
                brute.append(((len(diff), tuple(diff), tuple(d[j] for j in diff)), k))
        brute.sort()
        got = NB.ball(radix, pd, radius)
        assert got.tolist() == [k for _, k in brute]
        assert NB.ball_size(radix, radius) == len(brute)


def test_ball_size_closed_forms():
    # binary parameters: sum of binomials; uniform radix r: C(P, d) (r - 1)^d
    for P in (1, 5, 12, 32):
        for h in (1, 2, 3):
            assert NB.ball_size([2] * P, h) == sum(math.comb(P, d) for d in range(1, h + 1))
            assert NB.ball_size([5] * P, h) == sum(math.comb(P, d) * 4 ** d for d in range(1, h + 1))
    assert NB.ball_size([1, 1, 1], 2) == 0


def _prepared(seed):
    """seed None: the 30,720-configuration space and its tree; otherwise a
    random small space (constraints, zero and negative values)."""
    if seed is None:
        spec = synth.space_c1()
        return spec, SR.prepare(spec, synth.forest_c1(spec))
    while True:
        radix, values, cons = random_small_space(np.random.default_rng(seed), 6, 5)
        spec = synth.Space(radix, values, cons)
        valid = SP.enumerate_valid(spec.radix, spec.values, spec.constraints)
        if len(valid) >= 8:
            break
        seed += 1000
    forest = synth.random_forest(synth.rng(90, seed), spec.radix, 3, 4, 12)
    return spec, SR.prepare(spec, forest)


@pytest.mark.parametrize("seed", [None, 0, 1, 2, 3])
def test_full_radius_scores_and_weights_equal_the_full_step(seed):
    """Radius = number of parameters: the neighbourhood is the whole space
    without the profile, so scores, weights and Q equal the full step's."""
    spec, prep = _prepared(seed)
    g = np.random.default_rng(7 if seed is None else seed)
    delta = synth.deltas(synth.rng(91, 7 if seed is None else seed), 1, 12)[0]
    prof = int(g.integers(0, len(prep.valid)))
    ex_full = np.zeros(len(prep.valid), dtype=bool)
    ex_nb = ex_full.copy()
    full = SR.step(prep, ex_full, prof, delta, [], with_fp64=False)
    nb = NB.step(prep, spec.radix, ex_nb, prof, delta, [], len(spec.radix))
    assert sorted(nb.cand.tolist()) == [l for l in range(len(prep.valid)) if l != prof]
    assert (nb.s32 == full.s32[nb.cand]).all()
    assert (nb.q == full.q[nb.cand]).all()
    assert nb.total == full.total
    assert nb.s_min == full.s_min and nb.s_max == full.s_max


def test_zero_delta_is_uniform_over_candidates():
    spec, prep = _prepared(None)
    ex = np.zeros(len(prep.valid), dtype=bool)
    r = NB.step(prep, spec.radix, ex, 0, np.zeros(12, np.float32), [], 2)
    assert len(r.cand) > 0 and (r.q == 1 << 23).all()


def test_draws_stay_in_the_neighbourhood_until_exhausted():
    spec, prep = _prepared(None)
    ex = np.zeros(len(prep.valid), dtype=bool)
    prof = 0
    pd = prep.digits[prof]
    U = synth.uniforms_u64(synth.rng(92), 400)
    delta = synth.deltas(synth.rng(93), 1, 12)[0]
    r = NB.step(prep, spec.radix, ex, prof, delta, U, 1)
    picks = [p for p in r.picks if p is not None]
    assert r.picks[-1] is None and len(picks) == len(r.cand)
    assert len(set(picks)) == len(picks) and set(picks) == set(r.cand.tolist())
    for p in picks:
        assert 1 <= int((prep.digits[p] != pd).sum()) <= 1
    # the same step again: every neighbour explored, nothing to draw
    r2 = NB.step(prep, spec.radix, ex, prof, delta, U[:3], 1)
    assert len(r2.cand) == 0 and r2.total == 0 and r2.picks == [None]
