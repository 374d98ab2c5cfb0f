"""Oracle pins: the searcher's outer loop (Alg. 1, Sect. 3.7) and the
evaluation measure (Sect. 4.1)."""
import itertools

import numpy as np
import pytest

import synth
from oracle import search as SR
from oracle import space as SP
from oracle import tuning as TU


def _table_prep(spec, table):
    valid = SP.enumerate_valid(spec.radix, spec.values, spec.constraints)
    digits = SP.digits_of(valid, spec.radix)
    P = table.counters.copy()
    return SR.Prepared(valid, digits, None, P, P.astype(np.float32))


def _small():
    radix = [3, 4, 2, 5, 3]
    values = [[1, 2, 4], [1, 2, 4, 8], [0, 1], [1, 2, 4, 8, 16], [1, 2, 4]]
    spec = synth.Space(radix, values, [])
    valid = SP.enumerate_valid(spec.radix, spec.values, spec.constraints)
    table = synth.kernel_table(synth.rng(41), SP.digits_of(valid, radix), radix)
    return spec, table


def test_random_search_closed_form_against_sampling():
    spec, table = _small()
    N = len(table.runtime)
    K = int(TU.well_performing(table.runtime).sum())
    g = np.random.default_rng(0)
    tests = [TU.random_search(table.runtime, g.permutation(N)) for _ in range(20000)]
    mean, se = np.mean(tests), np.std(tests) / np.sqrt(len(tests))
    assert abs(mean - TU.random_search_expected(table.runtime)) < 4 * se
    assert TU.random_search_expected(table.runtime) == (N + 1) / (K + 1)


def test_trajectory_structure():
    """Profiled run, then n draws; the next profiled configuration is the
    fastest of those draws (the later one on a tie); no configuration is
    drawn twice or after being profiled."""
    spec, table = _small()
    prep = _table_prep(spec, table)
    for seed in range(5):
        U = synth.uniforms_u64(synth.rng(42, seed), 4000)
        r = TU.run(prep, table.runtime, table.counters, U, draws=4, stop_at_well=False)
        t, p = r.tested, r.profiled
        starts = [i for i in range(len(t)) if p[i]]
        assert starts[0] == 0
        blocks = [t[a + 1:b] for a, b in zip(starts, starts[1:] + [len(t)])]
        drawn = set()
        for k, block in enumerate(blocks):
            assert len(block) <= 4
            assert len(block) == 4 or k >= len(blocks) - 2       # short only at exhaustion
            for l in block:
                assert l not in drawn and l != t[0]
                drawn.add(l)
            if k + 1 < len(blocks) and block:
                best = min(block, key=lambda l: (table.runtime[l], -block.index(l)))
                assert t[starts[k + 1]] == best
        # the space is exhausted: every configuration was tested
        assert set(t) == set(range(len(table.runtime)))


def test_constant_model_is_random_search():
    """With every prediction equal, every score is 0 and every draw uniform:
    the first well-performing configuration is found, on average, after
    (N + 1) / (K + 1) distinct configurations."""
    spec, table = _small()
    prep = _table_prep(spec, table)
    flat = np.ones_like(prep.P64)
    prep = SR.Prepared(prep.valid, prep.digits, None, flat, flat.astype(np.float32))
    well = TU.well_performing(table.runtime)
    distinct = []
    for seed in range(2000):
        U = synth.uniforms_u64(synth.rng(43, seed), 1000)
        r = TU.run(prep, table.runtime, table.counters, U)
        seen = []
        for l in r.tested:
            if l not in seen:
                seen.append(l)
                if well[l]:
                    break
        distinct.append(len(seen))
    mean, se = np.mean(distinct), np.std(distinct) / np.sqrt(len(distinct))
    assert abs(mean - TU.random_search_expected(table.runtime)) < 4 * se


def test_counting_stops_at_the_first_well_performing_test():
    spec, table = _small()
    prep = _table_prep(spec, table)
    well = TU.well_performing(table.runtime)
    U = synth.uniforms_u64(synth.rng(44), 4000)
    full = TU.run(prep, table.runtime, table.counters, U, stop_at_well=False)
    first = next(i for i, l in enumerate(full.tested) if well[l]) + 1
    r = TU.run(prep, table.runtime, table.counters, U)
    assert r.tests_to_well == first == len(r.tested) == full.tests_to_well
    cut = TU.run(prep, table.runtime, table.counters, U, max_tests=7, stop_at_well=False)
    assert cut.tested == full.tested[:7]


def test_counter_guidance_beats_random_search_on_the_synthetic_kernel():
    """Sect. 4.3's claim on the synthetic kernel, with the measured counters
    as the model: fewer tests than random search on average.  A sign error
    in the score or the counter changes would steer towards the bottleneck
    and lose to random search."""
    spec = synth.space_c1()
    valid = SP.enumerate_valid(spec.radix, spec.values, spec.constraints)
    table = synth.kernel_table(synth.rng(9, 1), SP.digits_of(valid, spec.radix), spec.radix)
    prep = _table_prep(spec, table)
    res = [TU.run(prep, table.runtime, table.counters,
                  synth.uniforms_u64(synth.rng(45, r), 20000)).tests_to_well for r in range(30)]
    assert np.mean(res) < TU.random_search_expected(table.runtime) / 2
