"""Oracle pins: enumeration and constraint pruning (Sect. 1; TS of Alg. 1)."""
import itertools

import numpy as np
import pytest

import synth
from oracle import space as SP


def test_hand_example_divisibility():
    # values {1,2,4} x {1,2,4}, v0 % v1 == 0  <=>  digit0 >= digit1 (worked by hand)
    radix = [3, 3]
    values = [[1, 2, 4], [1, 2, 4]]
    cons = [("DIV", 0, 1, 0, 0)]
    assert SP.enumerate_bruteforce(radix, values, cons) == [0, 3, 4, 6, 7, 8]
    assert SP.enumerate_valid(radix, values, cons).tolist() == [0, 3, 4, 6, 7, 8]


def test_hand_example_each_kind():
    radix = [3, 2, 2]
    values = [[2, 3, 8], [0, 1], [1, 4]]
    # expected sets below were worked out by hand from the value tables
    configs = list(itertools.product(range(3), range(2), range(2)))
    vals = [[values[j][d] for j, d in enumerate(c)] for c in configs]
    # DIV by a zero value fails; v0 % v1 with v1 == 1 passes
    exp_div = [k for k, v in enumerate(vals) if v[1] == 1]
    assert SP.enumerate_bruteforce(radix, values, [("DIV", 0, 1, 0, 0)]) == exp_div
    # DIV2: v0 % (v1*v2): only v1 == 1 and (v2 == 1 or v0 == 8)
    exp_div2 = [k for k, v in enumerate(vals) if v[1] == 1 and (v[2] == 1 or v[0] == 8)]
    assert SP.enumerate_bruteforce(radix, values, [("DIV2", 0, 1, 2, 0)]) == exp_div2
    # PROD_LE v0*v2 <= 8: (2,1),(2,4),(3,1),(8,1)
    exp_le = [k for k, v in enumerate(vals) if (v[0], v[2]) in {(2, 1), (2, 4), (3, 1), (8, 1)}]
    assert SP.enumerate_bruteforce(radix, values, [("PROD_LE", 0, 2, 0, 8)]) == exp_le
    # PROD_GE v0*v2 >= 12: (3,4),(8,4)
    exp_ge = [k for k, v in enumerate(vals) if (v[0], v[2]) in {(3, 4), (8, 4)}]
    assert SP.enumerate_bruteforce(radix, values, [("PROD_GE", 0, 2, 0, 12)]) == exp_ge
    # PROD3_LE v0*v1*v2 <= 3: v1 == 0 always, or (2,1,1), (3,1,1)
    exp_p3 = [k for k, v in enumerate(vals) if v[1] == 0 or (v[0] in (2, 3) and v[2] == 1)]
    assert SP.enumerate_bruteforce(radix, values, [("PROD3_LE", 0, 1, 2, 3)]) == exp_p3
    # LE v2 <= v0: v2 == 1, or v2 == 4 with v0 == 8
    exp_lt = [k for k, v in enumerate(vals) if v[2] == 1 or v[0] == 8]
    assert SP.enumerate_bruteforce(radix, values, [("LE", 2, 0, 0, 0)]) == exp_lt


def test_decode_order_matches_itertools_product():
    radix = [3, 1, 4, 2]
    for k, digits in enumerate(itertools.product(*[range(r) for r in radix])):
        assert SP.decode(k, radix) == list(digits)
    ks = np.arange(int(np.prod(radix)))
    assert SP.digits_of(ks, radix).tolist() == [list(d) for d in itertools.product(*[range(r) for r in radix])]


@pytest.mark.parametrize("seed", range(12))
def test_vectorised_matches_bruteforce(seed):
    g = np.random.default_rng(seed)
    n_params = int(g.integers(1, 5))
    radix = [int(g.integers(1, 5)) for _ in range(n_params)]
    values = [sorted(g.choice(np.arange(0, 9), size=r, replace=False).tolist()) for r in radix]
    cons = []
    for _ in range(int(g.integers(0, 4))):
        kind = str(g.choice(synth.CONSTRAINT_KINDS))
        a, b, c = (int(x) for x in g.integers(0, n_params, size=3))
        cons.append((kind, a, b, c, int(g.integers(0, 40))))
    brute = SP.enumerate_bruteforce(radix, values, cons)
    assert SP.enumerate_valid(radix, values, cons).tolist() == brute
    # chunked evaluation gives the same mask
    m1 = SP.valid_mask(radix, values, cons)
    m2 = SP.valid_mask(radix, values, cons, chunk=3)
    assert (m1 == m2).all()


def test_raw_sizes_closed_form():
    assert synth.space_c1().n_raw == 4 * 4 * 5 * 6 * 8 * 8 == 30720
    assert synth.space_c2().n_raw == 2 ** 24
    assert synth.space_c5().n_raw == 2 ** 14 * 3 ** 8 == 107495424


def test_c1_survival_in_paper_range():
    sp = synth.space_c1()
    v = SP.enumerate_valid(sp.radix, sp.values, sp.constraints)
    # paper's benchmarks keep 0.025 % - 41.7 % of the cross product (Sect. 4.6)
    assert 0.30 <= len(v) / sp.n_raw <= 0.45
    assert v.tolist() == SP.enumerate_bruteforce(sp.radix, sp.values, sp.constraints)


def test_mask_words_bit_order():
    m = np.zeros(70, dtype=bool)
    m[[0, 5, 31, 32, 69]] = True
    w = SP.mask_words(m)
    assert w.tolist() == [(1 << 0) | (1 << 5) | (1 << 31), 1 << 0, 1 << 5]
