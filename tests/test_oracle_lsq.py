"""Oracle pins: least-squares polynomial models per binary subspace
(Sect. 3.4.1)."""
import itertools
import math

import numpy as np
import pytest

from oracle import lsq as LS


def _grid(radix):
    return np.array(list(itertools.product(*[range(r) for r in radix])), dtype=np.int64)


def test_term_counts():
    for k in range(0, 7):
        for order in range(0, 5):
            T = sum(math.comb(k, i) for i in range(min(order, k) + 1)) + k
            assert len(LS.terms(k, order)) == T
    assert LS.terms(3, 2) == [(), (0,), (1,), (2,), (0, 1), (0, 2), (1, 2), (0, 0), (1, 1), (2, 2)]


def test_roles_subspace_and_features_by_hand():
    radix = [2, 3, 1, 2, 4]
    values = [[0, 1], [1, 2, 4], [7], [32, 64], [-3, 0, 3, 9]]
    assert LS.roles(radix) == ([0, 3], [1, 4])
    d = np.array([[1, 2, 0, 0, 1], [0, 0, 0, 1, 3], [1, 1, 0, 1, 0]])
    assert LS.subspace(radix, d).tolist() == [1, 2, 3]
    x = LS.features(values, radix, d)
    # x = (2v - vmax - vmin) / (vmax - vmin): (8-5)/3 = 1, (2-5)/3 = -1, (4-5)/3
    # and (0-6)/12, (18-6)/12, (-6-6)/12
    assert np.allclose(x, [[1.0, -0.5], [-1.0, 1.0], [-1.0 / 3.0, -1.0]], rtol=0, atol=1e-15)


def test_mid_digit_and_design_by_hand():
    assert LS.mid_digit([1, 2, 4, 8, 16, 32, 64, 128]) == 6      # 64 is nearest 64.5
    assert LS.mid_digit([1, 2, 4]) == 1                           # 2 is nearest 2.5
    assert LS.mid_digit([0, 10, 20, 30]) == 1                     # tie 10 / 20: the lower
    radix = [4, 2, 3]
    values = [[0, 10, 20, 30], [0, 1], [1, 2, 4]]
    d = _grid(radix)
    got = LS.design(values, radix, d)
    want = [i for i, r in enumerate(d) if r[0] in (0, 1, 3)]
    assert got.tolist() == want


def _space(seed, n_bin=2, nb_radix=(3, 4, 5)):
    g = np.random.default_rng(seed)
    radix = [2] * n_bin + list(nb_radix)
    perm = g.permutation(len(radix))
    radix = [radix[i] for i in perm]
    values = [sorted(g.choice(np.arange(1, 200), r, replace=False).tolist()) for r in radix]
    return g, radix, values


@pytest.mark.parametrize("seed,order", [(0, 1), (1, 2), (2, 3), (3, 3)])
def test_recovers_a_polynomial_in_its_basis(seed, order):
    """Targets that are an exact polynomial of the basis, measured on the
    design: the fit returns its coefficients and predicts every configuration
    of the full space."""
    g, radix, values = _space(seed)
    d = _grid(radix)
    _, nb = LS.roles(radix)
    S, T, C = 4, len(LS.terms(len(nb), order)), 3
    truth = g.standard_normal((S, T, C))
    F = LS.basis(LS.features(values, radix, d), order)
    Y = np.einsum("nt,ntc->nc", F, truth[LS.subspace(radix, d)])
    des = LS.design(values, radix, d)
    m = LS.fit(values, radix, d[des], Y[des], order)
    assert np.allclose(m.beta, truth, rtol=1e-5, atol=1e-5)
    assert np.allclose(LS.value(m, values, radix, d), Y, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("seed", range(4))
def test_matches_numpy_lstsq_on_noisy_data(seed):
    g, radix, values = _space(10 + seed)
    d = _grid(radix)
    Y = g.standard_normal((len(d), 4)) * [1.0, 100.0, 1e-3, 7.0]
    m = LS.fit(values, radix, d, Y, 2)
    F = LS.basis(LS.features(values, radix, d), 2)
    s = LS.subspace(radix, d)
    for k in range(m.n_subspaces):
        ref = np.linalg.lstsq(F[s == k], Y[s == k], rcond=None)[0]
        assert np.allclose(m.beta[k], ref, rtol=1e-6, atol=1e-7 * np.abs(ref).max())


def test_binary_only_space_predicts_subspace_means():
    radix = [2, 2, 1, 2]
    values = [[0, 1], [0, 1], [5], [0, 1]]
    d = _grid(radix)
    g = np.random.default_rng(3)
    idx = g.integers(0, len(d), 200)
    Y = g.standard_normal((200, 2))
    m = LS.fit(values, radix, d[idx], Y, 3)
    assert len(m.terms) == 1
    s = LS.subspace(radix, d[idx])
    for k in range(8):
        assert np.allclose(m.beta[k, 0], Y[s == k].mean(axis=0), rtol=1e-8, atol=1e-12)


def test_three_levels_interpolate_the_quadratic():
    """One parameter with three values and order 1: basis {1, x, x^2}
    through three points is Lagrange interpolation."""
    radix, values = [3], [[1, 2, 4]]
    d = _grid(radix)
    y = np.array([[3.0], [-1.0], [10.0]])
    m = LS.fit(values, radix, d, y, 1)
    assert np.allclose(LS.value(m, values, radix, d), y, rtol=1e-7)
    # value at x = 0 from the Lagrange form through x = -1, -1/3, 1
    xs = [-1.0, -1.0 / 3.0, 1.0]
    lag = sum(y[i, 0] * np.prod([(0 - xs[j]) / (xs[i] - xs[j]) for j in range(3) if j != i])
              for i in range(3))
    assert np.isclose(m.beta[0, 0, 0], lag, rtol=1e-7)
    # predicted counters are the values clamped at 0: the negative middle
    # value becomes exactly 0, the others are unchanged
    p = LS.predict(m, values, radix, d)
    assert p[1, 0] == 0.0 and np.allclose(p[[0, 2]], y[[0, 2]], rtol=1e-7)


def test_rank_deficient_design_approaches_the_minimum_norm_solution():
    radix, values = [4, 3], [[1, 2, 3, 4], [1, 5, 9]]
    d = _grid(radix)[[0, 5]]                  # two points, 2 + 2 + 1 + 2 = 6 terms at order 2
    y = np.array([[1.0], [2.0]])
    m = LS.fit(values, radix, d, y, 2)
    F = LS.basis(LS.features(values, radix, d), 2)
    ref = np.linalg.pinv(F) @ y
    assert np.allclose(m.beta[0], ref, rtol=1e-3, atol=1e-4)
    assert np.allclose(LS.value(m, values, radix, d), y, rtol=1e-6)


def test_normalisation_does_not_change_predictions():
    """The basis span is closed under per-parameter affine maps: fitting on
    raw values gives the same predictions as on the normalised features."""
    g, radix, values = _space(20, nb_radix=(3, 4))
    d = _grid(radix)
    Y = g.standard_normal((len(d), 2))
    m = LS.fit(values, radix, d, Y, 2)
    _, nb = LS.roles(radix)
    raw = np.stack([np.asarray(values[j], float)[d[:, j]] for j in nb], axis=1)
    Fr = LS.basis(raw, 2)
    s = LS.subspace(radix, d)
    pred = np.empty_like(Y)
    for k in range(4):
        b = np.linalg.lstsq(Fr[s == k], Y[s == k], rcond=None)[0]
        pred[s == k] = Fr[s == k] @ b
    assert np.allclose(LS.value(m, values, radix, d), pred, rtol=1e-6, atol=1e-6)


def test_empty_subspace_has_zero_coefficients():
    radix, values = [2, 3], [[0, 1], [1, 2, 3]]
    d = _grid(radix)
    d = d[d[:, 0] == 0]
    m = LS.fit(values, radix, d, np.ones((len(d), 1)), 1)
    assert m.count.tolist() == [3, 0] and (m.beta[1] == 0).all()
