"""GPU least-squares polynomial models vs the oracle (Sect. 3.4.1): the
design, the coefficients of every subspace and counter, and the predictions
of every (or a sample of the) valid configurations.

Tolerances, derived per subspace s from the arithmetic.  The device sums the
Gram matrix A = F^T F + lam I in another order than the oracle's BLAS product
(relative differences up to (n_s + T) 2^-53) and factors it by Cholesky instead
of LU, so
- the device coefficients must satisfy the oracle's normal equations to
  1e-10 of |A| |beta| + |R| (both solvers are backward stable);
- fitted values at the training points must agree to 1e-10 of
  sum_t |F_t beta_t|: they do not see directions the design cannot identify;
- coefficients and predictions elsewhere may differ by up to
  kappa_s (n_s + T) 2^-53 of their scale (kappa_s = cond(A), large when
  constraints leave the design rank-deficient and the ridge fixes those
  directions), at least 1e-6 and at most 1e-2.
Predictions are evaluated in float32: each of the T terms is a product of at
most 4 rounded features times a rounded coefficient, accumulated in T steps,
so they may differ from the float64 values by 2 (T + 8) 2^-24 sum_t |F_t beta_t|
on top of the coefficients' share."""
import numpy as np
import pytest

import synth
from oracle import bounds as B
from oracle import lsq as LS
from oracle import space as SP
from tests.helpers import cgs

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def _space(spec):
    valid = SP.enumerate_valid(spec.radix, spec.values, spec.constraints)
    return valid, SP.digits_of(valid, spec.radix)


def _check(m, spec, digits, pts, Y, order, sample=None):
    sp = m.Space.from_spec(spec)
    print(f"poly fit: n={len(pts)} C={Y.shape[1]} order={order}", flush=True)
    model = m.PolyModel(sp, pts, Y, order)
    ref = LS.fit(spec.values, spec.radix, digits[pts], Y, order)
    beta = model.coefficients()
    assert beta.shape == ref.beta.shape
    assert model.report["pivot_clamped"] == 0
    T = len(ref.terms)
    F = LS.basis(LS.features(spec.values, spec.radix, digits[pts]), order)
    s_pts = LS.subspace(spec.radix, digits[pts])
    rtol = np.zeros(ref.n_subspaces)
    for k in range(ref.n_subspaces):
        rows = s_pts == k
        if not rows.any():
            assert (beta[k] == 0).all()
            continue
        Fk = F[rows]
        A = Fk.T @ Fk + ref.lam[k] * np.eye(T)
        R = Fk.T @ np.asarray(Y, np.float64)[rows]
        res = A @ beta[k] - R
        assert (np.abs(res) <= 1e-10 * (np.abs(A) @ np.abs(beta[k]) + np.abs(R)) + 1e-300).all(), k
        fit_gpu, fit_ref = Fk @ beta[k], Fk @ ref.beta[k]
        mag = np.abs(Fk) @ np.abs(ref.beta[k])
        assert (np.abs(fit_gpu - fit_ref) <= 1e-10 * mag + 1e-300).all(), k
        kappa = np.linalg.cond(A)
        rtol[k] = min(1e-2, max(1e-6, kappa * (rows.sum() + T) * 2.0 ** -53))
        scale = np.abs(ref.beta[k]).max(axis=0) + 1e-300
        assert (np.abs(beta[k] - ref.beta[k]) <= rtol[k] * scale).all(), (k, kappa)
    rows = np.arange(sp.n_valid) if sample is None else sample
    got = model.gather_predictions(rows) if sample is not None else model.copy_predictions()
    want = LS.predict(ref, spec.values, spec.radix, digits[rows])
    mag = LS.abs_terms(ref, spec.values, spec.radix, digits[rows])
    s_rows = LS.subspace(spec.radix, digits[rows])
    bound = 2 * (T + 8) * U * mag + rtol[s_rows][:, None] * mag
    assert (np.abs(got.astype(np.float64) - want) <= bound).all()
    # the training points: fitted values in float32 against the float64 ones
    fitted = model.gather_predictions(pts)
    want = LS.predict(ref, spec.values, spec.radix, digits[pts])
    mag = LS.abs_terms(ref, spec.values, spec.radix, digits[pts])
    assert (np.abs(fitted.astype(np.float64) - want) <= 2 * (T + 8) * U * mag + 1e-10 * mag).all()
    return model, ref


def test_design_equals_the_oracle():
    m = cgs()
    for spec in (synth.space_c1(), synth.space_c2(), synth.space_batch(63)):
        sp = m.Space.from_spec(spec)
        valid, digits = _space(spec)
        assert (m.PolyModel.design(sp) == LS.design(spec.values, spec.radix, digits)).all()


@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_c1_design_fit(order):
    m = cgs()
    spec = synth.space_c1()
    valid, digits = _space(spec)
    pts = LS.design(spec.values, spec.radix, digits).astype(np.uint32)
    Y = synth.measured_counters(synth.rng(30, order), digits[pts], spec.radix, 6)
    _check(m, spec, digits, pts, Y, order)


def test_c2_design_fit_order_three():
    """The 2^24 space: 3 binary parameters (8 subspaces), 9 non-binary, order
    3 (139 terms); the design's measured counters; predictions of 300,000
    sampled configurations."""
    m = cgs()
    spec = synth.space_c2()
    valid, digits = _space(spec)
    pts = LS.design(spec.values, spec.radix, digits).astype(np.uint32)
    Y = synth.measured_counters(synth.rng(31), digits[pts], spec.radix, 24)
    sample = np.sort(synth.rng(32).choice(len(valid), 300000, replace=False)).astype(np.uint32)
    model, ref = _check(m, spec, digits, pts, Y, 3, sample=sample)
    assert model.report["n_subspaces"] == 8 and model.report["n_terms"] == 139


def test_random_points_with_repeats_on_a_ragged_space():
    m = cgs()
    spec = synth.space_batch(63)
    valid, digits = _space(spec)
    g = synth.rng(33)
    pts = g.integers(0, len(valid), 40000).astype(np.uint32)
    Y = synth.measured_counters(g, digits[pts], spec.radix, 16)
    sample = np.sort(g.choice(len(valid), 100000, replace=False)).astype(np.uint32)
    _check(m, spec, digits, pts, Y, 2, sample=sample)


def test_binary_only_space_and_empty_subspaces():
    """No non-binary parameter: one term, the subspace mean; subspaces with no
    training point predict 0."""
    m = cgs()
    radix = [2, 2, 1, 2]
    values = [[0, 1], [0, 1], [5], [0, 1]]
    spec = synth.Space(radix, values, [])
    valid, digits = _space(spec)
    pts = np.array([0, 0, 1, 2, 3, 5, 5, 5], dtype=np.uint32)
    Y = synth.measured_counters(synth.rng(34), digits[pts], radix, 3)
    model, ref = _check(m, spec, digits, pts, Y, 2)
    trained = set(LS.subspace(radix, digits[pts]).tolist())
    assert trained == {0, 2, 4, 5, 6}      # subspace bit i = i-th binary parameter's digit
    P = model.copy_predictions()
    s = LS.subspace(radix, digits)
    assert (P[np.isin(s, [1, 3, 7])] == 0).all()


def _prediction_bounds(m, spec, digits, pts, Y, order, model):
    """Oracle prediction intervals of every valid configuration for the
    device's fit: the float64 polynomial values, widened by the bound the
    fit tests derive (conditioning of each subspace's normal equations plus
    float32 evaluation), clamped at 0 like the predictions."""
    ref = LS.fit(spec.values, spec.radix, digits[pts], Y, order)
    T = len(ref.terms)
    F = LS.basis(LS.features(spec.values, spec.radix, digits[pts]), order)
    s_pts = LS.subspace(spec.radix, digits[pts])
    rtol = np.full(ref.n_subspaces, 1e-6)
    for k in range(ref.n_subspaces):
        rows = s_pts == k
        if rows.any():
            A = F[rows].T @ F[rows] + ref.lam[k] * np.eye(T)
            rtol[k] = min(1e-2, max(1e-6, np.linalg.cond(A) * (rows.sum() + T) * 2.0 ** -53))
    v = LS.value(ref, spec.values, spec.radix, digits)
    mag = LS.abs_terms(ref, spec.values, spec.radix, digits)
    b = 2 * (T + 8) * U * mag + rtol[LS.subspace(spec.radix, digits)][:, None] * mag
    return v, np.maximum(v - b, 0.0), np.maximum(v + b, 0.0)


def _tiny_space():
    radix = [3, 4, 2, 3, 2, 4]
    return synth.Space(radix, synth.value_tables(radix, binary_radix2=True), [])


@pytest.mark.parametrize("which,order", [("tiny", 1), ("c1", 1), ("c1", 2)])
def test_scored_steps_on_a_polynomial_model(which, order):
    """Polynomials that go negative between the design points (predictions
    clamped at 0), scored steps from seeded states (explored sets, profiles,
    counter changes) and six draws each: every score, quantised weight and
    pick inside the oracle's intervals propagated from the prediction bound
    (oracle/bounds.py); picks that only one configuration can take are
    equal.  Reports the share of draws that could go to more than one: on
    the 576-configuration space most draws are certain, on the 11,496 one
    most are not (the bound of each prediction is summed over the space)."""
    m = cgs()
    spec = _tiny_space() if which == "tiny" else synth.space_c1()
    sp = m.Space.from_spec(spec)
    valid, digits = _space(spec)
    nv = len(valid)
    pts = LS.design(spec.values, spec.radix, digits).astype(np.uint32)
    Y = synth.measured_counters(synth.rng(35, order), digits[pts], spec.radix, 12)
    model = m.PolyModel(sp, pts, Y, order)
    v, lo, hi = _prediction_bounds(m, spec, digits, pts, Y, order, model)
    if which == "c1":
        assert (v < 0).any()                 # the clamp is exercised
    P = model.copy_predictions().astype(np.float64)
    assert ((P >= lo) & (P <= hi)).all() and P.min() >= 0.0
    g = synth.rng(36, order)
    certain = flagged = 0
    for state in range(6):
        explored = np.zeros(nv, bool)
        explored[synth.uniform_indices(g, int(g.integers(0, min(200, nv // 4))), nv)] = True
        prof = int(synth.uniform_indices(g, 1, nv)[0])
        delta = synth.deltas(g, 1, 12)[0]
        Us = synth.uniforms_u64(g, 6)
        sess = m.Session(sp)
        for l in np.flatnonzero(explored):
            sess.mark_explored(int(valid[l]))
        explored[prof] = True
        sess.search_step(model, int(valid[prof]), delta=delta)
        s = sess.copy_scores().astype(np.float64)
        q = sess.copy_weights().astype(np.uint64)
        s_lo, s_hi = B.score_interval(lo[prof], hi[prof], lo, hi, delta)
        un = ~explored
        assert ((s[un] >= s_lo[un]) & (s[un] <= s_hi[un])).all(), state
        w_lo, w_hi = B.weight_interval(s_lo, s_hi, explored)
        q_lo, q_hi = B.q_interval(w_lo, w_hi)
        assert ((q >= q_lo) & (q <= q_hi)).all(), state
        for U_ in Us:
            raw, l = sess.sample_next(int(U_))
            first, last, sure = B.feasible_picks(q_lo, q_hi, int(U_))
            assert first <= l <= last and q_hi[l] > 0 and raw == valid[l], (state, l, first, last)
            if not sure:
                flagged += 1
                break                        # later draws depend on this pick
            certain += 1
            assert l == first
            q_lo[l] = q_hi[l] = 0
    print(f"{which} order {order}: {certain} certain draws, {flagged} flagged", flush=True)
    assert certain + flagged >= 6
    if which == "tiny":
        assert certain >= flagged


def test_fit_errors():
    m = cgs()
    spec = synth.space_c2()
    sp = m.Space.from_spec(spec)
    pts = np.arange(10, dtype=np.uint32)
    Y = np.ones((10, 2), np.float32)
    with pytest.raises(m.CgsError) as ei:
        m.PolyModel(sp, pts, Y, 4)            # 265 terms for 9 non-binary parameters
    assert ei.value.status == m.ERANGE
    with pytest.raises(m.CgsError) as ei:
        m.PolyModel(sp, pts, Y, 5)
    assert ei.value.status == m.ERANGE
    bad = pts.copy()
    bad[4] = sp.n_valid
    with pytest.raises(m.CgsError) as ei:
        m.PolyModel(sp, bad, Y, 1)
    assert ei.value.status == m.EINVAL
    Yn = Y.copy()
    Yn[3, 1] = np.nan
    with pytest.raises(m.CgsError) as ei:
        m.PolyModel(sp, pts, Yn, 1)
    assert ei.value.status == m.EINVAL
