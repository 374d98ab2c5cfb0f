"""GPU regression-tree fitting vs the oracle (Sect. 3.4.2): training half,
quantisation scales, every cut depth's exact test errors, the selected depth,
the emitted tree and the fitted model's predictions, all bit-exact."""
import numpy as np
import pytest

import synth
from oracle import forest as F
from oracle import space as SP
from oracle import treefit as TF
from tests.helpers import cgs

pytestmark = pytest.mark.gpu


def _space_digits(spec):
    valid = SP.enumerate_valid(spec.radix, spec.values, spec.constraints)
    return valid, SP.digits_of(valid, spec.radix)


def _check(m, sp, spec, digits_valid, points, Y, keys, depth, min_leaf):
    print(f"fit: n={len(points)} C={Y.shape[1]} D={depth} min_leaf={min_leaf}", flush=True)
    model, rep = m.ForestModel.fit(sp, points, Y, keys, depth, min_leaf)
    ref = TF.fit(digits_valid[points], Y, keys, spec.radix, depth, min_leaf)
    assert rep["n_train"] == int(ref.train.sum()) and rep["n_test"] == int((~ref.train).sum())
    assert rep["scale_log2"] == ref.s.tolist()
    assert rep["abs_err"] == ref.A and rep["sq_err"] == ref.B
    assert rep["depth"] == ref.depth
    assert rep["n_split"] == int(ref.grown.split.sum())
    feat, thr, leaves = model.copy_forest()
    assert (feat == ref.feat).all() and (thr == ref.thr).all()
    assert (leaves == ref.leaves).all()
    # the fitted model predicts every valid configuration like the evaluator
    ids = F.leaf_ids(ref.feat, ref.thr, ref.depth, digits_valid)
    want = F.predict_fp32(ref.leaves, ids)
    got = model.copy_predictions()
    assert (got == want).all()
    return model, rep, ref


@pytest.mark.parametrize("n,C,depth,min_leaf", [
    (5000, 6, 6, 1), (5000, 6, 8, 3), (1537, 12, 4, 1), (4000, 3, 0, 1), (4000, 3, 1, 1),
    (2, 4, 3, 1), (3, 4, 3, 1), (700, 5, 14, 1)])
def test_fit_on_c1_matches_the_oracle(n, C, depth, min_leaf):
    m = cgs()
    spec = synth.space_c1()
    sp = m.Space.from_spec(spec)
    valid, digits = _space_digits(spec)
    assert (sp.copy_valid() == valid).all()
    g = synth.rng(20, n, C, depth)
    points = g.integers(0, len(valid), n).astype(np.uint32)
    Y = synth.measured_counters(g, digits[points], spec.radix, C)
    keys = synth.uniforms_u64(g, n)
    _check(m, sp, spec, digits, points, Y, keys, depth, min_leaf)


def test_fit_on_a_ragged_space_with_many_counters():
    """498,750 valid configurations of 8-14 parameters with constraints; 60,000
    points (repeats included) and 24 counters, depth 8."""
    m = cgs()
    spec = synth.space_batch(63)
    sp = m.Space.from_spec(spec)
    valid, digits = _space_digits(spec)
    g = synth.rng(21)
    points = g.integers(0, len(valid), 60000).astype(np.uint32)
    Y = synth.measured_counters(g, digits[points], spec.radix, 24)
    keys = synth.uniforms_u64(g, len(points))
    _check(m, sp, spec, digits, points, Y, keys, 8, 2)


def test_wide_rows_and_radix_one_parameters():
    """32 parameters (20 of radix 2, 12 of radix 1) and 64 counters: the
    widest (parameter, counter) item set the histogram kernel handles."""
    m = cgs()
    radix = [2 if j % 8 < 5 else 1 for j in range(32)]
    values = [list(range(r)) for r in radix]
    spec = synth.Space(radix, values, [])
    sp = m.Space(radix, values, [])
    valid, digits = _space_digits(spec)
    g = synth.rng(22)
    points = g.integers(0, len(valid), 3000).astype(np.uint32)
    Y = synth.measured_counters(g, digits[points], radix, 64)
    _check(m, sp, spec, digits, points, Y, synth.uniforms_u64(g, 3000), 5, 1)


def test_radix_sixteen_parameters():
    m = cgs()
    radix = [16, 16, 16, 3, 16]
    values = [list(range(r)) for r in radix]
    spec = synth.Space(radix, values, [])
    sp = m.Space(radix, values, [])
    valid, digits = _space_digits(spec)
    g = synth.rng(23)
    points = g.integers(0, len(valid), 20000).astype(np.uint32)
    Y = synth.measured_counters(g, digits[points], radix, 7)
    _check(m, sp, spec, digits, points, Y, synth.uniforms_u64(g, len(points)), 7, 1)


def test_degenerate_inputs():
    """Constant targets never split; one configuration measured many times
    cannot split; tied keys are ordered by point index."""
    m = cgs()
    spec = synth.space_c1()
    sp = m.Space.from_spec(spec)
    valid, digits = _space_digits(spec)
    g = synth.rng(24)
    points = g.integers(0, len(valid), 999).astype(np.uint32)
    zeros = np.zeros((999, 3), np.float32)
    keys = synth.uniforms_u64(g, 999)
    _, rep, _ = _check(m, sp, spec, digits, points, zeros, keys, 5, 1)
    assert rep["depth"] == 0 and rep["n_split"] == 0 and rep["abs_err"] == [0] * 6
    same = np.full(500, 17, np.uint32)
    Y = synth.measured_counters(g, digits[same], spec.radix, 4)
    _, rep, _ = _check(m, sp, spec, digits, same, Y, synth.uniforms_u64(g, 500), 4, 1)
    assert rep["n_split"] == 0
    tied = (keys[:999] & np.uint64(0xFFFF000000000000)) | np.uint64(5)
    Y = synth.measured_counters(g, digits[points], spec.radix, 4)
    _check(m, sp, spec, digits, points, Y, tied, 6, 2)


def test_fit_errors():
    m = cgs()
    spec = synth.space_c1()
    sp = m.Space.from_spec(spec)
    n_valid = sp.n_valid
    pts = np.arange(10, dtype=np.uint32)
    Y = np.ones((10, 2), np.float32)
    keys = np.arange(10, dtype=np.uint64)
    bad = pts.copy()
    bad[3] = n_valid
    cases = [
        ((bad, Y, keys, 3, 1), m.EINVAL),
        ((pts, np.where(np.arange(20).reshape(10, 2) == 7, np.nan, Y).astype(np.float32), keys, 3, 1), m.EINVAL),
        ((pts, np.where(np.arange(20).reshape(10, 2) == 7, np.inf, Y).astype(np.float32), keys, 3, 1), m.EINVAL),
        ((pts[:1], Y[:1], keys[:1], 3, 1), m.ERANGE),
        ((pts, Y, keys, 15, 1), m.ERANGE),
        ((pts, Y, keys, 3, 0), m.ERANGE),
        ((pts, Y, keys, 3, 11), m.ERANGE),
    ]
    for args, status in cases:
        with pytest.raises(m.CgsError) as ei:
            m.ForestModel.fit(sp, *args)
        assert ei.value.status == status
    model, rep = m.ForestModel.fit(sp, pts, Y, keys, 3, 1)
    assert rep["n_train"] == 5 and rep["n_test"] == 5


def test_full_space_fit_top_levels_match_the_oracle():
    """Every one of the 4,813,824 valid configurations of the 2^24 space
    measured once, 24 counters, depth 12: the root split, the depth-1 node
    values and the test errors of the depth-0 and depth-1 cuts equal the
    oracle's (greedy growth does not look ahead, so the top of the tree does
    not depend on the maximum depth); the fitted model predicts every
    configuration exactly as the evaluator does with the emitted tree."""
    m = cgs()
    spec = synth.space_c2()
    sp = m.Space.from_spec(spec)
    valid, digits = _space_digits(spec)
    n = len(valid)
    g = synth.rng(25)
    points = np.arange(n, dtype=np.uint32)
    Y = synth.measured_counters(g, digits, spec.radix, 24)
    keys = synth.uniforms_u64(g, n)
    print("fit: full space", flush=True)
    model, rep = m.ForestModel.fit(sp, points, Y, keys, 12, 4)
    tr = TF.train_half(keys)
    s = TF.scales(Y)
    q = TF.quantise(Y, s)
    assert rep["n_train"] == int(tr.sum()) and rep["scale_log2"] == s.tolist()
    top = TF.grow(digits[tr], q[tr], spec.radix, 1, 4)
    A, B = TF.candidate_errors(top, digits[~tr], q[~tr])
    assert rep["abs_err"][:2] == A and rep["sq_err"][:2] == B
    feat, thr, leaves = model.copy_forest()
    assert rep["depth"] >= 1
    assert (int(feat[0, 0]), int(thr[0, 0])) == (int(top.feat[0]), int(top.thr[0]))
    # every configuration: prediction = emitted tree under the evaluator
    ids = F.leaf_ids(feat, thr, rep["depth"], digits)
    assert (model.copy_predictions() == F.predict_fp32(leaves, ids)).all()
    # test errors shrink from the root to the selected cut
    assert rep["abs_err"][rep["depth"]] < rep["abs_err"][0]
