"""GPU forest evaluation vs the oracle (Sect. 3.4.2): leaf ids bit-exact,
predictions bit-exact against the oracle's float32 sum order and within
float32 rounding of its float64 mean."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import forest as F
from oracle import space as SP
from tests.helpers import cgs, golden

pytestmark = pytest.mark.gpu


def test_hand_traced_trees():
    m = cgs()
    g = golden("tree_hand_traced.json")
    radix = g["radix"]
    values = [list(range(r)) for r in radix]
    sp = m.Space(radix, values, [])
    for tree in g["trees"]:
        D = tree["depth"]
        leaves = np.arange(1 << D, dtype=np.float32)[None, :, None] + np.zeros((1, 1, 4), np.float32)
        model = m.ForestModel(sp, np.array([tree["feat"]], np.uint8), np.array([tree["thr"]], np.uint8),
                              leaves)
        ids = model.copy_leaf_ids()[0]
        P = model.copy_predictions()
        for case in tree["cases"]:
            k = int(np.ravel_multi_index(case["digits"], radix))
            assert ids[k] == case["leaf"]
            assert (P[k] == case["leaf"]).all()


def _check_full(spec, forest):
    m = cgs()
    sp = m.Space.from_spec(spec)
    model = m.ForestModel.from_spec(sp, forest)
    valid = sp.copy_valid()
    digits = SP.digits_of(valid.astype(np.int64), spec.radix)
    ids = F.leaf_ids(forest.feat, forest.thr, forest.depth, digits)
    assert (model.copy_leaf_ids() == ids).all()
    P = model.copy_predictions()
    assert (P == F.predict_fp32(forest.leaves, ids)).all()
    P64 = F.predict_fp64(forest.leaves, ids)
    T = forest.n_trees
    assert (np.abs(P - P64) <= (T + 1) * 2.0 ** -24 * np.abs(P64) + 1e-30).all()


def test_c1_forest_full():
    spec = synth.space_c1()
    _check_full(spec, synth.forest_c1(spec))


@pytest.mark.parametrize("T,D,C", [(1, 0, 3), (3, 1, 5), (4, 7, 12), (64, 4, 2), (2, 14, 7),
                                   (5, 9, 64), (1, 0, 12), (8, 10, 16), (12, 6, 32), (16, 12, 24),
                                   (3, 5, 24), (16, 8, 32), (2, 11, 16), (7, 9, 12)])
def test_shapes_on_c1_space(T, D, C):
    spec = synth.space_c1()
    _check_full(spec, synth.random_forest(synth.rng(50, T, D, C), spec.radix, T, D, C))


def test_c2_forest_sampled():
    """Full c2 space (4.8M valid, 16 trees of depth 12): leaf ids and
    predictions of 3000 sampled valid configurations, walked one by one."""
    m = cgs()
    spec = synth.space_c2()
    forest = synth.forest_c2(spec)
    sp = m.Space.from_spec(spec)
    model = m.ForestModel.from_spec(sp, forest)
    valid = sp.copy_valid()
    g = np.random.default_rng(5)
    pos = np.unique(np.concatenate([[0, len(valid) - 1], g.integers(0, len(valid), 3000)]))
    P = model.copy_predictions()
    for l in pos[:: max(1, len(pos) // 200)]:
        d = SP.decode(int(valid[l]), spec.radix)
        ids_l = [F.leaf_of(forest.feat[t], forest.thr[t], forest.depth, d) for t in range(16)]
        got = model.copy_leaf_ids(int(l), 1)[:, 0]
        assert got.tolist() == ids_l
    digits = SP.digits_of(valid[pos].astype(np.int64), spec.radix)
    ids = F.leaf_ids(forest.feat, forest.thr, forest.depth, digits)
    assert (P[pos] == F.predict_fp32(forest.leaves, ids)).all()


def test_forest_rejects_bad_input():
    m = cgs()
    sp = m.Space([3, 2], [[1, 2, 3], [0, 1]], [])
    with pytest.raises(m.CgsError) as ei:
        m.ForestModel(sp, np.array([[5]], np.uint8), np.array([[0]], np.uint8),
                      np.ones((1, 2, 2), np.float32))
    assert ei.value.status == m.EINVAL
    bad = np.ones((1, 2, 2), np.float32)
    bad[0, 1, 1] = np.nan
    with pytest.raises(m.CgsError) as ei:
        m.ForestModel(sp, np.array([[0]], np.uint8), np.array([[0]], np.uint8), bad)
    assert ei.value.status == m.EINVAL


def test_gather_predictions_equal_the_oracle():
    """Predictions of listed valid indices (unsorted, with repeats, both ends
    of the list): equal to the full copy and to the oracle's float32 mean."""
    m = cgs()
    spec = synth.space_c1()
    forest = synth.forest_c1(spec)
    sp = m.Space.from_spec(spec)
    model = m.ForestModel.from_spec(sp, forest)
    valid = sp.copy_valid()
    g = np.random.default_rng(11)
    idx = np.concatenate([[len(valid) - 1, 0, 0], g.integers(0, len(valid), 5000)]).astype(np.uint32)
    got = model.gather_predictions(idx)
    assert (got == model.copy_predictions()[idx]).all()
    ids = F.leaf_ids(forest.feat, forest.thr, forest.depth,
                     SP.digits_of(valid[idx].astype(np.int64), spec.radix))
    assert (got == F.predict_fp32(forest.leaves, ids)).all()
    assert model.gather_predictions(np.zeros(0, np.uint32)).shape == (0, 12)
    with pytest.raises(m.CgsError) as ei:
        model.gather_predictions([len(valid)])
    assert ei.value.status == m.EINVAL
