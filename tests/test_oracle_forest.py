"""Oracle pins: decision-tree model evaluation (Sect. 3.4.2)."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import forest as F
from oracle import space as SP

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tree_hand_traced.json")


def test_hand_traced_trees():
    g = json.load(open(GOLDEN))
    for tree in g["trees"]:
        feat = np.array([tree["feat"]], dtype=np.uint8)
        thr = np.array([tree["thr"]], dtype=np.uint8)
        digits = np.array([c["digits"] for c in tree["cases"]], dtype=np.int64)
        expect = [c["leaf"] for c in tree["cases"]]
        assert F.leaf_ids(feat, thr, tree["depth"], digits)[0].tolist() == expect
        for c in tree["cases"]:
            assert F.leaf_of(feat[0], thr[0], tree["depth"], c["digits"]) == c["leaf"]


def test_depth_zero_tree_is_its_leaf():
    feat = np.zeros((1, 0), dtype=np.uint8)
    thr = np.zeros((1, 0), dtype=np.uint8)
    digits = np.array([[0, 1], [3, 2]], dtype=np.int64)
    assert F.leaf_ids(feat, thr, 0, digits).tolist() == [[0, 0]]


def test_copies_of_one_tree_average_to_it():
    sp = synth.space_c1()
    f = synth.random_forest(synth.rng(99), sp.radix, 1, 6, 5)
    T = 8
    feat = np.repeat(f.feat, T, axis=0)
    thr = np.repeat(f.thr, T, axis=0)
    leaves = np.repeat(f.leaves, T, axis=0)
    digits = SP.digits_of(np.arange(0, sp.n_raw, 7), sp.radix)
    ids1 = F.leaf_ids(f.feat, f.thr, f.depth, digits)
    idsT = F.leaf_ids(feat, thr, f.depth, digits)
    assert (idsT == ids1[0]).all()
    single = f.leaves[0][ids1[0]].astype(np.float64)
    assert (F.predict_fp64(leaves, idsT) == single).all()
    p32 = F.predict_fp32(leaves, idsT)
    assert np.max(np.abs(p32 - single)) <= T * 2.0 ** -24 * np.max(np.abs(single))


def test_mean_of_constant_trees():
    # tree t's leaves all hold the value t: the mean is (T-1)/2 everywhere
    T, D, C = 4, 3, 2
    feat = np.zeros((T, (1 << D) - 1), dtype=np.uint8)
    thr = np.zeros_like(feat)
    leaves = np.broadcast_to(np.arange(T, dtype=np.float32)[:, None, None], (T, 1 << D, C)).copy()
    digits = np.array([[0], [1], [2]], dtype=np.int64)
    ids = F.leaf_ids(feat, thr, D, digits)
    assert (F.predict_fp64(leaves, ids) == 1.5).all()
    assert (F.predict_fp32(leaves, ids) == 1.5).all()


def test_vectorised_walk_matches_scalar_walk():
    sp = synth.space_c1()
    f = synth.random_forest(synth.rng(7), sp.radix, 3, 5, 4)
    ks = np.arange(0, sp.n_raw, 97)
    digits = SP.digits_of(ks, sp.radix)
    ids = F.leaf_ids(f.feat, f.thr, f.depth, digits)
    for i in range(0, len(ks), 13):
        for t in range(f.n_trees):
            assert ids[t, i] == F.leaf_of(f.feat[t], f.thr[t], f.depth, digits[i].tolist())


def test_leftmost_and_rightmost_paths():
    # all thresholds at the top digit: every config goes left to leaf 0;
    # all thresholds -1 impossible for uint8, so use digit > thr with thr = 0 and digits >= 1
    D = 4
    feat = np.zeros((1, (1 << D) - 1), dtype=np.uint8)
    thr = np.full_like(feat, 7)
    assert F.leaf_ids(feat, thr, D, np.array([[7]]))[0, 0] == 0
    thr0 = np.zeros_like(feat)
    assert F.leaf_ids(feat, thr0, D, np.array([[1]]))[0, 0] == (1 << D) - 1
