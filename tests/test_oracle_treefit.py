"""Oracle pins: regression-tree fitting (Sect. 3.4.2).

The greedy growth is checked against scikit-learn's tree builder (a special
case that reduces to a library routine: binary splits, multi-output
squared-error criterion, the same minimum leaf size); the split rule against
exact rational arithmetic by brute force; and the fit end to end against a
planted split it must recover."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import forest as F
from oracle import treefit as TF


# ---------------------------------------------------------------- halves
@pytest.mark.parametrize("n", [2, 3, 10, 101])
def test_train_half_is_the_first_half_in_key_order(n):
    g = np.random.default_rng(n)
    keys = synth.uniforms_u64(g, n)
    # force ties in the high 32 bits: the index must decide among them
    keys[: n // 2] = (keys[: n // 2] & np.uint64(0xFFFFFFFF00000000)) | np.uint64(7)
    keys[1::3] = keys[0] ^ np.uint64(0x1234)     # same high word as keys[0]
    tr = TF.train_half(keys)
    assert tr.sum() == (n + 1) // 2
    order = sorted(range(n), key=lambda i: (int(keys[i]) >> 32, i))
    assert set(np.flatnonzero(tr).tolist()) == set(order[: (n + 1) // 2])


# ------------------------------------------------------------ quantising
def test_scales_by_hand():
    Y = np.array([[1.0, 0.75, 0.0, -8.0, 3.0e-30]], dtype=np.float32)
    # frexp: 1.0 = 0.5 * 2^1, 0.75 = 0.75 * 2^0, 8 = 0.5 * 2^4
    assert TF.scales(Y).tolist()[:4] == [21, 22, 22, 18]
    q = TF.quantise(Y, TF.scales(Y))
    assert q[0, :4].tolist() == [1 << 21, 3 << 20, 0, -(1 << 21)]


def test_quantise_bounds_and_round_trip():
    g = np.random.default_rng(3)
    Y = (g.standard_normal((500, 6)) * np.array([1e-30, 1e-3, 1.0, 7.0, 1e5, 3e30])).astype(np.float32)
    Y[0, 0] = np.float32(1e-42)                   # a subnormal
    s = TF.scales(Y)
    q = TF.quantise(Y, s)
    assert np.abs(q).max() <= 1 << 22
    back = np.ldexp(q.astype(np.float64), -s[None, :])
    assert (np.abs(back - Y.astype(np.float64)) <= np.ldexp(0.5, -s)[None, :]).all()
    # the largest magnitude of each counter lands in [2^21, 2^22]
    top = np.abs(q).max(axis=0)
    assert ((top >= 1 << 21) & (top <= 1 << 22)).all()


# ------------------------------------------------------------ hand example
def test_grow_hand_example():
    """One parameter of radix 4, values q = 0, 0, 6, 6 at digits 0..3.
    Root: t=0 scores 0 + 144/3 = 48, t=1 scores 0 + 144/2 = 72, t=2 scores
    36/3 + 36/1 = 48; 72 > 144/4 = 36, so the root splits at t = 1.  Neither
    child can improve (the left one is constant; the right one's only split
    scores 36 + 36 = 72 = 144/2), so both are always-left."""
    g = TF.grow([[0], [1], [2], [3]], [[0], [0], [6], [6]], [4], 2, 1)
    assert g.feat.tolist() == [0, 0, 0] and g.thr.tolist() == [1, 255, 255]
    assert g.split.tolist() == [True, False, False]
    assert g.count.tolist() == [4, 2, 2, 2, 0, 2, 0]
    assert g.mean[:, 0].tolist() == [3, 0, 6, 0, 0, 6, 6]


def test_select_depth_rule():
    assert TF.select_depth([5, 3, 3, 3], [9, 8, 7, 7]) == 2
    assert TF.select_depth([5, 3, 3, 3], [9, 8, 8, 8]) == 1
    assert TF.select_depth([0], [0]) == 0


# ------------------------------------------------------------ brute force
def _sse(q):
    if len(q) == 0:
        return Fraction(0)
    tot = Fraction(0)
    for c in range(q.shape[1]):
        col = [int(v) for v in q[:, c]]
        mu = Fraction(sum(col), len(col))
        tot += sum((Fraction(v) - mu) ** 2 for v in col)
    return tot


@pytest.mark.parametrize("seed", range(12))
def test_root_split_is_the_exact_best_sse_reduction(seed):
    g = np.random.default_rng(seed)
    P = int(g.integers(1, 4))
    radix = [int(r) for r in g.integers(1, 5, P)]
    n = int(g.integers(2, 14))
    digits = np.stack([g.integers(0, r, n) for r in radix], axis=1)
    if seed % 3 == 0:
        digits = np.concatenate([digits, digits[:, :1]], axis=1)   # a duplicate column: exact ties
        radix = radix + radix[:1]
    q = g.integers(-50, 50, (n, int(g.integers(1, 4))))
    if seed % 4 == 1:
        q[:] = q[0]                                               # constant: never splits
    min_leaf = int(g.integers(1, 3))
    best = None
    for j, r in enumerate(radix):
        for t in range(r - 1):
            left = digits[:, j] <= t
            if left.sum() < min_leaf or (~left).sum() < min_leaf:
                continue
            red = _sse(q) - _sse(q[left]) - _sse(q[~left])
            if best is None or red > best[0]:
                best = (red, j, t)
    gr = TF.grow(digits, q, radix, 1, min_leaf)
    if best is None or best[0] == 0 or n < 2 * min_leaf:
        assert not gr.split[0]
    else:
        assert gr.split[0] and (int(gr.feat[0]), int(gr.thr[0])) == best[1:]


def test_ties_go_to_the_lower_parameter_then_the_lower_threshold():
    """Parameter 2 repeats parameter 0, and only digits 0 and 3 of radix 4
    occur: thresholds 0, 1 and 2 induce the same partition on both, so all
    six splits score the same and the split must be (0, 0)."""
    g = np.random.default_rng(9)
    d0 = g.choice([0, 3], 40)
    digits = np.stack([d0, g.integers(0, 2, 40), d0], axis=1)
    q = np.where(d0 == 0, 100, -100)[:, None] + g.integers(-3, 4, (40, 2))
    gr = TF.grow(digits, q, [4, 2, 4], 1, 1)
    assert gr.split[0] and (int(gr.feat[0]), int(gr.thr[0])) == (0, 0)
    scores = [c for c in TF.split_scores(digits, q, [4, 2, 4], 1) if c[0] != 1]
    assert len(scores) == 6 and len({c[2] for c in scores}) == 1


# ------------------------------------------------------------ scikit-learn
@pytest.mark.parametrize("seed,depth,min_leaf", [(0, 3, 1), (1, 5, 1), (2, 6, 3), (3, 4, 10), (4, 8, 2)])
def test_growth_matches_sklearn(seed, depth, min_leaf):
    """Same partition of the training points and the same node values as
    scikit-learn's squared-error tree on the digits (continuous random
    targets, so no two splits tie)."""
    from sklearn.tree import DecisionTreeRegressor
    g = np.random.default_rng(seed)
    radix = [int(r) for r in g.integers(1, 9, 7)]
    n = 600
    digits = np.stack([g.integers(0, r, n) for r in radix], axis=1)
    base = np.sin(digits @ g.standard_normal((7, 5))) + 0.1 * g.standard_normal((n, 5))
    q = TF.quantise(base.astype(np.float32), TF.scales(base.astype(np.float32)))
    gr = TF.grow(digits, q, radix, depth, min_leaf)
    sk = DecisionTreeRegressor(max_depth=depth, min_samples_leaf=min_leaf, random_state=0)
    sk.fit(digits.astype(np.float64), q.astype(np.float64))
    ours = TF.node_at_depths(gr, digits)[depth]
    theirs = sk.apply(digits.astype(np.float64))
    pairs = set(zip(ours.tolist(), theirs.tolist()))
    assert len(pairs) == len(set(ours.tolist())) == len(set(theirs.tolist()))
    pred = sk.predict(digits.astype(np.float64)).reshape(n, -1)
    assert (gr.mean[ours] == np.rint(pred)).all()
    # internal nodes that split, counted both ways
    assert int(gr.split.sum()) == int((sk.tree_.children_left >= 0).sum())


# ------------------------------------------------------------ invariants
@pytest.mark.parametrize("seed", range(4))
def test_children_partition_their_parent(seed):
    g = np.random.default_rng(40 + seed)
    radix = [2, 3, 5, 1, 8]
    n = 300
    digits = np.stack([g.integers(0, r, n) for r in radix], axis=1)
    q = g.integers(-1000, 1000, (n, 3))
    min_leaf = 1 + seed * 3
    gr = TF.grow(digits, q, radix, 5, min_leaf)
    for node in range(len(gr.feat)):
        l, r = 2 * node + 1, 2 * node + 2
        assert gr.count[node] == gr.count[l] + gr.count[r]
        assert (gr.sums[node] == gr.sums[l] + gr.sums[r]).all()
        if gr.split[node]:
            assert min(gr.count[l], gr.count[r]) >= min_leaf
        else:
            assert gr.count[r] == 0 and (gr.mean[r] == gr.mean[node]).all()
    last = gr.count[len(gr.feat):]
    assert last.sum() == n
    nodes = TF.node_at_depths(gr, digits)
    for d in range(gr.depth + 1):
        for node in np.unique(nodes[d]):
            sel = nodes[d] == node
            assert sel.sum() == gr.count[node]
            assert (q[sel].sum(axis=0) == gr.sums[node]).all()


# ------------------------------------------------------------ end to end
def _full_factorial(radix):
    return np.array(list(itertools.product(*[range(r) for r in radix])), dtype=np.int64)


@pytest.mark.parametrize("j,t", [(1, 1), (3, 2), (0, 0)])
def test_fit_recovers_a_planted_split(j, t):
    radix = [3, 4, 2, 5]
    digits = _full_factorial(radix)
    g = np.random.default_rng(10 * j + t)
    lo = (g.integers(0, 1024, 4) / 1024.0).astype(np.float32)
    hi = (g.integers(0, 1024, 4) / 1024.0).astype(np.float32)
    hi[0] = np.float32(1.0)                         # distinct, max exactly 1
    Y = np.where((digits[:, j] <= t)[:, None], lo[None, :], hi[None, :]).astype(np.float32)
    keys = synth.uniforms_u64(g, len(Y))
    r = TF.fit(digits, Y, keys, radix, 3, 1)
    assert r.depth == 1
    assert (int(r.feat[0, 0]), int(r.thr[0, 0])) == (j, t)
    assert (r.leaves[0, 0] == lo).all() and (r.leaves[0, 1] == hi).all()
    assert r.A[0] > 0 and r.A[1:] == [0, 0, 0] and r.B[1:] == [0, 0, 0]


def test_candidate_zero_is_the_root_mean():
    g = np.random.default_rng(5)
    radix = [4, 4, 3]
    digits = _full_factorial(radix)
    Y = g.random((len(digits), 4), dtype=np.float32)
    r = TF.fit(digits, Y, synth.uniforms_u64(g, len(Y)), radix, 4, 2)
    q = TF.quantise(Y, r.s)
    m0 = np.rint(q[r.train].sum(axis=0) / r.train.sum())
    e = m0[None, :] - q[~r.train]
    assert r.A[0] == int(np.abs(e).sum()) and r.B[0] == int((e * e).sum())
    assert r.depth == TF.select_depth(r.A, r.B)


@pytest.mark.parametrize("seed", range(3))
def test_emitted_tree_evaluates_to_the_node_values(seed):
    """The evaluator (heap walk, always-left at threshold 255) applied to the
    emitted tree gives every configuration the value of the node it reaches at
    the selected depth."""
    g = np.random.default_rng(60 + seed)
    radix = [3, 2, 4, 3, 2]
    digits = _full_factorial(radix)
    Y = (g.random((len(digits), 3)) * [1.0, 50.0, 0.01]).astype(np.float32)
    r = TF.fit(digits, Y, synth.uniforms_u64(g, len(Y)), radix, 6, 2 + seed)
    ids = F.leaf_ids(r.feat, r.thr, r.depth, digits)
    pred = F.predict_fp32(r.leaves, ids)
    node = TF.node_at_depths(r.grown, digits)[r.depth]
    want = np.ldexp(r.grown.mean[node].astype(np.float64), -r.s[None, :]).astype(np.float32)
    assert (pred == want).all()
