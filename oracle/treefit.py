"""Regression-tree fitting (oracle; test infrastructure only), Sect. 3.4.2.

The paper creates its counter model as a regression tree.  Growth is greedy
and top-down (ID3 with a variance criterion in place of information gain;
the MSE criterion is named as the usual choice for regression).  It keeps a
set of candidate trees, trains on a random half of the measured
configurations and tests on the other half, and keeps the candidate with the
lowest MAE on the test half, breaking a tie by the lower RMSE.

Readings (the paper fixes none of these details):

* halves: with keys k_i (one random 64-bit number per measured point, an
  input), the training half is the ceil(n/2) points that come first in the
  order of (k_i >> 32, i); the rest is the test half;
* exact sums: counter c is quantised to integers q = rint(y * 2^s_c), with
  s_c = 22 - e_c, where 2^(e_c - 1) <= max_i |y_ic| < 2^e_c (e_c = 0 when
  every y_ic is 0); so |q| <= 2^22 and every node sum is an exact integer;
* splits are binary, on one parameter's digit (left when digit <= t), the
  layout the tree evaluation uses.  A split (j, t) is admissible when both
  sides hold at least ``min_leaf`` training points; its score is
  sum over c of (S_L^2 / n_L + S_R^2 / n_R) in float64 (each S converted
  exactly, c ascending, folded left to right from 0.0).  Maximising it
  minimises the summed squared error over all counters (multi-output MSE).
  The best score wins, a tie goes to the lower parameter, then the lower
  threshold; the node splits only when that score exceeds the node's own
  sum over c of S^2 / n, folded the same way;
* growth is level by level to the maximum depth D; a node that does not
  split keeps all its points in its left child (parameter 0, threshold 255,
  the form the evaluator reads as "always left"), its right child is empty,
  and neither child is searched again;
* a node's value is its quantised mean m = rint(S / n) (float64 quotient,
  ties to even); an empty node takes its parent's value;
* the candidate trees are the greedy tree cut at depths 0..D ("altering the
  parent nodes"): the nodes at the cut depth become leaves;
* test errors are taken in quantised units, e = m - q over every test point
  and counter, as exact integers: A_d = sum |e|, B_d = sum e^2 for the tree
  cut at depth d.  MAE_d = A_d / (n_test C), RMSE_d = sqrt(B_d / (n_test C));
  the selected depth minimises A_d, then B_d, then d;
* the emitted tree (one tree of the selected depth, in the evaluator's heap
  layout) holds leaf values float32(m * 2^-s_c).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

ALWAYS_LEFT_THR = 255


def train_half(keys) -> np.ndarray:
    """Boolean mask of the training half: the ceil(n/2) points first in the
    order of (key >> 32, index)."""
    keys = np.asarray(keys, dtype=np.uint64)
    n = len(keys)
    hi = (keys >> np.uint64(32)).astype(np.int64)
    order = np.lexsort((np.arange(n), hi))   # primary hi, then index
    mask = np.zeros(n, dtype=bool)
    mask[order[: (n + 1) // 2]] = True
    return mask


def scales(Y) -> np.ndarray:
    """s_c = 22 - e_c with 2^(e_c - 1) <= max |y_c| < 2^e_c (0 -> e_c = 0)."""
    Y = np.asarray(Y, dtype=np.float32)
    s = np.empty(Y.shape[1], dtype=np.int64)
    for c in range(Y.shape[1]):
        mx = float(np.max(np.abs(Y[:, c]))) if len(Y) else 0.0
        e = int(np.frexp(mx)[1]) if mx > 0.0 else 0
        s[c] = 22 - e
    return s


def quantise(Y, s) -> np.ndarray:
    """q = rint(y * 2^s_c) in float64 (exact scaling, ties to even): int64."""
    Y = np.asarray(Y, dtype=np.float32).astype(np.float64)
    return np.rint(np.ldexp(Y, np.asarray(s, dtype=np.int64)[None, :])).astype(np.int64)


def _fold(S, n) -> float:
    """sum over c of S_c^2 / n in float64, c ascending."""
    acc = 0.0
    nn = float(n)
    for v in S:
        a = float(int(v))
        acc = acc + (a * a) / nn
    return acc


def split_scores(digits, q, radix, min_leaf):
    """Scores of every admissible split of one node's points.

    Returns a list of (j, t, score, n_L, S_L); S_L int64 [C]."""
    n = len(q)
    S = q.sum(axis=0)
    out = []
    for j, r in enumerate(radix):
        if r < 2:
            continue
        # per-digit counts and sums, then left sums by prefix over digits
        cnt = np.array([int((digits[:, j] == v).sum()) for v in range(r)], dtype=np.int64)
        sums = np.stack([q[digits[:, j] == v].sum(axis=0) for v in range(r)])
        nL = 0
        SL = np.zeros(q.shape[1], dtype=np.int64)
        for t in range(r - 1):
            nL += int(cnt[t])
            SL = SL + sums[t]
            nR = n - nL
            if nL < min_leaf or nR < min_leaf:
                continue
            SR = S - SL
            acc = 0.0
            for c in range(q.shape[1]):
                a = float(int(SL[c]))
                b = float(int(SR[c]))
                acc = acc + ((a * a) / float(nL) + (b * b) / float(nR))
            out.append((j, t, acc, nL, SL.copy()))
    return out


@dataclass
class Grown:
    depth: int              # D
    feat: np.ndarray        # uint8 [2^D - 1]
    thr: np.ndarray         # uint8 [2^D - 1]
    count: np.ndarray       # int64 [2^(D+1) - 1] training points per node
    sums: np.ndarray        # int64 [2^(D+1) - 1][C]
    mean: np.ndarray        # int64 [2^(D+1) - 1][C] quantised node values
    split: np.ndarray       # bool [2^D - 1] node split (else always-left)


def grow(digits, q, radix, max_depth: int, min_leaf: int) -> Grown:
    """Greedy level-by-level growth of one multi-output tree."""
    digits = np.asarray(digits, dtype=np.int64)
    q = np.asarray(q, dtype=np.int64)
    D = int(max_depth)
    C = q.shape[1]
    n_nodes = (1 << (D + 1)) - 1
    n_int = (1 << D) - 1
    feat = np.zeros(n_int, dtype=np.uint8)
    thr = np.full(n_int, ALWAYS_LEFT_THR, dtype=np.uint8)
    split = np.zeros(n_int, dtype=bool)
    count = np.zeros(n_nodes, dtype=np.int64)
    sums = np.zeros((n_nodes, C), dtype=np.int64)
    mean = np.zeros((n_nodes, C), dtype=np.int64)
    rows = {0: np.arange(len(q))}       # points of the nodes still searched
    count[0] = len(q)
    sums[0] = q.sum(axis=0)
    mean[0] = _mean(sums[0], count[0], np.zeros(C, dtype=np.int64))
    for node in range(n_int):
        left, right = 2 * node + 1, 2 * node + 2
        best = None
        if node in rows and count[node] >= max(2, 2 * min_leaf):
            idx = rows.pop(node)
            for cand in split_scores(digits[idx], q[idx], radix, min_leaf):
                if best is None or cand[2] > best[2]:
                    best = cand
            if best is not None and not best[2] > _fold(sums[node], count[node]):
                best = None
        else:
            idx = rows.pop(node, None)
        if best is None:
            # always-left: the left child keeps everything, is not searched
            count[left], sums[left], mean[left] = count[node], sums[node], mean[node]
            count[right], sums[right], mean[right] = 0, 0, mean[node]
            continue
        j, t, _, nL, SL = best
        feat[node], thr[node], split[node] = j, t, True
        count[left], sums[left] = nL, SL
        count[right], sums[right] = count[node] - nL, sums[node] - SL
        mean[left] = _mean(sums[left], count[left], mean[node])
        mean[right] = _mean(sums[right], count[right], mean[node])
        go_left = digits[idx, j] <= t
        rows[left], rows[right] = idx[go_left], idx[~go_left]
    return Grown(D, feat, thr, count, sums, mean, split)


def _mean(S, n, parent) -> np.ndarray:
    """rint(S / n) in float64 (ties to even); the parent's value when n = 0."""
    if n == 0:
        return np.asarray(parent, dtype=np.int64).copy()
    return np.rint(np.asarray(S, dtype=np.int64).astype(np.float64) / float(n)).astype(np.int64)


def node_at_depths(g: Grown, digits) -> np.ndarray:
    """Heap node reached at each depth 0..D: int64 [D+1][n]."""
    digits = np.asarray(digits, dtype=np.int64)
    n = len(digits)
    out = np.zeros((g.depth + 1, n), dtype=np.int64)
    node = np.zeros(n, dtype=np.int64)
    rows = np.arange(n)
    for d in range(g.depth):
        f = g.feat[node].astype(np.int64)
        left = digits[rows, f] <= g.thr[node].astype(np.int64)
        node = np.where(left, 2 * node + 1, 2 * node + 2)
        out[d + 1] = node
    return out


def candidate_errors(g: Grown, digits, q):
    """Exact test errors of the cut trees: lists A[0..D], B[0..D] (ints)."""
    q = np.asarray(q, dtype=np.int64)
    nodes = node_at_depths(g, digits)
    A, B = [], []
    for d in range(g.depth + 1):
        e = g.mean[nodes[d]] - q
        A.append(int(np.abs(e).sum()))
        B.append(sum(int(v) for v in (e * e).sum(axis=1)))
    return A, B


def select_depth(A, B) -> int:
    """Lowest A, then lowest B, then the shallower depth."""
    return min(range(len(A)), key=lambda d: (A[d], B[d], d))


def emit(g: Grown, d: int, s):
    """The tree cut at depth d in the evaluator's layout (one tree):
    feat, thr uint8 [1][2^d - 1], leaves float32 [1][2^d][C]."""
    n_int = (1 << d) - 1
    feat = g.feat[:n_int].reshape(1, n_int).copy()
    thr = g.thr[:n_int].reshape(1, n_int).copy()
    m = g.mean[n_int: n_int + (1 << d)].astype(np.float64)
    leaves = np.ldexp(m, -np.asarray(s, dtype=np.int64)[None, :]).astype(np.float32)
    return feat, thr, leaves.reshape(1, 1 << d, -1)


@dataclass
class FitResult:
    train: np.ndarray       # bool [n]
    s: np.ndarray           # int64 [C]
    grown: Grown
    A: list                 # test sum |e| per cut depth
    B: list                 # test sum e^2 per cut depth
    depth: int              # selected depth
    feat: np.ndarray
    thr: np.ndarray
    leaves: np.ndarray

    def mae(self, d: int) -> float:
        return self.A[d] / (int((~self.train).sum()) * len(self.s))

    def rmse(self, d: int) -> float:
        return float(np.sqrt(self.B[d] / (int((~self.train).sum()) * len(self.s))))


def fit(digits, Y, keys, radix, max_depth: int, min_leaf: int) -> FitResult:
    """Split, quantise, grow on the training half, score the cut trees on
    the test half and emit the selected one.  Needs n >= 2 points."""
    digits = np.asarray(digits, dtype=np.int64)
    Y = np.asarray(Y, dtype=np.float32)
    if len(Y) < 2:
        raise ValueError("need at least two points")
    tr = train_half(keys)
    s = scales(Y)
    q = quantise(Y, s)
    g = grow(digits[tr], q[tr], radix, max_depth, min_leaf)
    A, B = candidate_errors(g, digits[~tr], q[~tr])
    d = select_depth(A, B)
    feat, thr, leaves = emit(g, d, s)
    return FitResult(tr, s, g, A, B, d, feat, thr, leaves)
