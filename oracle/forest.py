"""Decision-tree model evaluation (oracle), Sect. 3.4.2.

The paper's model is one regression tree whose internal nodes test tuning
parameters and whose leaves hold predicted counter values; it is used to
predict the counters of unexplored configurations.

Readings:
* binary splits on a parameter's *digit* (its index in the ascending value
  table): go left when ``digit[feat] <= thr``; with strictly ascending
  tables this is the same as comparing values;
* trees are complete, stored in heap order (children of node i are 2i+1 and
  2i+2), leaves numbered left to right;
* with T > 1 trees the prediction is the mean of the T leaf vectors (a
  regression forest; T = 1 is the paper's single tree).
"""
from __future__ import annotations

import numpy as np


def leaf_of(feat_t, thr_t, depth: int, digits) -> int:
    """Leaf reached by one configuration in one tree (scalar walk)."""
    node = 0
    for _ in range(depth):
        f = int(feat_t[node])
        node = 2 * node + 1 if digits[f] <= int(thr_t[node]) else 2 * node + 2
    return node - ((1 << depth) - 1)


def leaf_ids(feat, thr, depth: int, digits: np.ndarray) -> np.ndarray:
    """Vectorised walk: digits int64 [n][P] -> leaf ids int64 [T][n]."""
    n_trees = feat.shape[0]
    n = digits.shape[0]
    rows = np.arange(n)
    out = np.empty((n_trees, n), dtype=np.int64)
    for t in range(n_trees):
        node = np.zeros(n, dtype=np.int64)
        ft = feat[t].astype(np.int64)
        tt = thr[t].astype(np.int64)
        for _ in range(depth):
            f = ft[node]
            go_left = digits[rows, f] <= tt[node]
            node = np.where(go_left, 2 * node + 1, 2 * node + 2)
        out[t] = node - ((1 << depth) - 1)
    return out


def predict_fp64(leaves: np.ndarray, ids: np.ndarray) -> np.ndarray:
    """Mean leaf vector over trees in float64: [n][C]."""
    n_trees = leaves.shape[0]
    acc = np.zeros((ids.shape[1], leaves.shape[2]), dtype=np.float64)
    for t in range(n_trees):
        acc += leaves[t][ids[t]].astype(np.float64)
    return acc / n_trees


def predict_fp32(leaves: np.ndarray, ids: np.ndarray) -> np.ndarray:
    """The same mean in float32 with a fixed order: trees summed in ascending
    t starting from tree 0's leaf, then one IEEE division by T.  [n][C]."""
    n_trees = leaves.shape[0]
    acc = leaves[0][ids[0]].astype(np.float32)
    for t in range(1, n_trees):
        acc = (acc + leaves[t][ids[t]]).astype(np.float32)
    return (acc / np.float32(n_trees)).astype(np.float32)
