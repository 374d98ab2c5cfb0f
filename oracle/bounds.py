"""What a scored step can return when the model's predictions are known only
within bounds (oracle; test infrastructure only), Sect. 3.6 and Alg. 1.

The tree path computes predictions with the oracle's own float32 order, so
its scores, weights and picks are compared bit for bit.  A model evaluated
in another arithmetic (least-squares polynomials in float32 with contracted
multiply-adds, the perceptron's bf16 activations) gives predictions that the
oracle knows only within an error bound.  This module carries such bounds
through the score equation, the score normalisation, the quantisation and
the weighted draw, as closed intervals:

* prediction of counter p of configuration k: [X_lo, X_hi], both >= 0
  (counters are non-negative);
* score: every float32 score the step can compute from predictions inside
  the intervals, with the float32 chain t = (x - a) / (a + x),
  s = s + dpc * t (counters ascending, every operation rounded, counters with
  a prediction of 0 left out);
* weight: every float32 weight the normalisation can give such a score, with
  s_min / s_max the step's own extremes over unexplored configurations;
* quantised weight q = rint(w * 2^23): [floor(w_lo 2^23), ceil(w_hi 2^23)];
* draw r = floor(U Q / 2^64): the configurations that can be picked for some
  weights inside the intervals.  When exactly one configuration can, the
  pick is certain and must be matched exactly; otherwise the draw is
  flagged and the pick must lie among the feasible ones.

Every interval is evaluated in float64 from monotonicity: t rises with x and
falls with a; the weight rises with s, falls with s_max (s > 0) and rises
with |s_min| (s <= 0); q, Q and r rise with their inputs.  Rounding of the
float32 chain is covered by explicit slack (u = 2^-24):
* score: each term t carries three roundings (|t| <= 1), the product one
  more, and each of the m additions at most u * sum |dpc|; the slack is
  (m + 5) u sum_p |dpc_p| over the m counters that can enter the row's score;
* weight: the ratio s / s_ext, 1 +- ratio and three squarings, at most
  23 u relative; the slack is 32 u relative.
"""
from __future__ import annotations

import numpy as np

from . import score as SC

U32 = 2.0 ** -24


def score_interval(a_lo, a_hi, X_lo, X_hi, delta):
    """Interval [s_lo, s_hi] of the float32 score of every row of X.

    a_lo, a_hi [C]: the profiled configuration's prediction interval;
    X_lo, X_hi [n][C]: the candidates'; delta [C] float32 counter changes.
    All prediction bounds must be >= 0 with lo <= hi."""
    a_lo = np.asarray(a_lo, np.float64)
    a_hi = np.asarray(a_hi, np.float64)
    X_lo = np.asarray(X_lo, np.float64)
    X_hi = np.asarray(X_hi, np.float64)
    d = np.asarray(delta, np.float32).astype(np.float64)
    assert (a_lo >= 0).all() and (X_lo >= 0).all(), "counter bounds must be non-negative"
    assert (a_lo <= a_hi).all() and (X_lo <= X_hi).all()
    n = X_lo.shape[0]
    s_lo = np.zeros(n)
    s_hi = np.zeros(n)
    slack = np.zeros(n)                     # sum of |dpc| over the row's possible terms
    terms = np.zeros(n)                     # and their number
    for p in range(len(d)):
        if d[p] == 0.0 or a_hi[p] == 0.0:
            continue                        # the term is exactly 0
        xl, xh = X_lo[:, p], X_hi[:, p]
        live = xh > 0.0                     # else x == 0: the term is exactly 0
        # smallest t: smallest x against the largest a; x -> 0+ gives -1
        with np.errstate(divide="ignore", invalid="ignore"):
            t_min = np.where(xl > 0.0, (xl - a_hi[p]) / (a_hi[p] + xl), -1.0)
            t_max = ((xh - a_lo[p]) / (a_lo[p] + xh)) if a_lo[p] > 0.0 else np.ones(n)
        # a prediction that may be 0 may also drop the term (t counts as 0)
        maybe0 = (xl == 0.0) | (a_lo[p] == 0.0)
        t_min = np.where(maybe0, np.minimum(t_min, 0.0), t_min)
        t_max = np.where(maybe0, np.maximum(t_max, 0.0), t_max)
        lo = np.minimum(d[p] * t_min, d[p] * t_max)
        hi = np.maximum(d[p] * t_min, d[p] * t_max)
        s_lo += np.where(live, lo, 0.0)
        s_hi += np.where(live, hi, 0.0)
        slack += np.where(live, abs(d[p]), 0.0)
        terms += live
    pad = (terms + 5) * U32 * slack + 1e-15 * slack
    return s_lo - pad, s_hi + pad


def _weight_bound(s, s_min, s_max, upper: bool, gamma, w_min):
    """The normalisation at an interval corner: the ratios s / s_ext are
    clipped to [0, 1], which they are for the step's own extremes."""
    s = np.asarray(s, np.float64)
    out = np.full(s.shape, w_min)
    pos = s > 0.0
    if s_max > 0.0:
        rp = np.clip(s / s_max, 0.0, 1.0)
    else:                                   # s > 0 >= s_max cannot happen on the step's own values
        rp = np.ones(s.shape) if upper else np.zeros(s.shape)
    out = np.where(pos, (1.0 + rp) ** 8, out)
    mid = ~pos & (s > gamma)
    if s_min < 0.0:
        rn = np.clip(s / s_min, 0.0, 1.0)
    else:                                   # s <= 0 <= s_min: only s == 0 is possible
        rn = np.zeros(s.shape) if upper else np.ones(s.shape)
    neg = np.where(s == 0.0, 1.0, np.maximum(w_min, (1.0 - rn) ** 8))
    return np.where(mid, neg, out)


def weight_interval(s_lo, s_hi, explored, gamma=SC.GAMMA, w_min=None):
    """Interval [w_lo, w_hi] of every configuration's float32 weight (0 for
    explored ones) when each float32 score lies in [s_lo, s_hi].  w_min
    defaults to float32(1e-4), the value the float32 chain uses."""
    s_lo = np.asarray(s_lo, np.float64)
    s_hi = np.asarray(s_hi, np.float64)
    un = ~np.asarray(explored, bool)
    if w_min is None:
        w_min = float(np.float32(SC.W_MIN))
    gamma = float(np.float32(gamma))
    w_lo = np.zeros(len(s_lo))
    w_hi = np.zeros(len(s_lo))
    if not un.any():
        return w_lo, w_hi
    # the step's extremes over unexplored configurations
    smin_lo, smin_hi = s_lo[un].min(), s_hi[un].min()
    smax_lo, smax_hi = s_lo[un].max(), s_hi[un].max()
    # lowest weight: lowest s, largest s_max, s_min nearest 0 (smallest |s_min|)
    lo = _weight_bound(s_lo[un], smin_hi, smax_hi, False, gamma, w_min)
    # highest weight: highest s, smallest s_max, s_min farthest below 0
    hi = _weight_bound(s_hi[un], smin_lo, smax_lo, True, gamma, w_min)
    w_lo[un] = lo * (1.0 - 32 * U32)
    w_hi[un] = hi * (1.0 + 32 * U32)
    return w_lo, w_hi


def q_interval(w_lo, w_hi):
    """Interval of q = rint(w * 2^23) as exact integers (uint64)."""
    scale = float(1 << SC.W_SCALE_LOG2)
    q_lo = np.floor(np.asarray(w_lo, np.float64) * scale).astype(np.uint64)
    q_hi = np.ceil(np.asarray(w_hi, np.float64) * scale).astype(np.uint64)
    return q_lo, q_hi


def feasible_picks(q_lo, q_hi, U: int):
    """Valid indices that a draw with uniform U can return for some integer
    weights q with q_lo <= q <= q_hi: every l with q_hi[l] > 0 whose interval
    [sum_{i<l} q_i, sum_{i<=l} q_i) can contain r = floor(U Q / 2^64).
    Returns (first, last, certain): the range holding every feasible pick
    (zero-weight indices inside it are never picked) and whether exactly one
    index is feasible; (None, None, True) when Q is 0 for every choice."""
    q_lo = np.asarray(q_lo, np.uint64)
    q_hi = np.asarray(q_hi, np.uint64)
    zero = np.zeros(1, np.uint64)
    P_lo = np.concatenate([zero, np.cumsum(q_lo, dtype=np.uint64)])
    P_hi = np.concatenate([zero, np.cumsum(q_hi, dtype=np.uint64)])
    Q_lo, Q_hi = int(P_lo[-1]), int(P_hi[-1])
    if Q_hi == 0:
        return None, None, True
    r_lo = (int(U) * Q_lo) >> 64
    r_hi = (int(U) * Q_hi) >> 64
    if Q_lo == 0:
        r_lo = 0
    # l is feasible when P_lo(l) <= r_hi and r_lo < P_hi(l + 1) and q_hi[l] > 0
    first = int(np.searchsorted(P_hi[1:], np.uint64(r_lo), side="right"))
    last = int(np.searchsorted(P_lo[:-1], np.uint64(r_hi), side="right")) - 1
    cand = np.flatnonzero(q_hi[first:last + 1] > 0) + first
    if cand.size == 0:
        return None, None, True
    return int(cand[0]), int(cand[-1]), bool(cand.size == 1)
