"""Configuration score and score normalisation (oracle), Sect. 3.6.

Score (score equation): for a candidate c and the profiled configuration
c_profile, both predicted by the model, the score sums, over the counters p
in PC_used (predictions non-zero for both configurations), dpc_p times the
relative difference of the two predictions.

Sign reading: printed literally, the relative difference is
(pc(c_profile) - pc(c)) / (pc(c_profile) + pc(c)); with dpc_p < 0 meaning
"decrease counter p" (Sect. 3.5.2) that gives a candidate which lowers the
counter a *negative* score, against the section's stated aim of scoring
higher the configurations that change the counters the required way (and
against the worked example of Sect. 2).  This module uses the sign that
realises the aim:

    s(c) = sum_{p in PC_used} dpc_p * (pc_p(c) - pc_p(c_profile))
                                    / (pc_p(c_profile) + pc_p(c)).

Normalisation (score-normalisation equation) into [1e-4, 256], with
s_min / s_max the extreme scores and gamma = -0.25:

    s > 0            ->  (1 + s / s_max)^8
    gamma < s <= 0   ->  max(1e-4, (1 - s / s_min)^8)
    s <= gamma       ->  1e-4

Readings:
* s_min and s_max are taken over the unexplored valid configurations only;
  explored configurations get weight 0 (Alg. 1 zeroes their score);
* s = 0 gives weight 1 even when s_min = 0 (the formula's limit);
* the eighth power is three squarings;
* sampling weights are quantised to integers q = rint(w * 2^23) so that the
  prefix sums of the draw are exact.  That quantisation is a decision taken
  from a float, so besides the float64 definitions this module evaluates the
  score -> weight chain in float32 with a fixed operation order:
  t = (x - a) / (a + x); s = s + dpc * t, counters ascending, every operation
  rounded to float32, no fused multiply-add.
"""
from __future__ import annotations

import numpy as np

GAMMA = -0.25
W_MIN = 1e-4
W_SCALE_LOG2 = 23


# ----------------------------- float64 definitions -----------------------------
def score_one(a, x, delta) -> float:
    """Score equation for one candidate, plain float64 loop."""
    s = 0.0
    for p in range(len(delta)):
        ap, xp = float(a[p]), float(x[p])
        if ap != 0.0 and xp != 0.0:
            s += float(delta[p]) * (xp - ap) / (ap + xp)
    return s


def score_fp64(a: np.ndarray, X: np.ndarray, delta: np.ndarray) -> np.ndarray:
    """Score equation for every row of X [n][C] (float64)."""
    a = np.asarray(a, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    d = np.asarray(delta, dtype=np.float64)
    s = np.zeros(X.shape[0], dtype=np.float64)
    for p in range(X.shape[1]):
        if a[p] == 0.0:
            continue
        xp = X[:, p]
        used = xp != 0.0
        term = d[p] * (xp - a[p]) / np.where(used, a[p] + xp, 1.0)
        s += np.where(used, term, 0.0)
    return s


def normalize_one(s: float, s_min: float, s_max: float) -> float:
    """Score-normalisation equation for one unexplored configuration (float64)."""
    if s > 0.0:
        return (1.0 + s / s_max) ** 8
    if s > GAMMA:
        if s == 0.0:
            return 1.0
        return max(W_MIN, (1.0 - s / s_min) ** 8)
    return W_MIN


def normalize_fp64(s: np.ndarray, explored: np.ndarray) -> np.ndarray:
    """Weights for all configurations; explored ones get 0."""
    s = np.asarray(s, dtype=np.float64)
    un = ~np.asarray(explored, dtype=bool)
    w = np.zeros_like(s)
    if not un.any():
        return w
    s_min = s[un].min()
    s_max = s[un].max()
    for i in np.flatnonzero(un):
        w[i] = normalize_one(float(s[i]), s_min, s_max)
    return w


# ------------------------ float32 decision chain -------------------------------
def score_fp32(a: np.ndarray, X: np.ndarray, delta: np.ndarray) -> np.ndarray:
    """Score equation in float32, counters ascending, each op rounded."""
    a = np.asarray(a, dtype=np.float32)
    X = np.asarray(X, dtype=np.float32)
    d = np.asarray(delta, dtype=np.float32)
    s = np.zeros(X.shape[0], dtype=np.float32)
    for p in range(X.shape[1]):
        if a[p] == 0:
            continue
        xp = X[:, p]
        t = (xp - a[p]) / (a[p] + xp)
        term = d[p] * t
        s = np.where(xp != 0, s + term, s).astype(np.float32)
    return s


def _pow8_f32(y: np.ndarray) -> np.ndarray:
    y2 = (y * y).astype(np.float32)
    y4 = (y2 * y2).astype(np.float32)
    return (y4 * y4).astype(np.float32)


def weights_fp32(s: np.ndarray, explored: np.ndarray):
    """Normalised weights in float32; returns (w, s_min, s_max)."""
    s = np.asarray(s, dtype=np.float32)
    un = ~np.asarray(explored, dtype=bool)
    w = np.zeros_like(s)
    if not un.any():
        return w, np.float32(np.inf), np.float32(-np.inf)
    s_min = s[un].min()
    s_max = s[un].max()
    one = np.float32(1.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        pos = _pow8_f32((one + (s / s_max).astype(np.float32)).astype(np.float32))
        neg = _pow8_f32((one - (s / s_min).astype(np.float32)).astype(np.float32))
    neg = np.maximum(np.float32(W_MIN), neg)
    w = np.where(s > 0, pos,
                 np.where(s > np.float32(GAMMA),
                          np.where(s == 0, one, neg),
                          np.float32(W_MIN))).astype(np.float32)
    w = np.where(un, w, np.float32(0.0)).astype(np.float32)
    return w, s_min, s_max


def quantize(w: np.ndarray) -> np.ndarray:
    """q = rint(w * 2^23), round half to even, as uint64 integers."""
    scaled = (np.asarray(w, dtype=np.float32) * np.float32(1 << W_SCALE_LOG2)).astype(np.float32)
    return np.rint(scaled).astype(np.uint64)
