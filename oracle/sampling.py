"""Score-weighted random draw with removal (oracle), Sect. 3.7 / Alg. 1.

Alg. 1 draws a random number r below the total score, picks the
configuration l whose cumulative-score interval contains r, and then sets
S_l to zero before the next draw of the same iteration.  Its printed
interval conditions are garbled; the reading used here is the half-open
inverse-CDF rule

    0 <= r < sum_i q_i,     sum_{i<l} q_i <= r < sum_{i<=l} q_i,

so zero-weight configurations are never chosen.  Weights are the integer
quantised weights q; the random input is a 64-bit integer U and
r = floor(U * Q / 2^64) with Q the total (exact 128-bit product), which is
uniform over [0, Q) up to the resolution of U.
"""
from __future__ import annotations

import numpy as np


def pick_scalar(q, U: int):
    """Linear-scan draw over a list of integer weights; None when all are 0."""
    total = sum(int(v) for v in q)
    if total == 0:
        return None
    r = (int(U) * total) >> 64
    acc = 0
    for l, v in enumerate(q):
        if acc <= r < acc + int(v):
            return l
        acc += int(v)
    raise AssertionError("unreachable: r < total")


def pick(q: np.ndarray, U: int):
    """Vectorised draw: prefix sums in exact uint64 arithmetic."""
    q = np.asarray(q, dtype=np.uint64)
    incl = np.cumsum(q, dtype=np.uint64)
    total = int(incl[-1]) if incl.size else 0
    if total == 0:
        return None
    r = (int(U) * total) >> 64
    return int(np.searchsorted(incl, np.uint64(r), side="right"))


def draws(q: np.ndarray, uniforms) -> list:
    """Consecutive draws of one iteration, zeroing each pick (S_l <- 0)."""
    q = np.array(q, dtype=np.uint64, copy=True)
    out = []
    for U in uniforms:
        l = pick(q, int(U))
        out.append(l)
        if l is None:
            break
        q[l] = 0
    return out
