"""Neighbourhood-restricted search step (oracle; test infrastructure only).

For huge tuning spaces the paper suggests scoring a restricted set of
configurations, for instance only the neighbourhood of the profiled one
(Sect. 3.7, footnote to the scoring line of Alg. 1).  It does not define the
neighbourhood; the reading taken here:

- the neighbourhood of radius h is every configuration whose parameters
  differ from the profiled configuration's in 1..h positions (Hamming
  distance over the parameters' values);
- candidates are its valid, unexplored members, in the order: distance, then
  the set of changed parameters (lexicographic), then their new digits
  (lexicographic, the profile's own digit skipped);
- the step scores the candidates with the score equation, normalises over
  the candidates only and draws among them with removal, exactly as the
  full step does over the whole space (same float32 chain, same quantised
  weights, same draw rule, prefix in candidate order).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

from . import sampling as S
from . import score as SC


def strides_of(radix) -> np.ndarray:
    """Mixed-radix place values, parameter 0 most significant."""
    radix = [int(r) for r in radix]
    st = np.ones(len(radix), dtype=np.int64)
    for j in range(len(radix) - 2, -1, -1):
        st[j] = st[j + 1] * radix[j + 1]
    return st


def ball(radix, profile_digits, radius: int) -> np.ndarray:
    """Raw indices of the configurations at distance 1..radius from the
    profile, in candidate order."""
    pd = [int(d) for d in profile_digits]
    st = strides_of(radix)
    base = int(sum(pd[j] * int(st[j]) for j in range(len(pd))))
    out = []
    for dist in range(1, radius + 1):
        for subset in itertools.combinations(range(len(pd)), dist):
            choices = [[v for v in range(int(radix[j])) if v != pd[j]] for j in subset]
            for vs in itertools.product(*choices):
                out.append(base + sum((v - pd[j]) * int(st[j]) for j, v in zip(subset, vs)))
    return np.array(out, dtype=np.int64)


def ball_size(radix, radius: int) -> int:
    """Number of configurations at distance 1..radius: the elementary
    symmetric sums e_1 .. e_radius of (r_j - 1)."""
    e = [1] + [0] * radius
    for r in radix:
        a = int(r) - 1
        for d in range(radius, 0, -1):
            e[d] += e[d - 1] * a
    return sum(e[1:])


@dataclass
class NeighbourhoodResult:
    cand: np.ndarray       # valid indices of the candidates, in candidate order
    s32: np.ndarray        # their scores
    w32: np.ndarray
    q: np.ndarray
    s_min: float
    s_max: float
    total: int
    picks: list            # valid indices (None when nothing is left)


def step(prep, radix, explored: np.ndarray, profile: int, delta, uniforms,
         radius: int) -> NeighbourhoodResult:
    """Score the neighbourhood of ``profile`` (a valid index, marked
    explored) and draw ``len(uniforms)`` configurations from it.
    ``prep`` is a search.Prepared; ``explored`` is updated in place."""
    delta = np.asarray(delta, dtype=np.float32)
    explored[profile] = True
    raw = ball(radix, prep.digits[profile], radius)
    pos = np.searchsorted(prep.valid.astype(np.int64), raw)
    inside = pos < len(prep.valid)
    hit = np.zeros(len(raw), dtype=bool)
    hit[inside] = prep.valid[pos[inside]].astype(np.int64) == raw[inside]
    cand = pos[hit]
    cand = cand[~explored[cand]]
    s32 = SC.score_fp32(prep.P32[profile], prep.P32[cand], delta)
    w32, s_min, s_max = SC.weights_fp32(s32, np.zeros(len(cand), dtype=bool))
    q = SC.quantize(w32)
    total = int(q.sum(dtype=np.uint64))
    local = S.draws(q, uniforms)
    picks = [None if l is None else int(cand[l]) for l in local]
    for l in picks:
        if l is not None:
            explored[l] = True
    return NeighbourhoodResult(cand, s32, w32, q, float(s_min), float(s_max), total, picks)
