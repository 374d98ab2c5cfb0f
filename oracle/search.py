"""One search step of Alg. 1 (oracle), composed from the other modules.

Per iteration Alg. 1 (Sect. 3.7) scores every configuration of TS that was
not evaluated yet (zero otherwise), using the model's predictions for the
candidate and for the profiled configuration and the required counter
changes, then performs n + 1 weighted draws, zeroing each drawn score.

Readings: the profiled configuration and every drawn configuration count as
evaluated; the starting configuration (a uniform draw over TS) is the
special case dPC = 0 of the same step, where every score is 0 and every
weight is 1.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import forest as F
from . import sampling as S
from . import score as SC
from . import space as SP


@dataclass
class Prepared:
    """Enumerated space and model predictions for it."""
    valid: np.ndarray      # uint32 [Nv] raw indices, ascending
    digits: np.ndarray     # int64 [Nv][P]
    leaf_ids: np.ndarray   # int64 [T][Nv]
    P64: np.ndarray        # float64 [Nv][C]
    P32: np.ndarray        # float32 [Nv][C]


def prepare(space, forest, valid=None) -> Prepared:
    if valid is None:
        valid = SP.enumerate_valid(space.radix, space.values, space.constraints)
    digits = SP.digits_of(valid.astype(np.int64), space.radix)
    ids = F.leaf_ids(forest.feat, forest.thr, forest.depth, digits)
    return Prepared(valid, digits, ids, F.predict_fp64(forest.leaves, ids),
                    F.predict_fp32(forest.leaves, ids))


@dataclass
class StepResult:
    s32: np.ndarray
    s64: np.ndarray
    w32: np.ndarray
    q: np.ndarray
    s_min: float
    s_max: float
    total: int
    picks: list            # valid indices (None when nothing is left)


def step(prep: Prepared, explored: np.ndarray, profile: int, delta: np.ndarray,
         uniforms, with_fp64: bool = True) -> StepResult:
    """Score all unexplored configurations against ``profile`` (a valid
    index, marked explored) and draw ``len(uniforms)`` configurations.
    ``profile=None`` is the start of Alg. 1 (nothing profiled): every score
    is 0.  ``explored`` is updated in place with the profile and the picks."""
    delta = np.asarray(delta, dtype=np.float32)
    if profile is None:
        s32 = np.zeros(len(prep.valid), dtype=np.float32)
        s64 = np.zeros(len(prep.valid)) if with_fp64 else None
    else:
        explored[profile] = True
        s32 = SC.score_fp32(prep.P32[profile], prep.P32, delta)
        s64 = (SC.score_fp64(prep.P64[profile], prep.P64, delta.astype(np.float64))
               if with_fp64 else None)
    w32, s_min, s_max = SC.weights_fp32(s32, explored)
    q = SC.quantize(w32)
    total = int(q.sum(dtype=np.uint64))
    picks = S.draws(q, uniforms)
    for l in picks:
        if l is not None:
            explored[l] = True
    return StepResult(s32, s64, w32, q, float(s_min), float(s_max), total, picks)
