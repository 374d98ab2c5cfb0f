"""Tuning-space enumeration (oracle).

Sect. 1 defines a tuning space as the cross product of the discrete value
sets of all tuning parameters, restricted by a-priori constraints; Sect. 3.7
(input TS of Alg. 1) treats it as an array holding every valid configuration.

Readings (the paper fixes no order or constraint language):
* configurations are numbered by a mixed-radix index k, parameter 0 most
  significant, i.e. the order of ``itertools.product``;
* the array TS lists the valid configurations in ascending k;
* constraint kinds are DIV, DIV2, PROD_LE, PROD3_LE, PROD_GE and LE over the
  parameter *values* (see ``satisfies``); a divisibility test by zero fails.
"""
from __future__ import annotations

import itertools
from typing import List, Sequence, Tuple

import numpy as np


def satisfies(kind: str, a: int, b: int, c: int, bound: int, v: Sequence[int]) -> bool:
    """One constraint on the value vector ``v`` of a configuration (exact ints)."""
    if kind == "DIV":
        return v[b] != 0 and v[a] % v[b] == 0
    if kind == "DIV2":
        d = v[b] * v[c]
        return d != 0 and v[a] % d == 0
    if kind == "PROD_LE":
        return v[a] * v[b] <= bound
    if kind == "PROD3_LE":
        return v[a] * v[b] * v[c] <= bound
    if kind == "PROD_GE":
        return v[a] * v[b] >= bound
    if kind == "LE":
        return v[a] <= v[b]
    raise ValueError(f"unknown constraint kind {kind!r}")


def decode(k: int, radix: Sequence[int]) -> List[int]:
    """Digits of raw index ``k`` (parameter 0 most significant)."""
    digits = [0] * len(radix)
    for j in range(len(radix) - 1, -1, -1):
        digits[j] = k % radix[j]
        k //= radix[j]
    return digits


def enumerate_bruteforce(radix, values, constraints) -> List[int]:
    """Raw indices of valid configurations by walking the cross product.

    Pure-Python loops: only for small spaces.
    """
    valid = []
    for k, digits in enumerate(itertools.product(*[range(r) for r in radix])):
        v = [values[j][d] for j, d in enumerate(digits)]
        if all(satisfies(kind, a, b, c, bound, v) for (kind, a, b, c, bound) in constraints):
            valid.append(k)
    return valid


def digits_of(raw: np.ndarray, radix: Sequence[int]) -> np.ndarray:
    """Vectorised decode: int64 [n] raw indices -> int64 [n][P] digits."""
    raw = np.asarray(raw, dtype=np.int64)
    out = np.empty((raw.shape[0], len(radix)), dtype=np.int64)
    rest = raw.copy()
    for j in range(len(radix) - 1, -1, -1):
        out[:, j] = rest % radix[j]
        rest //= radix[j]
    return out


def _mask_vectorised(vals: List[np.ndarray], constraints) -> np.ndarray:
    ok = np.ones(vals[0].shape[0], dtype=bool)
    for (kind, a, b, c, bound) in constraints:
        va, vb, vc = vals[a], vals[b], vals[c]
        if kind == "DIV":
            nz = vb != 0
            ok &= nz & (np.remainder(va, np.where(nz, vb, 1)) == 0)
        elif kind == "DIV2":
            d = vb * vc
            nz = d != 0
            ok &= nz & (np.remainder(va, np.where(nz, d, 1)) == 0)
        elif kind == "PROD_LE":
            ok &= va * vb <= bound
        elif kind == "PROD3_LE":
            ok &= va * vb * vc <= bound
        elif kind == "PROD_GE":
            ok &= va * vb >= bound
        elif kind == "LE":
            ok &= va <= vb
        else:
            raise ValueError(kind)
    return ok


def valid_mask(radix, values, constraints, chunk: int = 1 << 22) -> np.ndarray:
    """Boolean [N_raw]: True where the configuration satisfies every constraint."""
    n_raw = int(np.prod(np.array(radix, dtype=object)))
    tables = [np.asarray(v, dtype=np.int64) for v in values]
    out = np.empty(n_raw, dtype=bool)
    for lo in range(0, n_raw, chunk):
        hi = min(n_raw, lo + chunk)
        d = digits_of(np.arange(lo, hi, dtype=np.int64), radix)
        vals = [tables[j][d[:, j]] for j in range(len(radix))]
        out[lo:hi] = _mask_vectorised(vals, constraints)
    return out


def enumerate_valid(radix, values, constraints) -> np.ndarray:
    """The array TS: valid raw indices, ascending, uint32."""
    return np.flatnonzero(valid_mask(radix, values, constraints)).astype(np.uint32)


def mask_words(mask: np.ndarray) -> np.ndarray:
    """Pack a boolean mask into uint32 words, bit i of word w <-> index 32w+i."""
    n = mask.shape[0]
    padded = np.zeros(((n + 31) // 32) * 32, dtype=bool)
    padded[:n] = mask
    bits = padded.reshape(-1, 32).astype(np.uint64)
    weights = (np.uint64(1) << np.arange(32, dtype=np.uint64))
    return (bits * weights).sum(axis=1).astype(np.uint32)
