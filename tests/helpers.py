"""Shared helpers for the GPU parity tests (inputs only; no method arithmetic)."""
import json
import os

import numpy as np

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def cgs():
    """The HIP binding; raises ImportError (a failure, not a skip) when the
    library was not built."""
    from paper_2102_05297_amd import cgs as mod
    return mod


def golden(name):
    with open(os.path.join(GOLDEN_DIR, name)) as f:
        return json.load(f)


def bits_to_bool(words: np.ndarray, n: int) -> np.ndarray:
    b = ((words[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1).astype(bool)
    return b.ravel()[:n]


def random_small_space(g: np.random.Generator, max_params=5, max_radix=6):
    """A random small space (radices, ascending value tables incl. zero and
    negative values, random constraints)."""
    n_params = int(g.integers(1, max_params + 1))
    radix = [int(g.integers(1, max_radix + 1)) for _ in range(n_params)]
    values = [sorted(g.choice(np.arange(-6, 40), size=r, replace=False).tolist()) for r in radix]
    cons = []
    kinds = ("DIV", "DIV2", "PROD_LE", "PROD3_LE", "PROD_GE", "LE")
    for _ in range(int(g.integers(0, 5))):
        kind = kinds[int(g.integers(0, len(kinds)))]
        a, b, c = (int(x) for x in g.integers(0, n_params, size=3))
        cons.append((kind, a, b, c, int(g.integers(-50, 400))))
    return radix, values, cons
