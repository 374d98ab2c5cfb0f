"""Seeded synthetic inputs for the counter-guided search sweep.

This module only draws random numbers and fixes shapes: parameter value
tables, constraint lists, random regression forests (feature / threshold /
leaf arrays), bottleneck-change vectors, 64-bit uniforms, synthetic profiler
counters, noise and network initialisations.  It evaluates no constraint,
traverses no tree, scores, normalises or samples nothing: the CPU oracle and
the GPU library both consume these arrays and each does the method's
arithmetic on its own.

Workload shapes follow the paper's evaluation: tuning spaces of 6-16
parameters with small discrete value sets (binary switches and powers of two,
Sect. 3.4.1 and Table 2), a-priori constraints that remove most of the cross
product (Sect. 1), and the 24 hardware counters of Table 1.

Every generator is keyed by a fixed root seed and a spawn key, so the same
call always yields the same arrays.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

ROOT_SEED = 210205297

# Constraint kinds, by name.  Both sides map the names to their own codes.
#   DIV       v[a] % v[b] == 0
#   DIV2      v[a] % (v[b] * v[c]) == 0
#   PROD_LE   v[a] * v[b] <= bound
#   PROD3_LE  v[a] * v[b] * v[c] <= bound
#   PROD_GE   v[a] * v[b] >= bound
#   LE        v[a] <= v[b]
CONSTRAINT_KINDS = ("DIV", "DIV2", "PROD_LE", "PROD3_LE", "PROD_GE", "LE")

# Table 1 counter names in table order (17 operation counters, then 7 stress
# counters).  Index p of every counter axis in this project is this order.
TABLE1_COUNTERS = (
    "DRAM_RT", "DRAM_WT", "L2_RT", "L2_WT", "TEX_RWT", "LOC_O", "SHR_LT",
    "SHR_WT", "INST_F32", "INST_F64", "INST_INT", "INST_MISC", "INST_LDST",
    "INST_CONT", "INST_BCONV", "INST_EXE", "INST_ISSUE_U", "DRAM_U", "L2_U",
    "TEX_U", "SHR_U", "SM_E", "WARP_E", "WARP_NP_E",
)


def rng(*key: int) -> np.random.Generator:
    """Independent generator for spawn key ``key`` under the root seed."""
    ss = np.random.SeedSequence(ROOT_SEED, spawn_key=tuple(int(k) for k in key))
    return np.random.Generator(np.random.PCG64(ss))


# --------------------------------------------------------------------------
# Tuning spaces
# --------------------------------------------------------------------------
@dataclass
class Space:
    """A tuning space: per-parameter ascending value tables + constraints.

    ``constraints`` holds tuples ``(kind, a, b, c, bound)`` with ``kind`` one
    of :data:`CONSTRAINT_KINDS`; unused fields are 0.
    """
    radix: List[int]
    values: List[List[int]]
    constraints: List[Tuple[str, int, int, int, int]] = field(default_factory=list)

    @property
    def n_params(self) -> int:
        return len(self.radix)

    @property
    def n_raw(self) -> int:
        return int(np.prod(np.array(self.radix, dtype=object)))


def value_tables(radix: Sequence[int], binary_radix2: bool) -> List[List[int]]:
    """Powers of two 2^0..2^(r-1); radix-2 parameters optionally binary {0,1}."""
    out = []
    for r in radix:
        if r == 2 and binary_radix2:
            out.append([0, 1])
        else:
            out.append([1 << i for i in range(r)])
    return out


def _quantile_bound(g: np.random.Generator, tables: Sequence[Sequence[int]], lo: float,
                    hi: float) -> int:
    """A product of one value per table, at a seeded quantile in [lo, hi) of
    all such products (the bound is a value some configuration reaches)."""
    prods = np.array([1], dtype=np.int64)
    for t in tables:
        prods = (prods[:, None] * np.asarray(t, dtype=np.int64)[None, :]).ravel()
    prods.sort()
    u = g.uniform(lo, hi)
    return int(prods[min(len(prods) - 1, int(u * len(prods)))])


def random_constraints(g: np.random.Generator, values: List[List[int]], n: int,
                       kinds: Sequence[str], loose: float = 0.0) -> List[Tuple[str, int, int, int, int]]:
    """Draw ``n`` constraints over parameters whose tables hold no zero.

    Upper bounds sit at a seeded quantile in [loose, 1) of the attainable
    products, lower bounds in [0, 1 - loose), so ``loose`` > 0 makes each
    product constraint keep more of the space.
    """
    usable = [j for j, v in enumerate(values) if len(v) > 1 and min(v) > 0]
    cons = []
    for _ in range(n):
        kind = str(g.choice(list(kinds)))
        a, b, c = (int(x) for x in g.choice(usable, size=3, replace=False))
        bound = 0
        if kind == "PROD_LE":
            bound = _quantile_bound(g, [values[a], values[b]], loose, 1.0)
            c = 0
        elif kind == "PROD_GE":
            bound = _quantile_bound(g, [values[a], values[b]], 0.0, 1.0 - loose)
            c = 0
        elif kind == "PROD3_LE":
            bound = _quantile_bound(g, [values[a], values[b], values[c]], loose, 1.0)
        elif kind in ("DIV", "LE"):
            c = 0
        cons.append((kind, a, b, c, bound))
    return cons


# Variants below were picked once, offline, so that the share of the cross
# product surviving the constraints lands in the ranges the paper reports
# for its benchmarks (0.025 % - 41.7 %, Sect. 4.6); the oracle tests assert
# the resulting counts.
C1_VARIANT = 48
C2_VARIANT = 11
C5_VARIANT = 103

C1_RADIX = (4, 4, 5, 6, 8, 8)
C2_RADIX = (8, 4, 2, 8, 4, 2, 8, 4, 2, 4, 4, 4)
C5_RADIX = (4, 3, 2, 3, 4, 3, 4, 3, 2, 3, 4, 3, 4, 3, 4, 3)


def space_c1(variant: int = C1_VARIANT) -> Space:
    """6 parameters, 30,720 raw configurations, 3 divisibility/product constraints."""
    vals = value_tables(C1_RADIX, binary_radix2=False)
    cons = random_constraints(rng(1, 1, variant), vals, 3, ("DIV", "PROD_LE", "PROD3_LE"))
    return Space(list(C1_RADIX), vals, cons)


def space_c2(variant: int = C2_VARIANT) -> Space:
    """12 parameters, 2^24 raw configurations, 6 constraints."""
    vals = value_tables(C2_RADIX, binary_radix2=True)
    cons = random_constraints(rng(2, 1, variant), vals, 6,
                              ("DIV", "DIV2", "PROD_LE", "PROD3_LE", "PROD_GE", "LE"), loose=0.5)
    return Space(list(C2_RADIX), vals, cons)


def space_c5(variant: int = C5_VARIANT) -> Space:
    """16 parameters, 2^14 * 3^8 = 107,495,424 raw configurations, 10 constraints."""
    vals = value_tables(C5_RADIX, binary_radix2=True)
    cons = random_constraints(rng(5, 1, variant), vals, 10,
                              ("DIV", "PROD_LE", "PROD3_LE", "PROD_GE", "LE"), loose=0.6)
    return Space(list(C5_RADIX), vals, cons)


C5_SLICE_RADIX = (3, 2, 2, 3, 2, 2, 2, 3, 2, 2, 2, 2, 2, 2, 2, 2)
C5_SLICE_VARIANT = 2


def space_c5_slice(variant: int = C5_SLICE_VARIANT) -> Space:
    """16 parameters like the large space but 2^13 * 3^3 = 221,184 raw
    configurations and 4 constraints: a size at which the oracle evaluates
    the 16 -> 512 -> 512 -> 32 perceptron on every configuration."""
    vals = value_tables(C5_SLICE_RADIX, binary_radix2=True)
    cons = random_constraints(rng(7, 1, variant), vals, 4,
                              ("DIV", "PROD_LE", "PROD3_LE", "PROD_GE", "LE"), loose=0.6)
    return Space(list(C5_SLICE_RADIX), vals, cons)


def fit_radices(g: np.random.Generator, target: float, n_params: int) -> List[int]:
    """Greedy radices in {2..8} whose product approaches ``target`` from below."""
    radix = [2] * n_params
    prod = 2 ** n_params
    order = list(g.permutation(n_params))
    improved = True
    while improved:
        improved = False
        for j in order:
            r = radix[j]
            if r < 8 and prod // r * (r + 1) <= target:
                prod = prod // r * (r + 1)
                radix[j] = r + 1
                improved = True
    return radix


def space_batch(session: int) -> Space:
    """One of the 64 batched sessions: log10(N_raw) ~ U(4,7), 8-14 parameters."""
    g = rng(4, 1, session)
    target = 10.0 ** g.uniform(4.0, 7.0)
    n_params = int(g.integers(8, 15))
    radix = fit_radices(g, target, n_params)
    vals = value_tables(radix, binary_radix2=False)
    n_cons = int(math.ceil(n_params / 3))
    cons = random_constraints(g, vals, n_cons, ("DIV", "PROD_LE", "PROD3_LE", "PROD_GE", "LE"),
                              loose=0.4)
    return Space(radix, vals, cons)


# --------------------------------------------------------------------------
# Random regression forests (complete binary trees in heap layout)
# --------------------------------------------------------------------------
@dataclass
class Forest:
    """``feat``/``thr``: uint8 [T][2^D-1]; ``leaves``: float32 [T][2^D][C]."""
    n_trees: int
    depth: int
    n_counters: int
    feat: np.ndarray
    thr: np.ndarray
    leaves: np.ndarray


def random_forest(g: np.random.Generator, radix: Sequence[int], n_trees: int, depth: int,
                  n_counters: int) -> Forest:
    """Splits on random parameters (radix > 1) at random digit thresholds
    0..r-2; leaf counter vectors ~ U(0,1) in float32."""
    n_int = (1 << depth) - 1
    splittable = np.array([j for j, r in enumerate(radix) if r > 1], dtype=np.int64)
    feat = splittable[g.integers(0, len(splittable), size=(n_trees, n_int))]
    r_of = np.asarray(radix, dtype=np.int64)[feat]
    thr = np.floor(g.random(size=(n_trees, n_int)) * (r_of - 1)).astype(np.int64)
    leaves = g.random(size=(n_trees, 1 << depth, n_counters), dtype=np.float32)
    return Forest(n_trees, depth, n_counters, feat.astype(np.uint8), thr.astype(np.uint8),
                  np.ascontiguousarray(leaves))


def forest_c1(space: Space) -> Forest:
    return random_forest(rng(1, 2), space.radix, 1, 8, 12)


def forest_c2(space: Space) -> Forest:
    return random_forest(rng(2, 2), space.radix, 16, 12, 24)


def forest_c5(space: Space) -> Forest:
    return random_forest(rng(5, 2), space.radix, 16, 12, 32)


def forest_batch(session: int, space: Space) -> Forest:
    return random_forest(rng(4, 2, session), space.radix, 8, 10, 16)


# --------------------------------------------------------------------------
# Per-step random inputs
# --------------------------------------------------------------------------
def deltas(g: np.random.Generator, n: int, n_counters: int) -> np.ndarray:
    """Bottleneck-change vectors ~ U(-1,1), float32 [n][C]."""
    return (g.random(size=(n, n_counters), dtype=np.float64) * 2.0 - 1.0).astype(np.float32)


def uniforms_u64(g: np.random.Generator, n: int) -> np.ndarray:
    """Uniform 64-bit integers, the random input of each weighted draw."""
    return g.integers(0, np.iinfo(np.uint64).max, size=n, dtype=np.uint64, endpoint=True)


def profiler_counters(g: np.random.Generator, n: int) -> np.ndarray:
    """Synthetic Table 1 counter vectors (float64 [n][24]) in the pre-Volta scales.

    Utilisations DRAM_U, L2_U, TEX_U, SHR_U lie in 0..10; LOC_O,
    INST_ISSUE_U, SM_E, WARP_E, WARP_NP_E in 0..100.  Transaction counts are
    counts.  Thread-level instruction counts split 32 * INST_EXE (scaled by
    both warp efficiencies) over the seven instruction classes by a random
    mix, so a class occasionally dominates.
    """
    out = np.zeros((n, 24), dtype=np.float64)
    for i in range(n):
        inst_exe = g.uniform(1e5, 1e6)
        we = g.uniform(80.0, 100.0)
        wnpe = g.uniform(80.0, 100.0)
        mix = g.dirichlet(np.full(7, 0.35))
        thread_inst = 32.0 * inst_exe * (we / 100.0) * (wnpe / 100.0)
        rt, wt = g.uniform(0, 1e6, size=2)
        l2r, l2w = g.uniform(0, 4e6, size=2)
        out[i, 0:4] = (rt, wt, l2r, l2w)
        out[i, 4] = g.uniform(0, 8e6)                  # TEX_RWT
        out[i, 5] = g.uniform(0, 60.0)                 # LOC_O (percent)
        out[i, 6:8] = g.uniform(0, 2e6, size=2)        # SHR_LT, SHR_WT
        out[i, 8:15] = thread_inst * mix               # INST_F32 .. INST_BCONV
        out[i, 15] = inst_exe
        out[i, 16] = g.uniform(20.0, 100.0)            # INST_ISSUE_U
        out[i, 17:21] = g.uniform(0.0, 10.0, size=4)   # DRAM_U L2_U TEX_U SHR_U
        out[i, 21] = g.uniform(40.0, 100.0)            # SM_E
        out[i, 22] = we
        out[i, 23] = wnpe
    return out


def threads_launched(g: np.random.Generator, n: int) -> np.ndarray:
    """Threads of the profiled launch (for the parallelism bottleneck)."""
    return np.floor(g.uniform(1e3, 2e4, size=n))


def normal_noise(g: np.random.Generator, shape, sigma: float) -> np.ndarray:
    return (g.standard_normal(size=shape) * sigma).astype(np.float32)


def he_uniform(g: np.random.Generator, fan_out: int, fan_in: int) -> np.ndarray:
    """Weight matrix [fan_out][fan_in] ~ U(-sqrt(6/fan_in), sqrt(6/fan_in)), float32."""
    lim = math.sqrt(6.0 / fan_in)
    return ((g.random(size=(fan_out, fan_in)) * 2.0 - 1.0) * lim).astype(np.float32)


@dataclass
class MLPInit:
    """Three-layer perceptron: W1 [H][F], W2 [H][H], W3 [C][H], biases 0."""
    sizes: Tuple[int, int, int, int]
    w: List[np.ndarray]
    b: List[np.ndarray]


def mlp_init(key: Tuple[int, ...], n_in: int, hidden: int, n_out: int) -> MLPInit:
    g = rng(*key)
    dims = [(hidden, n_in), (hidden, hidden), (n_out, hidden)]
    w = [he_uniform(g, o, i) for (o, i) in dims]
    b = [np.zeros(o, dtype=np.float32) for (o, _) in dims]
    return MLPInit((n_in, hidden, hidden, n_out), w, b)


def minibatches(g: np.random.Generator, n_steps: int, batch: int, n_pairs: int) -> np.ndarray:
    """Indices into the training pairs, int32 [n_steps][batch]."""
    return g.integers(0, n_pairs, size=(n_steps, batch), dtype=np.int64).astype(np.int32)


def uniform_indices(g: np.random.Generator, n: int, upper: int) -> np.ndarray:
    """``n`` uniform integers in [0, upper), int64 (e.g. positions in a valid list)."""
    return g.integers(0, upper, size=n, dtype=np.int64)


# --------------------------------------------------------------------------
# Measured (configuration, counter) pairs for model fitting
# --------------------------------------------------------------------------
def measured_counters(g: np.random.Generator, digits: np.ndarray, radix: Sequence[int],
                      n_counters: int, noise: float = 0.02) -> np.ndarray:
    """Synthetic measured counters of configurations, float32 [n][C].

    Each counter is a sum of four axis-aligned steps on random parameters
    (what a tuning parameter switching a code path does), a smooth product
    of two normalised parameter values and multiplicative Gaussian noise; the
    counters' magnitudes spread over eight decades, like transaction counts
    next to utilisation percentages."""
    digits = np.asarray(digits)
    n, P = digits.shape
    x = (digits / np.maximum(np.asarray(radix, dtype=np.float64) - 1.0, 1.0)).astype(np.float32)
    xt = np.ascontiguousarray(x.T)
    Yt = np.empty((n_counters, n), dtype=np.float32)
    for c in range(n_counters):
        js = g.integers(0, P, 4)
        th = g.random(4).astype(np.float32)
        w = (g.random(4) + 0.2).astype(np.float32)
        a, b = g.integers(0, P, 2)
        scale = np.float32(10.0 ** g.uniform(-2.0, 6.0))
        v = np.float32(0.5) * xt[a] * xt[b] + np.float32(0.1)
        for k in range(4):
            v += np.where(xt[js[k]] > th[k], w[k], np.float32(0.0))
        v *= np.float32(1.0) + np.float32(noise) * g.standard_normal(n, dtype=np.float32)
        np.multiply(v, scale, out=Yt[c])
    return np.ascontiguousarray(Yt.T)


# --------------------------------------------------------------------------
# A synthetic GPU kernel: runtime and Table 1 counters of every configuration
# --------------------------------------------------------------------------
@dataclass
class KernelTable:
    """Measured runtimes [Nv] (float32, seconds) and Table 1 counter vectors
    [Nv][24] (float64, pre-Volta scales) of every valid configuration."""
    runtime: np.ndarray
    counters: np.ndarray


def kernel_table(g: np.random.Generator, digits: np.ndarray, radix: Sequence[int]) -> KernelTable:
    """A synthetic kernel whose bottlenecks decide its runtime.

    Every configuration moves work between four memory resources (DRAM, L2,
    texture, shared memory) and the instruction pipes: each resource's
    transaction count is base * exp(sum_j a_rj (x_j - 1/2)) over the
    parameters' normalised digits x_j, with random slopes a_rj (a tiling
    parameter lowers DRAM traffic and raises shared-memory traffic, say).
    Each resource's time is its count over its peak rate; the runtime is the
    slowest resource's time over the SM efficiency, so the counters of the
    bottleneck show full utilisation (10 on the 0..10 scale) and the others
    show their share of the runtime.  Instruction counts split over the seven
    classes by a parameter-dependent mix; warp efficiencies 80..100%."""
    digits = np.asarray(digits)
    n, P = digits.shape
    x = digits / np.maximum(np.asarray(radix, dtype=np.float64) - 1.0, 1.0) - 0.5
    def work(scale, spread):
        a = g.normal(0.0, spread, size=P)
        return scale * np.exp(x @ a)
    dram, l2, tex, shr = work(4e5, 1.2), work(2e6, 1.0), work(3e6, 0.8), work(1e6, 1.4)
    inst = work(2e5, 0.9)
    rd = g.uniform(0.5, 0.9, size=4)                    # read share per resource
    t_mem = np.stack([dram / 1.0e6, l2 / 4.0e6, tex / 6.0e6, shr / 2.5e6])
    t_inst = inst / 6.0e5
    sm_e = 100.0 * (0.7 + 0.3 / (1.0 + np.exp(-(x @ g.normal(0.0, 2.0, size=P)))))
    we = 100.0 * (0.85 + 0.15 / (1.0 + np.exp(-(x @ g.normal(0.0, 2.0, size=P)))))
    wnpe = 100.0 * (0.8 + 0.2 / (1.0 + np.exp(-(x @ g.normal(0.0, 2.0, size=P)))))
    t_busy = np.maximum(t_mem.max(axis=0), t_inst)
    runtime = t_busy / (sm_e / 100.0) * 1e-3 + 2e-6
    mix = np.abs(g.dirichlet(np.full(7, 0.5)) + 0.2 * np.tanh(x @ g.normal(0.0, 1.0, size=(P, 7))))
    mix /= mix.sum(axis=1, keepdims=True)
    c = np.zeros((n, 24), dtype=np.float64)
    for i, (tot, r) in enumerate(zip((dram, l2, tex, shr), rd)):
        if i == 2:
            c[:, 4] = tot                                # TEX_RWT
        else:
            k = {0: 0, 1: 2, 3: 6}[i]
            c[:, k], c[:, k + 1] = tot * r, tot * (1.0 - r)
    c[:, 5] = 60.0 / (1.0 + np.exp(-(x @ g.normal(0.0, 3.0, size=P)) - 2.0))     # LOC_O
    c[:, 8:15] = (32.0 * inst * (we / 100.0) * (wnpe / 100.0))[:, None] * mix
    c[:, 15] = inst
    c[:, 16] = 100.0 * t_inst / t_busy                                            # INST_ISSUE_U
    c[:, 17:21] = (10.0 * t_mem / t_busy).T                                       # DRAM_U .. SHR_U
    c[:, 21], c[:, 22], c[:, 23] = sm_e, we, wnpe
    return KernelTable(runtime.astype(np.float32), c)
