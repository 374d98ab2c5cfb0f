"""Least-squares polynomial counter models (oracle; test infrastructure only),
Sect. 3.4.1.

The paper's first model family: the tuning space is split into subspaces by
the values of its binary parameters; in each subspace, every counter is
modelled as a polynomial in the non-binary parameters with main effects,
interactions (high orders included) and quadratic terms, its coefficients
fitted by least squares on deliberately chosen points (two or three values
of every non-binary parameter, spread evenly over its range).  Predictions
take the binary parameters' values to pick the subspace and evaluate that
subspace's polynomial at the non-binary values.

Readings (the paper fixes none of these details):

* binary parameters are the parameters with exactly two values; parameters
  with one value are constants and take no part; the others (three values
  or more) are non-binary;
* subspace index s = sum over the binary parameters, in parameter order, of
  digit * 2^i (i = the binary parameter's rank);
* feature of non-binary parameter j: x_j = (2 v - v_max - v_min) /
  (v_max - v_min), its value mapped affinely onto [-1, 1] (the span of the
  basis below is closed under such maps, so this changes no prediction in
  exact arithmetic; it only conditions the solve);
* basis, in this order: the products of x_j over every set S of non-binary
  parameters with |S| <= order (sets by size, then lexicographically;
  the empty set is the constant), then x_j^2 for every non-binary j;
* design (the points to measure): the valid configurations whose every
  non-binary digit is one of {0, m_j, R_j - 1}, m_j the digit whose value is
  nearest to (v_min + v_max) / 2 (the lower on a tie);
* fit per subspace: beta = (F^T F + lam I)^-1 F^T Y in float64 with
  lam = 1e-9 * trace(F^T F) / T, a ridge that keeps the solve defined when
  constraints leave the design rank-deficient; a subspace without training
  points has beta = 0;
* predictions are F(x) beta of the configuration's subspace, clamped at 0:
  the score equation (Sect. 3.6) divides by the sum of two counters and
  assumes both are non-negative, so a negative polynomial value would let a
  term leave [-1, 1] or divide by zero.  A clamped prediction of exactly 0
  drops the counter from PC_used for that configuration.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

RIDGE = 1e-9


def roles(radix):
    """(binary parameters, non-binary parameters) in parameter order."""
    b = [j for j, r in enumerate(radix) if int(r) == 2]
    nb = [j for j, r in enumerate(radix) if int(r) >= 3]
    return b, nb


def terms(n_nonbinary: int, order: int):
    """The basis as tuples of non-binary positions (0..k-1): subsets by size
    then lexicographically, then the squares (j, j)."""
    k = int(n_nonbinary)
    out = []
    for size in range(0, min(order, k) + 1):
        out.extend(itertools.combinations(range(k), size))
    out.extend((j, j) for j in range(k))
    return out


def features(values, radix, digits):
    """x [n][k] float64 for configurations given by digits [n][P]."""
    _, nb = roles(radix)
    digits = np.asarray(digits, dtype=np.int64)
    x = np.empty((len(digits), len(nb)), dtype=np.float64)
    for i, j in enumerate(nb):
        v = np.asarray(values[j], dtype=np.float64)
        lo, hi = v[0], v[-1]
        x[:, i] = (2.0 * v[digits[:, j]] - hi - lo) / (hi - lo)
    return x


def basis(x, order: int) -> np.ndarray:
    """F [n][T]: every basis term evaluated at x."""
    tt = terms(x.shape[1], order)
    F = np.ones((x.shape[0], len(tt)), dtype=np.float64)
    for t, S in enumerate(tt):
        for j in S:
            F[:, t] *= x[:, j]
    return F


def subspace(radix, digits) -> np.ndarray:
    """Subspace index of each configuration."""
    b, _ = roles(radix)
    digits = np.asarray(digits, dtype=np.int64)
    s = np.zeros(len(digits), dtype=np.int64)
    for i, j in enumerate(b):
        s += digits[:, j] << i
    return s


def mid_digit(values) -> int:
    """Digit whose value is nearest to the middle of the value range."""
    v = np.asarray(values, dtype=np.float64)
    m = (v[0] + v[-1]) / 2.0
    return int(np.argmin(np.abs(v - m)))     # first minimum: the lower digit


def design(values, radix, valid_digits) -> np.ndarray:
    """Indices (into the valid list) of the design configurations."""
    _, nb = roles(radix)
    d = np.asarray(valid_digits, dtype=np.int64)
    keep = np.ones(len(d), dtype=bool)
    for j in nb:
        levels = {0, mid_digit(values[j]), int(radix[j]) - 1}
        keep &= np.isin(d[:, j], sorted(levels))
    return np.flatnonzero(keep)


@dataclass
class PolyModel:
    order: int
    n_subspaces: int
    terms: list
    beta: np.ndarray        # float64 [S][T][C]
    lam: np.ndarray         # ridge per subspace
    count: np.ndarray       # training points per subspace


def fit(values, radix, digits, Y, order: int) -> PolyModel:
    """Least-squares fit of every subspace's polynomials (float64)."""
    b, nb = roles(radix)
    Y = np.asarray(Y, dtype=np.float64)
    S = 1 << len(b)
    tt = terms(len(nb), order)
    T, C = len(tt), Y.shape[1]
    F = basis(features(values, radix, digits), order)
    s = subspace(radix, digits)
    beta = np.zeros((S, T, C), dtype=np.float64)
    lam = np.zeros(S)
    count = np.zeros(S, dtype=np.int64)
    for k in range(S):
        rows = s == k
        count[k] = int(rows.sum())
        if count[k] == 0:
            continue
        G = F[rows].T @ F[rows]
        R = F[rows].T @ Y[rows]
        lam[k] = RIDGE * np.trace(G) / T
        beta[k] = np.linalg.solve(G + lam[k] * np.eye(T), R)
    return PolyModel(order, S, tt, beta, lam, count)


def value(model: PolyModel, values, radix, digits) -> np.ndarray:
    """The fitted polynomials' values [n][C] in float64 (unclamped)."""
    F = basis(features(values, radix, digits), model.order)
    s = subspace(radix, digits)
    return np.einsum("nt,ntc->nc", F, model.beta[s])


def predict(model: PolyModel, values, radix, digits) -> np.ndarray:
    """Predicted counters [n][C] in float64: the polynomial values clamped
    at 0 (counters are non-negative)."""
    return np.maximum(value(model, values, radix, digits), 0.0)


def abs_terms(model: PolyModel, values, radix, digits) -> np.ndarray:
    """sum over t of |F_t beta_tc| per configuration and counter: the scale
    of the rounding error of any evaluation of the polynomial."""
    F = basis(features(values, radix, digits), model.order)
    s = subspace(radix, digits)
    return np.einsum("nt,ntc->nc", np.abs(F), np.abs(model.beta[s]))
