"""Multilayer-perceptron surrogate of the counter model (oracle).

An extension of the method: the model of Sect. 3.4 maps tuning parameters to
predicted counters; here a three-layer perceptron plays that role next to
the decision trees.  Everything is plain float64 NumPy:

  features   x_j = digit_j / 8 (digit = index of parameter j's value)
  layers     z1 = W1 x + b1, h1 = gelu(z1); z2 = W2 h1 + b2, h2 = gelu(z2);
             y = W3 h2 + b3
  gelu       z Phi(z) = 0.5 z erfc(-z / sqrt 2)           (exact form; the
             erfc spelling of 0.5 z (1 + erf(z / sqrt 2)) keeps its
             relative accuracy for z << 0, where 1 + erf cancels)
  loss       mean over batch and counters of (y - target)^2
  backward   hand-written chain rule (no autodiff)
  optimiser  Adam (Kingma & Ba, "Adam: a method for stochastic optimization",
             ICLR 2015, Algorithm 1) with bias correction
  inference  predictions max(y, 0): the score equation needs non-negative
             counters (a prediction of exactly 0 drops the counter from
             PC_used)

``bf16`` rounds to bfloat16 (round to nearest even), used to feed the oracle
the same weights the device computes with.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def features(digits: np.ndarray) -> np.ndarray:
    return np.asarray(digits, dtype=np.float64) / 8.0


def gelu(z):
    return 0.5 * z * erfc(-z / SQRT2)


def gelu_grad(z):
    """d/dz gelu(z) = Phi(z) + z phi(z)."""
    return 0.5 * erfc(-z / SQRT2) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def bf16(x) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even); returns float32."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).reshape(f.shape)


def forward(params, X):
    """params = [W1, b1, W2, b2, W3, b3]; X [n][F].  Returns (y, cache)."""
    W1, b1, W2, b2, W3, b3 = params
    z1 = X @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    y = h2 @ W3.T + b3
    return y, (X, z1, h1, z2, h2)


def forward_bf16(params, X, round_activations: bool = True):
    """The forward pass with the device's precision choices: weights and the
    inputs rounded to bf16, biases kept, the hidden activations h1 and h2
    rounded to bf16; every sum in float64.  Returns y (float64)."""
    W1, b1, W2, b2, W3, b3 = params
    w1, w2, w3 = (bf16(w).astype(np.float64) for w in (W1, W2, W3))
    r = (lambda a: bf16(a).astype(np.float64)) if round_activations else (lambda a: a)
    x = bf16(X).astype(np.float64)
    h1 = r(gelu(x @ w1.T + b1))
    h2 = r(gelu(h1 @ w2.T + b2))
    return h2 @ w3.T + b3


# ------------------------------------------------ bounds of a device forward
# A forward pass with the device's precision choices (bf16 weights, inputs and
# hidden activations, biases in float32, products summed in float32, GELU's
# tail by the exponential of a fitted polynomial) differs from forward_bf16 by:
#   * summation: any order of K float32 additions (round to nearest, or any
#     rounding of at most one float32 ulp) errs by at most
#     (K + 1) 2^-23 (sum |w x| + |b|), plus 2^-126 per product for a
#     flushed subnormal;
#   * GELU: max(z, 0) - |z| Phi(-|z|) with Phi(-x) taken as
#     2^p(min(x, GELU_TAIL_MAX)), p within TAIL_LOG2_ERR of log2 Phi(-x) on
#     [0, GELU_TAIL_MAX] in its float32 evaluation, and an exponential within
#     one float32 ulp: the tail term errs by at most
#     rho = 2^TAIL_LOG2_ERR - 1 + 2^-22 of itself for |z| <= GELU_TAIL_MAX
#     and by at most 2 (1 + rho) |z| Phi(-GELU_TAIL_MAX) beyond; one final
#     rounding (2^-24 |gelu(z)|); doubled for safety;
#   * bf16 rounding of an activation: the device rounds its float32 GELU
#     value, which lies within the two bounds above of the exact GELU of the
#     exact pre-activation; rounding is monotone, so the device's bf16 value
#     lies between the roundings of the interval's ends, and equals the
#     oracle's whenever no rounding boundary falls inside the interval.
TAIL_LOG2_ERR = 1.15e-4
GELU_TAIL_MAX = 6.0
_RHO = 2.0 ** TAIL_LOG2_ERR - 1.0 + 2.0 ** -22
_PHI_CUT = 0.5 * math.erfc(GELU_TAIL_MAX / SQRT2)


def gelu_error_bound(z):
    """Bound of |device GELU(z) - gelu(z)| for float32 evaluation (above)."""
    az = np.abs(z)
    tail = az * 0.5 * erfc(az / SQRT2)
    t = np.where(az <= GELU_TAIL_MAX, _RHO * tail, 2.0 * (1.0 + _RHO) * az * _PHI_CUT)
    return 2.0 * (t + 2.0 ** -24 * np.abs(gelu(z))) + 1e-30


def _sum_bound(absW, absA, absb, K):
    return (K + 1) * 2.0 ** -23 * (absA @ absW.T + absb) + K * 2.0 ** -126


def _bf16_range(g, dg):
    """bf16 values a float32 rounding of anything in [g - dg, g + dg] can give."""
    lo32 = np.asarray(g - dg, np.float32)
    lo32 = np.where(lo32.astype(np.float64) > g - dg, np.nextafter(lo32, np.float32(-np.inf)), lo32)
    hi32 = np.asarray(g + dg, np.float32)
    hi32 = np.where(hi32.astype(np.float64) < g + dg, np.nextafter(hi32, np.float32(np.inf)), hi32)
    return bf16(lo32).astype(np.float64), bf16(hi32).astype(np.float64)


def forward_bf16_interval(params, X):
    """forward_bf16's output y and a bound E with |y_device - y| <= E for
    every device forward with the precision choices above (the same bf16
    weights, inputs and activation rounding, float32 sums in any order, a
    GELU within gelu_error_bound).  Returns (y, E), both [n][C] float64."""
    W1, b1, W2, b2, W3, b3 = params
    w1, w2, w3 = (bf16(w).astype(np.float64) for w in (W1, W2, W3))
    b1, b2, b3 = (np.asarray(b, np.float32).astype(np.float64) for b in (b1, b2, b3))
    x = bf16(X).astype(np.float64)
    K1, H = w1.shape[1], w1.shape[0]
    # layer 1: exact inputs and weights; only the sum rounds
    z1 = x @ w1.T + b1
    dz1 = _sum_bound(np.abs(w1), np.abs(x), np.abs(b1), K1)
    g1 = gelu(z1)
    dg1 = 1.1295 * dz1 + gelu_error_bound(z1)      # |gelu'| <= 1.1295
    h1 = bf16(g1).astype(np.float64)
    lo, hi = _bf16_range(g1, dg1)
    dh1 = np.maximum(h1 - lo, hi - h1)
    # layer 2: the device's h1 differs by at most dh1
    z2 = h1 @ w2.T + b2
    a2 = np.abs(w2)
    dz2 = dh1 @ a2.T + _sum_bound(a2, np.abs(h1) + dh1, np.abs(b2), H)
    g2 = gelu(z2)
    dg2 = 1.1295 * dz2 + gelu_error_bound(z2)
    h2 = bf16(g2).astype(np.float64)
    lo, hi = _bf16_range(g2, dg2)
    dh2 = np.maximum(h2 - lo, hi - h2)
    a3 = np.abs(w3)
    y = h2 @ w3.T + b3
    E = dh2 @ a3.T + _sum_bound(a3, np.abs(h2) + dh2, np.abs(b3), H)
    return y, E


def predict(params, X) -> np.ndarray:
    return np.maximum(forward(params, X)[0], 0.0)


def loss_and_grads(params, X, T):
    """MSE loss and its gradients for every parameter (same order as params)."""
    W1, b1, W2, b2, W3, b3 = params
    y, (X, z1, h1, z2, h2) = forward(params, X)
    n, C = y.shape
    diff = y - T
    loss = float((diff * diff).sum() / (n * C))
    dy = 2.0 * diff / (n * C)
    dW3 = dy.T @ h2
    db3 = dy.sum(axis=0)
    dz2 = (dy @ W3) * gelu_grad(z2)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * gelu_grad(z1)
    dW1 = dz1.T @ X
    db1 = dz1.sum(axis=0)
    return loss, [dW1, db1, dW2, db2, dW3, db3]


class Adam:
    """Kingma & Ba, Algorithm 1."""

    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        out = []
        for i, (p, g) in enumerate(zip(params, grads)):
            self.m[i] = self.b1 * self.m[i] + (1.0 - self.b1) * g
            self.v[i] = self.b2 * self.v[i] + (1.0 - self.b2) * g * g
            mhat = self.m[i] / (1.0 - self.b1 ** self.t)
            vhat = self.v[i] / (1.0 - self.b2 ** self.t)
            out.append(p - self.lr * mhat / (np.sqrt(vhat) + self.eps))
        return out


def init_params(init) -> list:
    """float64 copies of a synth.MLPInit."""
    return [init.w[0].astype(np.float64), init.b[0].astype(np.float64),
            init.w[1].astype(np.float64), init.b[1].astype(np.float64),
            init.w[2].astype(np.float64), init.b[2].astype(np.float64)]


def train(params, X_all, T_all, batches, lr=1e-3):
    """Adam over the given minibatch index rows; returns (params, losses)."""
    opt = Adam(params, lr=lr)
    losses = []
    for idx in batches:
        loss, g = loss_and_grads(params, X_all[idx], T_all[idx])
        losses.append(loss)
        params = opt.step(params, g)
    return params, losses
