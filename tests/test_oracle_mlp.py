"""Oracle pins: the perceptron surrogate's forward, backward, Adam and bf16
rounding (plain float64; see oracle/mlp.py)."""
import numpy as np
from scipy.special import erfc
import pytest

from oracle import mlp as M


def _toy(seed, F=5, H=7, C=3, n=16):
    g = np.random.default_rng(seed)
    params = [g.normal(0, 0.5, (H, F)), g.normal(0, 0.1, H), g.normal(0, 0.5, (H, H)),
              g.normal(0, 0.1, H), g.normal(0, 0.5, (C, H)), g.normal(0, 0.1, C)]
    X = g.random((n, F))
    T = g.random((n, C))
    return params, X, T


@pytest.mark.parametrize("seed", range(3))
def test_backprop_matches_central_differences(seed):
    params, X, T = _toy(seed)
    _, grads = M.loss_and_grads(params, X, T)
    h = 1e-6
    for i, p in enumerate(params):
        num = np.zeros_like(p)
        flat = p.reshape(-1)
        for j in range(flat.size):
            old = flat[j]
            flat[j] = old + h
            lp, _ = M.loss_and_grads(params, X, T)
            flat[j] = old - h
            lm, _ = M.loss_and_grads(params, X, T)
            flat[j] = old
            num.reshape(-1)[j] = (lp - lm) / (2 * h)
        err = np.abs(num - grads[i]).max() / max(1e-12, np.abs(num).max())
        assert err < 1e-6, (i, err)


def test_gelu_closed_forms():
    x = np.linspace(-6, 6, 241)
    assert M.gelu(0.0) == 0.0
    # Phi(x) + Phi(-x) = 1  =>  gelu(x) - gelu(-x) = x
    assert np.allclose(M.gelu(x) - M.gelu(-x), x, atol=1e-15)
    assert M.gelu_grad(0.0) == 0.5
    assert abs(M.gelu(40.0) - 40.0) < 1e-12 and abs(M.gelu(-40.0)) < 1e-12
    # known value: gelu(1) = Phi(1) = 0.8413447460685429
    assert abs(M.gelu(1.0) - 0.8413447460685429) < 1e-15
    h = 1e-6
    assert np.allclose((M.gelu(x + h) - M.gelu(x - h)) / (2 * h), M.gelu_grad(x), atol=1e-8)


def test_adam_first_and_second_step_closed_form():
    p0 = [np.array([0.5, -1.0, 2.0])]
    g1 = np.array([0.2, -3.0, 1e-9])
    g2 = np.array([-0.1, 1.0, 4.0])
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    opt = M.Adam(p0, lr, b1, b2, eps)
    p1 = opt.step(p0, [g1])[0]
    # t = 1: mhat = g, vhat = g^2  ->  step = lr * g / (|g| + eps)
    assert np.allclose(p1, p0[0] - lr * g1 / (np.abs(g1) + eps), rtol=0, atol=1e-15)
    p2 = opt.step([p1], [g2])[0]
    m = b1 * (1 - b1) * g1 + (1 - b1) * g2
    v = b2 * (1 - b2) * g1 ** 2 + (1 - b2) * g2 ** 2
    mhat, vhat = m / (1 - b1 ** 2), v / (1 - b2 ** 2)
    assert np.allclose(p2, p1 - lr * mhat / (np.sqrt(vhat) + eps), rtol=0, atol=1e-15)


def test_bf16_rounding():
    vals = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 3.14159265, -2.5, 0.0, 1 + 2.0 ** -7],
                    dtype=np.float32)
    # ties to even at 1 + 2^-8; 1 + 3*2^-8 rounds up to 1 + 2^-6; pi -> 3.140625
    assert M.bf16(vals).tolist() == [1.0, 1.0, 1 + 2.0 ** -6, 3.140625, -2.5, 0.0, 1 + 2.0 ** -7]


def test_features_are_exact_eighths():
    d = np.array([[0, 1, 7, 15]])
    assert M.features(d).tolist() == [[0.0, 0.125, 0.875, 1.875]]
    assert (M.bf16(M.features(d).astype(np.float32)) == M.features(d)).all()


def test_training_reduces_loss_on_a_smooth_target():
    g = np.random.default_rng(4)
    F, H, C = 4, 16, 2
    X = g.random((512, F))
    T = np.stack([X @ np.array([1.0, -0.5, 0.25, 0.0]), np.sin(X[:, 0] * 3)], axis=1)
    params = [g.normal(0, (1 / F) ** 0.5, (H, F)), np.zeros(H), g.normal(0, (1 / H) ** 0.5, (H, H)),
              np.zeros(H), g.normal(0, (1 / H) ** 0.5, (C, H)), np.zeros(C)]
    batches = g.integers(0, 512, (300, 64))
    _, losses = M.train(params, X, T, batches, lr=1e-2)
    assert np.mean(losses[-20:]) < 0.1 * np.mean(losses[:5])


def test_bf16_forward_reduces_to_plain_forward():
    params, X, T = _toy(7, F=6, H=16, C=4, n=32)
    X = M.features(np.random.default_rng(1).integers(0, 8, (32, 6)))
    pb = [M.bf16(p.astype(np.float32)).astype(np.float64) if i % 2 == 0 else p
          for i, p in enumerate(params)]
    # without activation rounding it is the float64 forward of the rounded weights
    assert np.array_equal(M.forward_bf16(params, X, round_activations=False), M.forward(pb, X)[0])
    # with it, the output moves by at most the bf16 relative rounding (2^-9) of
    # each hidden value, propagated through |W3| and |W2|
    y = M.forward(pb, X)[0]
    yb = M.forward_bf16(params, X)
    _, (_, _, h1, _, h2) = M.forward(pb, X)
    w2, w3 = np.abs(pb[2]), np.abs(pb[4])
    bound = (np.abs(h2) @ w3.T + (np.abs(h1) @ w2.T) @ w3.T * 1.2) * 2.0 ** -8
    assert (np.abs(yb - y) <= bound + 1e-12).all()


# ------------------------------------------- bound of a device-like forward
# A float32 model of the device's arithmetic, written from its published
# description (not from the kernels): products of bf16 values summed in
# float32 in a random order, the bias added in float32, GELU as max(z, 0)
# minus |z| 2^p with p anywhere within the tail bound of
# log2 Phi(-min(|z|, GELU_TAIL_MAX))
# (the kernels' fitted polynomial stays within it), the exponential
# perturbed by up to 2 ulps, the subtraction rounded once (a fused
# multiply-add), then rounded to bf16.


def _ulps(g, v, k=2):
    for _ in range(int(g.integers(0, k + 1))):
        v = np.nextafter(v, np.where(g.random(v.shape) < 0.5, np.float32(np.inf),
                                     np.float32(-np.inf))).astype(np.float32)
    return v


def _gelu_f32(g, z):
    z = np.asarray(z, np.float32)
    az = np.abs(z).astype(np.float64)
    lp = np.log2(0.5 * erfc(np.minimum(az, M.GELU_TAIL_MAX) / np.sqrt(2.0)))
    p = (lp + g.uniform(-1.0, 1.0, np.shape(z)) * M.TAIL_LOG2_ERR).astype(np.float32)
    e = _ulps(g, np.exp2(p.astype(np.float64)).astype(np.float32)).astype(np.float64)
    return (np.maximum(z, np.float32(0)).astype(np.float64) - az * e).astype(np.float32)


def test_gelu_error_bound_covers_a_float32_evaluation():
    g = np.random.default_rng(5)
    z = np.concatenate([np.linspace(-15, 15, 400001), g.normal(0, 3, 100000),
                        [-40.0, -1e-30, 0.0, 1e-30, 40.0]]).astype(np.float32)
    for _ in range(3):
        got = _gelu_f32(g, z).astype(np.float64)
        zz = z.astype(np.float64)
        assert (np.abs(got - M.gelu(zz)) <= M.gelu_error_bound(zz)).all()


def _device_like_forward(g, params, X):
    W1, b1, W2, b2, W3, b3 = params
    h = M.bf16(X)
    for W, b, act in ((W1, b1, True), (W2, b2, True), (W3, b3, False)):
        w = M.bf16(W)
        z = np.zeros((h.shape[0], w.shape[0]), np.float32)
        for k in g.permutation(w.shape[1]):
            z = (z + np.outer(h[:, k], w[:, k]).astype(np.float32)).astype(np.float32)
        z = (z + np.asarray(b, np.float32)).astype(np.float32)
        h = M.bf16(_gelu_f32(g, z)) if act else z
    return h.astype(np.float64)


@pytest.mark.parametrize("seed,H", [(0, 16), (1, 64), (2, 64)])
def test_forward_bound_covers_device_like_forwards(seed, H):
    g = np.random.default_rng(seed)
    F_, C, n = 6, 5, 400
    params = [g.normal(0, 1.0, (H, F_)).astype(np.float32), g.normal(0, 0.5, H).astype(np.float32),
              g.normal(0, 2.0 / np.sqrt(H), (H, H)).astype(np.float32),
              g.normal(0, 0.5, H).astype(np.float32),
              g.normal(0, 2.0 / np.sqrt(H), (C, H)).astype(np.float32),
              g.normal(0, 0.5, C).astype(np.float32)]
    X = g.integers(0, 8, (n, F_)) / 8.0
    y, E = M.forward_bf16_interval(params, X)
    assert np.allclose(y, M.forward_bf16(params, X), rtol=0, atol=1e-12)
    worst = 0.0
    for _ in range(4):
        got = _device_like_forward(g, params, X)
        assert (np.abs(got - y) <= E).all()
        worst = max(worst, float((np.abs(got - y) / E).max()))
    # the bound is not vacuous: some forward comes within a factor 50 of it
    assert worst > 0.02
