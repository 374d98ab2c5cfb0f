"""GPU perceptron surrogate vs the oracle: forward (bf16 weights and
activations, fp32 accumulation) against the oracle's forward with the same
roundings; gradients against float64 backprop; Adam's first step in closed
form; loss curves against the oracle's training on the same batches; and
what the trained network gains over random search."""
import numpy as np
import pytest

import synth
from oracle import forest as F
from oracle import mlp as M
from oracle import score as SC
from oracle import space as SP
from tests.helpers import cgs

pytestmark = pytest.mark.gpu


def _space():
    spec = synth.space_c1()
    valid = SP.enumerate_valid(spec.radix, spec.values, spec.constraints)
    return spec, valid


def _params(F_, H, C, key):
    init = synth.mlp_init(key, F_, H, C)
    g = synth.rng(*key, 99)
    b = [synth.normal_noise(g, (H,), 0.1), synth.normal_noise(g, (H,), 0.1),
         synth.normal_noise(g, (C,), 0.1)]
    return [init.w[0], b[0], init.w[1], b[1], init.w[2], b[2]]


def _bound(params, X):
    """Two bf16 ulps (2^-7 relative) of every hidden value, propagated through
    the absolute weights, plus fp32 accumulation noise."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(p, np.float64) for p in params]
    h1 = np.abs(M.gelu(X @ W1.T + b1))
    h2 = np.abs(M.gelu(M.gelu(X @ W1.T + b1) @ W2.T + b2))
    prop = h2 @ np.abs(W3).T + (h1 @ np.abs(W2).T) @ np.abs(W3).T
    return 2.0 ** -7 * prop + 1e-4


@pytest.mark.parametrize("H,C", [(64, 12), (128, 40), (256, 12), (512, 32)])
def test_forward_matches_bf16_oracle(H, C):
    m = cgs()
    spec, valid = _space()
    sp = m.Space.from_spec(spec)
    params = _params(6, H, C, (30, H, C))
    model = m.MLPModel(sp, params)
    g = np.random.default_rng(H)
    cfg = valid[g.integers(0, len(valid), 1000)]
    X = M.features(SP.digits_of(cfg.astype(np.int64), spec.radix))
    y = model.forward(cfg).astype(np.float64)
    ref = M.forward_bf16([np.asarray(p, np.float64) for p in params], X)
    assert (np.abs(y - ref) <= _bound(params, X)).all(), np.abs(y - ref).max()
    cos = (y * ref).sum() / np.sqrt((y * y).sum() * (ref * ref).sum())
    assert cos > 0.99999


@pytest.mark.parametrize("H,C", [(64, 12), (128, 40), (256, 24), (256, 40), (512, 32),
                                 (512, 40)])
def test_full_space_predictions_are_clamped_forward(H, C):
    """Every valid configuration of the 30,720-configuration space (a ragged
    last tile), through the inference kernels: weights resident in LDS
    (H <= 256 when they fit) or the second layer's streamed through it."""
    m = cgs()
    spec, valid = _space()
    sp = m.Space.from_spec(spec)
    params = _params(6, H, C, (31, H, C))
    model = m.MLPModel(sp, params)
    P = model.copy_predictions().astype(np.float64)
    X = M.features(SP.digits_of(valid.astype(np.int64), spec.radix))
    ref = np.maximum(M.forward_bf16([np.asarray(p, np.float64) for p in params], X), 0.0)
    assert P.min() >= 0.0
    assert (np.abs(P - ref) <= _bound(params, X)).all()


@pytest.mark.parametrize("H,C", [(64, 8), (256, 40), (512, 8), (512, 40)])
def test_twenty_parameter_inference(H, C):
    """Full-space inference with 20 inputs (two first-layer K steps), checked
    on 4,000 sampled configurations and the last 70; at 512 / 40 the first
    layer's weights are read from global memory instead of LDS."""
    m = cgs()
    radix = [2] * 20
    values = [[1, 2]] * 20
    sp = m.Space(radix, values, [("PROD_LE", 0, 1, 0, 2)])
    params = _params(20, H, C, (33, H, C))
    model = m.MLPModel(sp, params)
    P = model.copy_predictions().astype(np.float64)
    valid = sp.copy_valid()
    g = np.random.default_rng(H + C)
    pick = np.concatenate([g.choice(len(valid), 4000, replace=False),
                           np.arange(len(valid) - 70, len(valid))])
    X = M.features(SP.digits_of(valid[pick].astype(np.int64), radix))
    ref = np.maximum(M.forward_bf16([np.asarray(p, np.float64) for p in params], X), 0.0)
    assert (np.abs(P[pick] - ref) <= _bound(params, X)).all()


def test_twenty_parameter_inputs_use_two_k_steps():
    """F = 20 inputs pad to K = 32 (two 16-deep steps of the first layer)."""
    m = cgs()
    radix = [2] * 20
    values = [[1, 2]] * 20
    sp = m.Space(radix, values, [("PROD_LE", 0, 1, 0, 2)])
    params = _params(20, 64, 8, (32,))
    model = m.MLPModel(sp, params)
    g = np.random.default_rng(3)
    cfg = g.integers(0, 1 << 20, 700).astype(np.uint32)
    X = M.features(SP.digits_of(cfg.astype(np.int64), radix))
    y = model.forward(cfg).astype(np.float64)
    ref = M.forward_bf16([np.asarray(p, np.float64) for p in params], X)
    assert (np.abs(y - ref) <= _bound(params, X)).all()


def _pairs(spec, valid, n, seed):
    forest = synth.forest_c1(spec)
    g = synth.rng(1, 7, seed)
    pos = synth.uniform_indices(g, n, len(valid))
    cfg = valid[pos]
    d = SP.digits_of(cfg.astype(np.int64), spec.radix)
    ids = F.leaf_ids(forest.feat, forest.thr, forest.depth, d)
    T = (F.predict_fp32(forest.leaves, ids) + synth.normal_noise(g, (n, 12), 0.02)).astype(np.float32)
    return cfg, T, M.features(d)


@pytest.mark.parametrize("H", [64, 256, 512])
def test_gradients_match_float64_backprop(H):
    m = cgs()
    spec, valid = _space()
    sp = m.Space.from_spec(spec)
    params = _params(6, H, 12, (33, H))
    model = m.MLPModel(sp, params)
    cfg, T, X = _pairs(spec, valid, 256, 1)
    g_gpu, loss = model.gradients(cfg, T)
    pr = [np.asarray(p, np.float64) for p in params]
    pr = [M.bf16(p).astype(np.float64) if i % 2 == 0 else p for i, p in enumerate(pr)]
    loss_ref, g_ref = M.loss_and_grads(pr, X, T.astype(np.float64))
    assert abs(loss - loss_ref) <= 1e-2 * loss_ref
    for got, ref in zip(model.unflatten(g_gpu), g_ref):
        got = got.astype(np.float64)
        cos = (got * ref).sum() / np.sqrt((got * got).sum() * (ref * ref).sum())
        assert cos > 0.999, cos
        assert np.abs(got - ref).max() <= 2e-2 * np.abs(ref).max()


def test_gradients_with_two_output_tiles():
    """C = 40 outputs: dY spans two 32-column tiles, the transposed bf16 copy
    of W3 has rows of 64, and the 40-deep product dY W3 ends on a full
    8-value fragment."""
    m = cgs()
    spec, valid = _space()
    sp = m.Space.from_spec(spec)
    params = _params(6, 128, 40, (36, 128))
    model = m.MLPModel(sp, params)
    cfg, _, X = _pairs(spec, valid, 256, 2)
    T = synth.normal_noise(synth.rng(36, 5), (256, 40), 1.0).astype(np.float32)
    g_gpu, loss = model.gradients(cfg, T)
    pr = [np.asarray(p, np.float64) for p in params]
    pr = [M.bf16(p).astype(np.float64) if i % 2 == 0 else p for i, p in enumerate(pr)]
    loss_ref, g_ref = M.loss_and_grads(pr, X, T.astype(np.float64))
    assert abs(loss - loss_ref) <= 1e-2 * loss_ref
    for got, ref in zip(model.unflatten(g_gpu), g_ref):
        got = got.astype(np.float64)
        cos = (got * ref).sum() / np.sqrt((got * got).sum() * (ref * ref).sum())
        assert cos > 0.999, cos
        assert np.abs(got - ref).max() <= 2e-2 * np.abs(ref).max()


@pytest.mark.parametrize("n", [1, 45, 200])
def test_gradients_of_a_ragged_batch(n):
    """Batches that are not a multiple of 32 rows: the last output tile is
    partly past the end (its rows read no targets and add no squared error),
    and a single row is a batch of one tile."""
    m = cgs()
    spec, valid = _space()
    sp = m.Space.from_spec(spec)
    params = _params(6, 64, 12, (38, n))
    model = m.MLPModel(sp, params)
    cfg, T, X = _pairs(spec, valid, n, 5)
    g_gpu, loss = model.gradients(cfg, T)
    pr = [np.asarray(p, np.float64) for p in params]
    pr = [M.bf16(p).astype(np.float64) if i % 2 == 0 else p for i, p in enumerate(pr)]
    loss_ref, g_ref = M.loss_and_grads(pr, X, T.astype(np.float64))
    assert abs(loss - loss_ref) <= 1e-2 * loss_ref
    for got, ref in zip(model.unflatten(g_gpu), g_ref):
        got = got.astype(np.float64)
        cos = (got * ref).sum() / np.sqrt((got * got).sum() * (ref * ref).sum())
        assert cos > 0.999, cos
        assert np.abs(got - ref).max() <= 2e-2 * np.abs(ref).max()


def test_gradients_after_adam_steps_use_the_updated_weights():
    """Adam rewrites the bf16 weight copies that the backward products read:
    after five steps (lr 1e-2, so W2 moves far beyond its bf16 rounding) the
    gradients must match the oracle's at the trained parameters."""
    m = cgs()
    spec, valid = _space()
    sp = m.Space.from_spec(spec)
    params = _params(6, 128, 40, (37, 128))
    model = m.MLPModel(sp, params)
    cfg, _, X = _pairs(spec, valid, 256, 4)
    T = synth.normal_noise(synth.rng(37, 5), (256, 40), 1.0).astype(np.float32)
    batches = np.tile(np.arange(256, dtype=np.int32), (5, 1))
    model.train(cfg, T, batches, lr=1e-2)
    trained = model.unflatten(model.copy_params())
    moved = np.abs(trained[2] - np.asarray(params[2])).max() / np.abs(params[2]).max()
    assert moved > 0.1, moved  # the oracle's training moves W2 by 0.23 of its max here
    g_gpu, loss = model.gradients(cfg, T)
    pr = [np.asarray(p, np.float64) for p in trained]
    pr = [M.bf16(p.astype(np.float32)).astype(np.float64) if i % 2 == 0 else p
          for i, p in enumerate(pr)]
    loss_ref, g_ref = M.loss_and_grads(pr, X, T.astype(np.float64))
    assert abs(loss - loss_ref) <= 1e-2 * loss_ref
    for got, ref in zip(model.unflatten(g_gpu), g_ref):
        got = got.astype(np.float64)
        cos = (got * ref).sum() / np.sqrt((got * got).sum() * (ref * ref).sum())
        assert cos > 0.999, cos
        assert np.abs(got - ref).max() <= 2e-2 * np.abs(ref).max()


def test_first_adam_step_closed_form():
    m = cgs()
    spec, valid = _space()
    sp = m.Space.from_spec(spec)
    params = _params(6, 128, 12, (34,))
    model = m.MLPModel(sp, params)
    cfg, T, X = _pairs(spec, valid, 256, 2)
    theta0 = model.copy_params().astype(np.float64)
    lr = 1e-3
    model.train(cfg, T, np.arange(256, dtype=np.int32)[None, :], lr=lr)
    step = model.copy_params().astype(np.float64) - theta0
    pr = [M.bf16(np.asarray(p, np.float32)).astype(np.float64) if i % 2 == 0 else
          np.asarray(p, np.float64) for i, p in enumerate(params)]
    _, g_ref = M.loss_and_grads(pr, X, T.astype(np.float64))
    g = np.concatenate([x.ravel() for x in g_ref])
    # t = 1: the step is -lr g / (|g| + eps) = -lr sign(g) wherever |g| >> eps
    strong = np.abs(g) > 1e-2 * np.abs(g).max()
    assert np.allclose(step[strong], -lr * np.sign(g[strong]), rtol=2e-3, atol=0)
    assert (np.sign(step) == -np.sign(g))[np.abs(g) > 1e-6].mean() > 0.98


def test_loss_curve_tracks_the_oracle():
    m = cgs()
    spec, valid = _space()
    sp = m.Space.from_spec(spec)
    params = _params(6, 64, 12, (35,))
    model = m.MLPModel(sp, params)
    cfg, T, X = _pairs(spec, valid, 2048, 3)
    batches = synth.minibatches(synth.rng(1, 8), 150, 128, 2048)
    losses = model.train(cfg, T, batches, lr=3e-3)
    _, ref = M.train([np.asarray(p, np.float64) for p in params], X, T.astype(np.float64),
                     batches, lr=3e-3)
    ref = np.asarray(ref)
    assert np.all(np.abs(losses[:10] - ref[:10]) <= 0.05 * ref[:10])
    assert np.mean(losses[-20:]) <= 1.10 * np.mean(ref[-20:])
    assert np.mean(losses[-20:]) < 0.5 * np.mean(losses[:5])


def test_trained_network_beats_random_search():
    """The method without a model is random search (every weight 1).  A
    perceptron trained on 4096 noisy samples of the forest steers the weighted
    draw toward configurations the forest itself scores highly."""
    m = cgs()
    spec, valid = _space()
    sp = m.Space.from_spec(spec)
    forest = synth.forest_c1(spec)
    tree = m.ForestModel.from_spec(sp, forest)
    params = _params(6, 128, 12, (36,))
    model = m.MLPModel(sp, params)
    cfg, T, X = _pairs(spec, valid, 4096, 4)
    model.train(cfg, T, synth.minibatches(synth.rng(1, 9), 600, 256, 4096), lr=2e-3)
    P_tree = tree.copy_predictions()
    P_mlp = model.copy_predictions()
    rmse = float(np.sqrt(np.mean((P_mlp.astype(np.float64) - P_tree) ** 2)))
    # better than predicting every counter's mean over the space
    baseline = float(np.sqrt(np.mean((P_tree - P_tree.mean(axis=0)) ** 2)))
    assert rmse < 0.9 * baseline, (rmse, baseline)
    g = synth.rng(1, 10)
    gains = []
    for trial in range(5):
        d = synth.deltas(g, 1, 12)[0]
        prof = int(synth.uniform_indices(g, 1, len(valid))[0])
        s_tree = SC.score_fp64(P_tree[prof], P_tree, d)
        sess = m.Session(sp)
        sess.search_step(model, int(valid[prof]), delta=d)
        U = synth.uniforms_u64(g, 200)
        picks = []
        for u in U:
            r = sess.sample_next(int(u))
            picks.append(r[1])
        uniform_mean = s_tree[np.arange(len(valid)) != prof].mean()
        gains.append(s_tree[picks].mean() - uniform_mean)
    assert np.mean(gains) > 0.0 and sum(x > 0 for x in gains) >= 4, gains
