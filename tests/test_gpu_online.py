"""Online retraining with tree fallback (cgs_online_run): the model choice
follows the RMSE rule, the run equals the same library calls made one by
one, and when every window falls back to the tree the search is the plain
tree search, pick for pick equal to the oracle.  On the large network shape
(16 -> 512 -> 512 -> 32) the surrogate's first scored step is checked
against the oracle's bf16 forward and score chain with propagated bounds."""
import numpy as np
import pytest

import synth
from oracle import bounds as B
from oracle import mlp as M
from oracle import search as SR
from oracle import space as SP
from tests.helpers import cgs

pytestmark = pytest.mark.gpu


def _setup(m, n_steps, spec=None, forest=None, H=64, key=(6,)):
    spec = spec or synth.space_c1()
    forest = forest or synth.forest_c1(spec)
    C = forest.leaves.shape[2]
    sp = m.Space.from_spec(spec)
    tree = m.ForestModel.from_spec(sp, forest)
    init = synth.mlp_init(key + (1,), len(spec.radix), H, C)
    mlp = m.MLPModel(sp, [init.w[0], init.b[0], init.w[1], init.b[1], init.w[2], init.b[2]])
    g = synth.rng(*key, 2)
    deltas = synth.deltas(g, n_steps, C)
    U = synth.uniforms_u64(g, n_steps + 1)
    noise = synth.normal_noise(g, (n_steps + 1, C), 0.02)
    valid = sp.copy_valid()
    pos = synth.uniform_indices(synth.rng(*key, 3), 512, sp.n_valid)
    seed_tgt = tree.gather_predictions(pos) + synth.normal_noise(synth.rng(*key, 4), (512, C), 0.02)
    val = synth.uniform_indices(synth.rng(*key, 5), 2048, sp.n_valid)
    return spec, forest, sp, tree, mlp, init, deltas, U, noise, valid[pos], seed_tgt, val


def _batch_u64(n_steps, opts, key=(6, 6)):
    W = 1 + n_steps // opts.retrain_every
    return synth.uniforms_u64(synth.rng(*key), max(1, (W - 1) * opts.train_steps * opts.batch))


def test_rmse_entry_point_is_the_definition():
    m = cgs()
    spec, forest, sp, tree, mlp, *_, val = _setup(m, 1)
    a = tree.copy_predictions().astype(np.float64)
    b = mlp.copy_predictions().astype(np.float64)
    ref = np.sqrt(np.mean((a[val] - b[val]) ** 2))
    assert abs(tree.rmse(mlp, val) - ref) <= 1e-12 * max(1.0, ref)


def test_fallback_everywhere_equals_the_oracle_tree_search():
    m = cgs()
    n = 60
    spec, forest, sp, tree, mlp, _, deltas, U, noise, cfg, tgt, val = _setup(m, n)
    opts = m.cgs_default_online_opts(threshold=1e-9, train_steps=50, batch=64)
    log = m.Session(sp).online_run(tree, mlp, deltas, U, noise, cfg, tgt, val,
                                   _batch_u64(n, opts), opts)
    assert [w["model"] for w in log["windows"]] == ["tree"] * 4
    assert len(log["retrain_ms"]) == 3 and (log["retrain_ms"] > 0).all()
    prep = SR.prepare(spec, forest)
    explored = np.zeros(len(prep.valid), dtype=bool)
    prof = None
    picks = []
    for i in range(n + 1):
        d = deltas[i - 1] if i else np.zeros(12, np.float32)
        r = SR.step(prep, explored, prof, d, [int(U[i])], with_fp64=False)
        picks.append(r.picks[0])
        prof = r.picks[0]
    assert log["picks"] == picks


def test_model_choice_follows_the_rmse_rule():
    m = cgs()
    n = 60
    spec, forest, sp, tree, mlp, init, deltas, U, noise, cfg, tgt, val = _setup(m, n)
    opts = m.cgs_default_online_opts(threshold=10.0, train_steps=50, batch=64)
    bu = _batch_u64(n, opts)
    log = m.Session(sp).online_run(tree, mlp, deltas, U, noise, cfg, tgt, val, bu, opts)
    assert all(w["model"] == "mlp" for w in log["windows"])
    rmses = [w["rmse"] for w in log["windows"]]
    # training on more of the forest's own counters brings the surrogate closer
    assert rmses[-1] < rmses[0]
    assert len(set(log["picks"])) == len(log["picks"]) == n + 1
    thr = float(np.median(rmses))
    mlp2 = m.MLPModel(sp, [init.w[0], init.b[0], init.w[1], init.b[1], init.w[2], init.b[2]])
    opts2 = m.cgs_default_online_opts(threshold=thr, train_steps=50, batch=64)
    log2 = m.Session(sp).online_run(tree, mlp2, deltas, U, noise, cfg, tgt, val, bu, opts2)
    assert [w["rmse"] for w in log2["windows"]][0] == rmses[0]
    for w in log2["windows"]:
        assert w["model"] == ("mlp" if w["rmse"] <= thr else "tree")


def test_run_equals_the_calls_one_by_one():
    """The policy spelled out with the single calls (cgs_model_rmse,
    cgs_mlp_train on the seed pairs plus the collected ones with rows
    floor(u * n_pairs / 2^64), cgs_search_step, cgs_sample_next) gives the
    same picks, windows and final parameters."""
    m = cgs()
    n = 45
    spec, forest, sp, tree, mlp, init, deltas, U, noise, cfg, tgt, val = _setup(m, n)
    opts = m.cgs_default_online_opts(retrain_every=15, threshold=0.2, train_steps=30, batch=32)
    bu = _batch_u64(n, opts)
    log = m.Session(sp).online_run(tree, mlp, deltas, U, noise, cfg, tgt, val, bu, opts)
    mlp2 = m.MLPModel(sp, [init.w[0], init.b[0], init.w[1], init.b[1], init.w[2], init.b[2]])
    sess = m.Session(sp)
    pairs_c, pairs_t = list(cfg), [row for row in tgt]
    r = tree.rmse(mlp2, val)
    use = r <= opts.threshold
    windows = [use]
    rmses = [r]
    sess.search_step(tree, m.NO_PROFILE)
    raw, l = sess.sample_next(int(U[0]))
    picks = [l]
    pairs_c.append(raw)
    pairs_t.append(tree.gather_predictions([l])[0] + noise[0])
    per = opts.train_steps * opts.batch
    for i in range(1, n + 1):
        if i % opts.retrain_every == 0:
            w = i // opts.retrain_every
            u = bu[(w - 1) * per:w * per].astype(object)
            rows = np.array([(int(x) * len(pairs_c)) >> 64 for x in u], np.int32)
            mlp2.train(np.array(pairs_c, np.uint32), np.array(pairs_t, np.float32),
                       rows.reshape(opts.train_steps, opts.batch), lr=opts.lr)
            r = tree.rmse(mlp2, val)
            use = r <= opts.threshold
            windows.append(use)
            rmses.append(r)
        sess.search_step(mlp2 if use else tree, raw, delta=deltas[i - 1])
        raw, l = sess.sample_next(int(U[i]))
        picks.append(l)
        pairs_c.append(raw)
        pairs_t.append(tree.gather_predictions([l])[0] + noise[i])
    assert log["picks"] == picks
    assert [w["model"] == "mlp" for w in log["windows"]] == windows
    # a retrained network's RMSE comes from its validation configurations
    # alone inside the run: the same sums as cgs_model_rmse on a full
    # evaluation
    assert [w["rmse"] for w in log["windows"]] == rmses
    assert (mlp.copy_params() == mlp2.copy_params()).all()


def test_predictions_are_current_after_the_run():
    """Every window falls back to the tree, so no retrained network is
    evaluated beyond the validation configurations during the run; the run
    evaluates the final one before returning: its predictions equal a fresh
    evaluation, and the last window's RMSE is cgs_model_rmse on them."""
    m = cgs()
    n = 40
    spec, forest, sp, tree, mlp, _, deltas, U, noise, cfg, tgt, val = _setup(m, n)
    opts = m.cgs_default_online_opts(retrain_every=20, threshold=1e-9, train_steps=20, batch=32)
    log = m.Session(sp).online_run(tree, mlp, deltas, U, noise, cfg, tgt, val,
                                   _batch_u64(n, opts), opts)
    assert [w["model"] for w in log["windows"]] == ["tree"] * 3
    after = mlp.copy_predictions()
    mlp.refresh()
    assert (mlp.copy_predictions() == after).all()
    assert log["windows"][-1]["rmse"] == tree.rmse(mlp, val)


def test_surrogate_step_on_the_large_network_shape():
    """16 -> 512 -> 512 -> 32 on a 16-parameter space (221,184 raw, 65,536
    valid), surrogate taken from the first window: the start is the
    oracle's uniform draw exactly; the first scored step's scores, weights
    and pick lie inside the oracle's intervals propagated from the bf16
    forward's error bound (oracle/bounds.py)."""
    m = cgs()
    spec = synth.space_c5_slice()
    forest = synth.random_forest(synth.rng(7, 2), spec.radix, 4, 8, 32)
    spec, forest, sp, tree, mlp, init, deltas, U, noise, cfg, tgt, val = _setup(
        m, 1, spec, forest, H=512, key=(7, 3))
    opts = m.cgs_default_online_opts(threshold=1e9)
    sess = m.Session(sp)
    log = sess.online_run(tree, mlp, deltas, U, noise, cfg, tgt, val, None, opts)
    assert [w["model"] for w in log["windows"]] == ["mlp"]
    valid = SP.enumerate_valid(spec.radix, spec.values, spec.constraints)
    assert (valid == sp.copy_valid()).all()
    nv = len(valid)
    # step 0: Delta = 0, every weight 1: the oracle's uniform draw
    q0 = np.full(nv, 1 << 23, np.uint64)
    first, last, certain = B.feasible_picks(q0, q0, int(U[0]))
    assert certain and log["picks"][0] == first
    prof = first
    # step 1 on the surrogate: prediction intervals from the bf16 forward
    params = [init.w[0], init.b[0], init.w[1], init.b[1], init.w[2], init.b[2]]
    X = M.features(SP.digits_of(valid.astype(np.int64), spec.radix))
    y, E = M.forward_bf16_interval(params, X)
    lo, hi = np.maximum(y - E, 0.0), np.maximum(y + E, 0.0)
    P = mlp.copy_predictions().astype(np.float64)
    assert ((P >= lo) & (P <= hi)).all()
    explored = np.zeros(nv, bool)
    explored[prof] = True
    s_lo, s_hi = B.score_interval(lo[prof], hi[prof], lo, hi, deltas[0])
    s = sess.copy_scores().astype(np.float64)
    un = ~explored
    un[log["picks"][1]] = True           # drawn after scoring
    assert ((s[un] >= s_lo[un]) & (s[un] <= s_hi[un])).all()
    w_lo, w_hi = B.weight_interval(s_lo, s_hi, explored)
    q_lo, q_hi = B.q_interval(w_lo, w_hi)
    first, last, certain = B.feasible_picks(q_lo, q_hi, int(U[1]))
    l1 = log["picks"][1]
    assert first <= l1 <= last and q_hi[l1] > 0
    if certain:
        assert l1 == first
    print(f"surrogate step: score interval width median {np.median(s_hi - s_lo):.3g}, "
          f"feasible picks {last - first + 1} of {nv}, certain={certain}", flush=True)
