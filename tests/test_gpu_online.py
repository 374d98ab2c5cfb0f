"""Online retraining with tree fallback (the driver in bench.py): the model
choice follows the RMSE rule, and when every window falls back to the tree
the search is the plain tree search, pick for pick equal to the oracle."""
import numpy as np
import pytest

import bench
import synth
from oracle import search as SR
from tests.helpers import cgs

pytestmark = pytest.mark.gpu


def _setup(m, n_steps):
    spec = synth.space_c1()
    sp = m.Space.from_spec(spec)
    forest = synth.forest_c1(spec)
    tree = m.ForestModel.from_spec(sp, forest)
    init = synth.mlp_init((6, 1), 6, 64, 12)
    mlp = m.MLPModel(sp, [init.w[0], init.b[0], init.w[1], init.b[1], init.w[2], init.b[2]])
    g = synth.rng(6, 2)
    deltas = synth.deltas(g, n_steps, 12)
    U = synth.uniforms_u64(g, n_steps + 1)
    noise = synth.normal_noise(g, (n_steps + 1, 12), 0.02)
    valid = sp.copy_valid()
    pos = synth.uniform_indices(synth.rng(6, 3), 512, sp.n_valid)
    seed_tgt = tree.copy_predictions()[pos] + synth.normal_noise(synth.rng(6, 4), (512, 12), 0.02)
    val = synth.uniform_indices(synth.rng(6, 5), 2048, sp.n_valid)
    return spec, forest, sp, tree, mlp, deltas, U, noise, valid[pos], seed_tgt, val


def test_rmse_entry_point_is_the_definition():
    m = cgs()
    spec, forest, sp, tree, mlp, *_ , val = _setup(m, 1)
    a = tree.copy_predictions().astype(np.float64)
    b = mlp.copy_predictions().astype(np.float64)
    ref = np.sqrt(np.mean((a[val] - b[val]) ** 2))
    assert abs(tree.rmse(mlp, val) - ref) <= 1e-12 * max(1.0, ref)


def test_fallback_everywhere_equals_the_oracle_tree_search():
    m = cgs()
    n = 60
    spec, forest, sp, tree, mlp, deltas, U, noise, cfg, tgt, val = _setup(m, n)
    log = bench.online_search(m, sp, tree, mlp, n, deltas, U, noise, cfg, tgt, val,
                              retrain_every=20, threshold=1e-9, train_steps=50, batch=64)
    assert [w["model"] for w in log["windows"]] == ["tree"] * 4
    assert len(log["retrain_ms"]) == 3
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
    spec, forest, sp, tree, mlp, deltas, U, noise, cfg, tgt, val = _setup(m, n)
    log = bench.online_search(m, sp, tree, mlp, n, deltas, U, noise, cfg, tgt, val,
                              retrain_every=20, threshold=10.0, train_steps=50, batch=64)
    assert all(w["model"] == "mlp" for w in log["windows"])
    rmses = [w["rmse"] for w in log["windows"]]
    # training on more of the forest's own counters brings the surrogate closer
    assert rmses[-1] < rmses[0]
    assert len(set(log["picks"])) == len(log["picks"]) == n + 1
    thr = float(np.median(rmses))
    mlp2 = m.MLPModel(sp, mlp.unflatten(mlp.copy_params()))
    log2 = bench.online_search(m, sp, tree, mlp2, n, deltas, U, noise, cfg, tgt, val,
                               retrain_every=20, threshold=thr, train_steps=50, batch=64)
    for w in log2["windows"]:
        assert w["model"] == ("mlp" if w["rmse"] <= thr else "tree")
