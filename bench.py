"""Benchmark of the counter-guided search sweep on one MI355X.

    python bench.py [--gpus 1] [--steps 100] [--warmup 5] [--no-cpu-baseline]

Workload: the 12-parameter tuning space (value-set sizes 8,4,2,8,4,2,8,4,2,4,
4,4: 16,777,216 raw configurations, 6 constraints keep 4,813,824), a forest of
16 depth-12 trees predicting 24 counters per configuration, and 100
sequential search steps.  Each step profiles the previous pick: seeded
synthetic Table 1 counters go through the expert system to the counter
changes, every unexplored configuration is scored and weighted, and one
configuration is drawn (Alg. 1 with one draw per scoring pass).

Timed region (after warm-up): one full model evaluation (forest -> predicted
counters of every valid configuration), the uniform starting draw, and K
scored steps, each synchronised on its pick.  value = configurations scored
in the K steps / wall time of the region.  The picks of the timed run are
compared with the oracle's stored trajectory of the same inputs.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CORES_PROFILED = 1920.0
# HIP event markers around a step's kernels cost a few microseconds each, so
# the timed run times every TIMING_PERIOD-th step
TIMING_PERIOD = 5


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload_inputs(n_steps: int):
    import synth
    g = synth.rng(2, 3)
    U = synth.uniforms_u64(g, n_steps + 1)
    pcs = synth.profiler_counters(synth.rng(2, 4), n_steps)
    thr = synth.threads_launched(synth.rng(2, 5), n_steps)
    return U, pcs, thr


def expert_settings(cgs, thr):
    """The expert system's settings of each step (threads launched per step)."""
    return [cgs.cgs_expert_params(inst_reaction=0.7, volta=0, reserved=0, cores=CORES_PROFILED,
                                  threads=float(x)) for x in thr]


def run_search(cgs, sp, model, U, pcs, eps, n_steps, timing):
    """Uniform start + n_steps scored steps in one library call
    (cgs_search_run: per step the expert system on the measured counters,
    the scored step and its draw); returns (picks, session).  timing = k > 0
    times the kernels of steps 0, k, 2k, ... with HIP events."""
    params = cgs.cgs_default_params()
    params.timing = int(timing)
    sess = cgs.Session(sp, params)
    _, val, t_us = sess.search_run(model, pcs[:n_steps], eps[:n_steps], U[:n_steps + 1])
    sess.step_wall_s = list(t_us * 1e-6)
    return [int(x) for x in val], sess


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "score_pass_c2_traffic.md")
VALU_PROFILE = os.path.join(ROOT, "profiles", "mlp_infer_valu.md")
SWEEP_SOURCES = ("sweep.hip", "device_common.h", "internal.h")
MLP_SOURCES = ("mlp.hip", "gelu.h", "device_common.h", "internal.h")
# VALU issue peak with packed FP32 off: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12


def counter_profile(path, sources):
    """The JSON block of a committed counter profile, or None when it is
    missing or was taken on other kernel sources (SHA-256 of the sources,
    concatenated in order)."""
    try:
        text = open(path).read()
        doc = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    h = hashlib.sha256()
    for name in sources:
        with open(os.path.join(ROOT, "paper_2102_05297_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return doc if h.hexdigest() == doc.get("source_sha256") else None


def pmc_traffic(active_counts):
    """HBM bytes per score-pass launch, averaged over launches with the given
    active-counter counts, from the committed FETCH_SIZE / WRITE_SIZE profile
    (already scaled by the copy-kernel calibration); None when the profile is
    missing, lacks a count, or was taken on other kernel sources."""
    doc = counter_profile(TRAFFIC_PROFILE, SWEEP_SOURCES)
    if doc is None:
        return None
    per = {int(k): float(v) for k, v in doc["bytes_per_launch_by_active"].items()}
    if not active_counts or any(a not in per for a in active_counts):
        return None
    return sum(per[a] for a in active_counts) / len(active_counts)


def valu_roofline(shape, n_configs, ms):
    """ALU roofline of a perceptron inference sweep: VALU lane instructions
    per second (counter-measured instructions per configuration x configs /
    the live duration) against the issue peak; None without a matching
    profile."""
    doc = counter_profile(VALU_PROFILE, MLP_SOURCES)
    per = None if doc is None else doc["valu_wave_instr_per_config"].get(shape)
    if per is None or ms <= 0:
        return None
    achieved = per * 64 * n_configs / (ms / 1e3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_T,
            "unit": "T VALU lane-instructions/s", "frac": achieved / VALU_PEAK_T}


def copy_probe(n_bytes: int = 1 << 30, reps: int = 5) -> dict:
    """Achievable HBM bandwidth of a plain device-to-device copy of n_bytes
    (the HIP runtime's copy kernel), timed with HIP events; reads + writes."""
    import ctypes as C
    hip = C.CDLL("libamdhip64.so.7")
    src, dst = C.c_void_p(), C.c_void_p()
    e0, e1 = C.c_void_p(), C.c_void_p()
    ok = (hip.hipMalloc(C.byref(src), C.c_size_t(n_bytes)) == 0 and
          hip.hipMalloc(C.byref(dst), C.c_size_t(n_bytes)) == 0 and
          hip.hipEventCreate(C.byref(e0)) == 0 and hip.hipEventCreate(C.byref(e1)) == 0)
    if not ok:
        return {"error": "allocation failed"}
    hip.hipMemset(src, 1, C.c_size_t(n_bytes))
    hip.hipMemcpy(dst, src, C.c_size_t(n_bytes), 3)     # warm-up, hipMemcpyDeviceToDevice
    hip.hipDeviceSynchronize()
    hip.hipEventRecord(e0, None)
    for _ in range(reps):
        hip.hipMemcpyAsync(dst, src, C.c_size_t(n_bytes), 3, None)
    hip.hipEventRecord(e1, None)
    hip.hipEventSynchronize(e1)
    ms = C.c_float()
    hip.hipEventElapsedTime(C.byref(ms), e0, e1)
    hip.hipFree(src)
    hip.hipFree(dst)
    hip.hipEventDestroy(e0)
    hip.hipEventDestroy(e1)
    gbs = 2.0 * n_bytes * reps / (ms.value / 1e3) / 1e9
    return {"copy_gbs": gbs, "bytes": n_bytes, "reps": reps, "avg_ms": ms.value / reps}


BF16_PEAK_TFLOPS = 2500.0


def mean_predictor_rmse(P_tree) -> float:
    """RMSE against the tree of the constant model that predicts each
    counter's mean over the same sample: what a surrogate that learned
    nothing of the configurations would score."""
    P = np.asarray(P_tree, dtype=np.float64)
    return float(np.sqrt(np.mean((P - P.mean(axis=0)) ** 2)))


def mlp_path(cgs, sp, tree, n_pairs=8192, steps=2000, batch=256, top_pairs=100):
    """Learned surrogate: train on forest samples + N(0, 0.02) noise, predict
    every valid configuration, compare with the tree and time both uses."""
    import synth
    U, pcs, thr = workload_inputs(max(top_pairs, 22))
    F_, H, Cn = len(sp.radix), 256, tree.n_counters
    valid = sp.copy_valid()
    g = synth.rng(3, 1)
    pos = synth.uniform_indices(g, n_pairs, sp.n_valid)
    # targets: tree predictions of the sampled configurations plus noise
    P_tree_all = tree.copy_predictions()
    tgt = (P_tree_all[pos] + synth.normal_noise(g, (n_pairs, Cn), 0.02)).astype(np.float32)
    cfg = valid[pos]
    init = synth.mlp_init((3, 2), F_, H, Cn)
    model = cgs.MLPModel(sp, [init.w[0], init.b[0], init.w[1], init.b[1], init.w[2], init.b[2]])
    batches = synth.minibatches(synth.rng(3, 3), steps, batch, n_pairs)
    # a few steps on a second network of the same shape load the training
    # kernels before the timed run
    spare = cgs.MLPModel(sp, [init.w[0], init.b[0], init.w[1], init.b[1], init.w[2], init.b[2]])
    spare.train(cfg, tgt, batches[:4], lr=1e-3)
    spare.close()
    sp.synchronize()
    t0 = time.perf_counter()
    losses = model.train(cfg, tgt, batches, lr=1e-3)
    t_train = time.perf_counter() - t0
    log(f"mlp: trained {steps} steps in {t_train * 1e3:.1f} ms, loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    # inference over every valid configuration (timed over a few refreshes)
    reps = 5
    ms = []
    for _ in range(reps):
        model.refresh()
        ms.append(model.eval_ms())
    inf_ms = float(np.median(ms))
    flop = 2.0 * (F_ * H + H * H + H * Cn) * sp.n_valid
    tflops = flop / (inf_ms / 1e3) / 1e12
    P_mlp = model.copy_predictions()
    sample = synth.uniform_indices(synth.rng(3, 4), 65536, sp.n_valid)
    rmse = float(np.sqrt(np.mean((P_mlp[sample].astype(np.float64) - P_tree_all[sample]) ** 2)))
    rmse_mean = mean_predictor_rmse(P_tree_all[sample])
    # top-10 agreement on the first scoring pairs of the search trajectory
    agree = []
    sess_t = cgs.Session(sp)
    sess_m = cgs.Session(sp)
    sess_t.search_step(tree, cgs.NO_PROFILE)
    raw, _ = sess_t.sample_next(int(U[0]))
    for i in range(top_pairs):
        ep = cgs.cgs_expert_params(inst_reaction=0.7, volta=0, reserved=0, cores=CORES_PROFILED,
                                   threads=float(thr[i]))
        sess_t.search_step(tree, raw, measured=pcs[i], expert=ep)
        sess_m.search_step(model, raw, measured=pcs[i], expert=ep)
        st, sm = sess_t.copy_scores(), sess_m.copy_scores()
        ex = np.unpackbits(sess_t.copy_explored().view(np.uint8), bitorder="little")[: sp.n_valid]
        st[ex.astype(bool)] = -np.inf
        sm[ex.astype(bool)] = -np.inf
        top_t = set(np.argpartition(-st, 10)[:10].tolist())
        top_m = set(np.argpartition(-sm, 10)[:10].tolist())
        agree.append(len(top_t & top_m) / 10.0)
        raw, _ = sess_t.sample_next(int(U[i + 1]))
        sess_m.mark_explored(raw)
    # search throughput with the surrogate's cached predictions
    K = 20
    picks, sess = run_search(cgs, sp, model, U, pcs, expert_settings(cgs, thr), 2, timing=False)
    sp.synchronize()
    t0 = time.perf_counter()
    picks, sess = run_search(cgs, sp, model, U, pcs, expert_settings(cgs, thr), K, timing=False)
    sp.synchronize()
    t_steps = time.perf_counter() - t0
    step_ms = t_steps * 1e3 / K
    scored = sum(sp.n_valid - i for i in range(1, K + 1)) / K
    return {
        "shape": f"{F_}->{H}->{H}->{Cn}",
        "pairs": n_pairs, "train_steps": steps, "batch": batch,
        "train_ms": t_train * 1e3, "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
        "inference_ms": inf_ms, "inference_configs": sp.n_valid,
        "inference_tflops": tflops,
        "mfma_roofline": {"bound": "mfma", "achieved": tflops, "peak": BF16_PEAK_TFLOPS,
                          "unit": "TFLOP/s", "frac": tflops / BF16_PEAK_TFLOPS},
        "valu_roofline": valu_roofline(f"{F_}-{H}-{H}-{Cn}", sp.n_valid, inf_ms),
        "rmse_vs_tree": rmse, "rmse_sample": 65536,
        "rmse_mean_predictor": rmse_mean,
        "top10_agreement": float(np.mean(agree)), "top10_pairs": top_pairs,
        "scored_per_s_cached": scored / (step_ms / 1e3),
        "scored_per_s_eval_in_step": sp.n_valid / ((inf_ms + step_ms) / 1e3),
    }


def batch_path(cgs, n_sess=64, n_steps=10):
    """64 independent searches (log-uniform 10^4..10^7 raw configurations,
    8-14 parameters, forests of 8 depth-10 trees over 16 counters) stepped
    together; compared with stepping the same sessions one by one."""
    import synth
    specs = [synth.space_batch(s) for s in range(n_sess)]
    spaces = [cgs.Space.from_spec(sp) for sp in specs]
    models = [cgs.ForestModel.from_spec(spc, synth.forest_batch(s, sp))
              for s, (sp, spc) in enumerate(zip(specs, spaces))]
    g = synth.rng(4, 3, 0)
    D = synth.deltas(g, n_steps * n_sess, 16).reshape(n_steps, n_sess, 16)
    U = synth.uniforms_u64(g, (n_steps + 1) * n_sess).reshape(n_steps + 1, n_sess)
    n_valid = np.array([spc.n_valid for spc in spaces], dtype=np.int64)

    def run_batch(batch, sessions, timed):
        prof = [cgs.NO_PROFILE] * n_sess
        raw, _, _ = batch.step(prof, None, U[0])
        prof = [int(x) for x in raw]
        dev = []
        t0 = time.perf_counter()
        for k in range(n_steps):
            raw, _, st = batch.step(prof, D[k], U[k + 1])
            dev.append(batch.step_ms())
            prof = [int(x) for x in raw]
        return time.perf_counter() - t0, dev

    sessions = [cgs.Session(spc) for spc in spaces]
    batch = cgs.Batch(sessions, models)
    t_tune = time.perf_counter()
    sched = batch.autotune(None)
    t_tune = time.perf_counter() - t_tune
    run_batch(batch, sessions, False)                       # warm-up run
    # the default schedule (grids capped at 2048, variant 0, graph) for the gain
    sessions = [cgs.Session(spc) for spc in spaces]
    batch = cgs.Batch(sessions, models)
    _, dev_default = run_batch(batch, sessions, True)
    sessions = [cgs.Session(spc) for spc in spaces]
    batch = cgs.Batch(sessions, models, sched)
    wall, dev = run_batch(batch, sessions, True)
    # step k scores every valid configuration but the profile and k earlier picks
    scored = sum(int((n_valid - np.minimum(n_valid, k + 1)).sum()) for k in range(1, n_steps + 1))
    # the same steps through the single-session calls, one session after another
    singles = [cgs.Session(spc) for spc in spaces]
    prof = []
    for i in range(n_sess):
        singles[i].search_step(models[i], cgs.NO_PROFILE)
        prof.append(singles[i].sample_next(int(U[0][i]))[0])
    t0 = time.perf_counter()
    for k in range(n_steps):
        for i in range(n_sess):
            singles[i].search_step(models[i], prof[i], delta=D[k][i])
            prof[i] = singles[i].sample_next(int(U[k + 1][i]))[0]
    wall_single = time.perf_counter() - t0
    return {
        "sessions": n_sess, "steps": n_steps,
        "raw_total": int(sum(sp.n_raw for sp in specs)), "valid_total": int(n_valid.sum()),
        "schedule": {"score_grid": sched.score_grid, "weight_grid": sched.weight_grid,
                     "use_graph": sched.use_graph, "variant": sched.variant},
        "autotune_ms": t_tune * 1e3,
        "ms_per_batch_step": wall * 1e3 / n_steps,
        "device_ms_per_batch_step": float(np.median(dev)),
        "device_ms_per_batch_step_default_schedule": float(np.median(dev_default)),
        "autotune_gain": float(np.median(dev_default)) / max(float(np.median(dev)), 1e-9),
        # algorithmic bytes of one batch step (every session scores all 16
        # counters: Delta ~ U(-1, 1) has no zero): score pass 4 * 16 + 4 + 1/8,
        # weight pass 4 + 1/8 per valid configuration; draws are negligible
        "step_roofline": {
            "bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBS,
            "algorithmic_bytes": float(n_valid.sum() * (4 * 16 + 4 + 0.125 + 4 + 0.125)),
            "achieved": float(n_valid.sum() * (4 * 16 + 8.25)) / (float(np.median(dev)) / 1e3) / 1e9,
            "frac": float(n_valid.sum() * (4 * 16 + 8.25)) / (float(np.median(dev)) / 1e3) / 1e9
                    / HBM_PEAK_GBS,
        },
        "scored_per_s": scored / wall,
        "ms_per_step_sessions_one_by_one": wall_single * 1e3 / n_steps,
        "scored_per_s_one_by_one": scored / wall_single,
    }


def online_path(cgs, n_steps=200):
    """The 16-parameter space (2^14 * 3^8 = 107,495,424 raw configurations),
    forest of 16 depth-12 trees over 32 counters as the tree model and the
    synthetic profiler, perceptron 16 -> 512 -> 512 -> 32 retrained online."""
    import synth
    spec = synth.space_c5()
    t0 = time.perf_counter()
    sp = cgs.Space.from_spec(spec)
    t_space = time.perf_counter() - t0
    tree = cgs.ForestModel.from_spec(sp, synth.forest_c5(spec))
    g = synth.rng(5, 3)
    C = 32
    deltas = synth.deltas(g, n_steps, C)
    U = synth.uniforms_u64(g, n_steps + 1)
    noise = synth.normal_noise(g, (n_steps + 1, C), 0.02)
    valid = sp.copy_valid()
    seed_pos = synth.uniform_indices(synth.rng(5, 4), 8192, sp.n_valid)
    seed_tgt = tree.gather_predictions(seed_pos)
    seed_tgt += synth.normal_noise(synth.rng(5, 5), (8192, C), 0.02)
    init = synth.mlp_init((5, 6), len(spec.radix), 512, C)
    mlp = cgs.MLPModel(sp, [init.w[0], init.b[0], init.w[1], init.b[1], init.w[2], init.b[2]])
    t0 = time.perf_counter()
    mlp.train(valid[seed_pos], seed_tgt, synth.minibatches(synth.rng(5, 7), 2000, 256, 8192))
    t_first = time.perf_counter() - t0
    val_sample = synth.uniform_indices(synth.rng(5, 8), 65536, sp.n_valid)
    opts = cgs.cgs_default_online_opts()
    n_windows = 1 + n_steps // opts.retrain_every
    batch_u64 = synth.uniforms_u64(synth.rng(5, 9),
                                   (n_windows - 1) * opts.train_steps * opts.batch)
    log = cgs.Session(sp).online_run(tree, mlp, deltas, U, noise, valid[seed_pos], seed_tgt,
                                     val_sample, batch_u64, opts)
    inf_ms = mlp.eval_ms()
    flop = 2.0 * (16 * 512 + 512 * 512 + 512 * C) * sp.n_valid
    return {
        "n_raw": sp.n_raw, "n_valid": sp.n_valid, "space_create_ms": t_space * 1e3,
        "tree_eval_ms": tree.eval_ms(), "mlp_first_train_ms": t_first * 1e3,
        "mlp_inference_ms": inf_ms, "mlp_inference_tflops": flop / (inf_ms / 1e3) / 1e12,
        "mlp_inference_valu_roofline": valu_roofline(f"16-512-512-{C}", sp.n_valid, inf_ms),
        "windows": log["windows"], "retrain_ms_mean": float(np.mean(log["retrain_ms"])),
        "rmse_mean_predictor": mean_predictor_rmse(tree.gather_predictions(val_sample)),
        "step_ms_median": float(np.median(log["step_us"])) / 1e3, "steps": len(log["step_us"]),
        "scored_per_s": float(sp.n_valid / (np.median(log["step_us"]) / 1e6)),
    }


def neighbourhood_path(cgs, n_steps=200):
    """Restricted steps (the neighbourhood of the profiled configuration, Sect.
    3.7 footnote) on the 1.07e8-configuration space with its tree: radius 1,
    2 and 3, n_steps each, one draw per step (the pick profiled next),
    counter changes ~ U(-1, 1)."""
    import synth
    spec = synth.space_c5()
    sp = cgs.Space.from_spec(spec)
    tree = cgs.ForestModel.from_spec(sp, synth.forest_c5(spec))
    g = synth.rng(6, 1)
    deltas = synth.deltas(g, n_steps, tree.n_counters)
    U = synth.uniforms_u64(g, n_steps + 1)
    out = {"n_raw": sp.n_raw, "n_valid": sp.n_valid}
    for radius in (1, 2, 3):
        params = cgs.cgs_default_params()
        params.timing = TIMING_PERIOD
        sess = cgs.Session(sp, params)
        sess.search_step(tree, cgs.NO_PROFILE)
        raw, _ = sess.sample_next(int(U[0]))
        wall, cand = [], []
        for i in range(n_steps):
            t0 = time.perf_counter()
            sess.search_step_neighbourhood(tree, raw, radius, delta=deltas[i])
            r = sess.sample_next(int(U[i + 1]))
            wall.append(time.perf_counter() - t0)
            cand.append(sess.step_info().n_unexplored)
            if r is None:
                break
            raw = r[0]
        ms, n = sess.kernel_times()
        step_ms = float(np.median(wall)) * 1e3
        out[f"radius_{radius}"] = {
            "steps": len(wall), "candidates_mean": float(np.mean(cand)),
            "step_wall_ms_median": step_ms,
            "scoring_us": ms[3] / max(1, n[3]) * 1e3, "draw_us": ms[2] / max(1, n[2]) * 1e3,
            "scored_per_s": float(np.mean(cand)) / (step_ms / 1e3),
        }
        sess.close()
    tree.close()
    sp.close()
    return out


def _digits(raw, radix):
    """Digits of raw indices (parameter 0 most significant), for the
    synthetic measured counters."""
    raw = np.asarray(raw, dtype=np.int64)
    out = np.empty((len(raw), len(radix)), dtype=np.int64)
    for j in range(len(radix) - 1, -1, -1):
        out[:, j] = raw % radix[j]
        raw = raw // radix[j]
    return out


FIT_DEPTH, FIT_MIN_LEAF, FIT_COUNTERS = 12, 4, 24


_FIT_INPUTS = {}


def fit_inputs(spec, valid_raw):
    """Every valid configuration measured once: synthetic counters (steps on
    random parameters, a smooth term, 2% noise) and the split keys."""
    import synth
    if "Y" not in _FIT_INPUTS:
        g = synth.rng(7, 1)
        _FIT_INPUTS["Y"] = synth.measured_counters(g, _digits(valid_raw, spec.radix), spec.radix,
                                                   FIT_COUNTERS)
        _FIT_INPUTS["keys"] = synth.uniforms_u64(g, len(valid_raw))
    return _FIT_INPUTS["Y"], _FIT_INPUTS["keys"]


def tree_fit_path(cgs, sp, spec, repeats=5):
    """Regression-tree fitting (Sect. 3.4.2) on the 2^24 space: all
    4,813,824 valid configurations as measured points, 24 counters, depth
    12, leaves of at least 4 points.  fit_ms is the device time of the whole
    fit (select, quantise, grow, test, choose), inputs resident."""
    valid = sp.copy_valid()
    Y, keys = fit_inputs(spec, valid)
    points = np.arange(len(valid), dtype=np.uint32)
    runs, walls = [], []
    rep = None
    for _ in range(repeats):
        t0 = time.perf_counter()
        model, rep = cgs.ForestModel.fit(sp, points, Y, keys, FIT_DEPTH, FIT_MIN_LEAF)
        walls.append(time.perf_counter() - t0)
        runs.append(rep["fit_ms"])
        eval_ms = model.eval_ms()
        model.close()
    fit_ms = float(np.median(runs))
    n_test = rep["n_test"] * FIT_COUNTERS
    return {
        "points": len(points), "counters": FIT_COUNTERS, "max_depth": FIT_DEPTH,
        "min_leaf": FIT_MIN_LEAF, "fit_ms_median": fit_ms, "fit_ms_all": runs,
        "points_per_s": len(points) / (fit_ms / 1e3),
        "wall_ms_median": float(np.median(walls)) * 1e3,
        "selected_depth": rep["depth"], "split_nodes": rep["n_split"],
        "test_mae_by_depth": [a / n_test for a in rep["abs_err"]],
        "model_eval_ms": eval_ms,
    }


POLY_ORDER, POLY_COUNTERS = 3, 24
VALU_FP32_PEAK_T = 78.6   # fp32 FMA on the vector units, packed FP32 not used


def poly_path(cgs, sp, spec, repeats=3, n_heldout=100000, n_steps=20):
    """Least-squares polynomial models (Sect. 3.4.1) on the 2^24 space: the
    three-level design (every non-binary parameter at its lowest, middle and
    highest value) measured with synthetic counters, order-3 interactions
    plus squares (139 terms) in each of the 8 binary subspaces, 24 counters.
    Times the fit and the evaluation of every valid configuration; the
    counters of 100,000 other configurations (drawn in the same call, so the
    same synthetic function) give the held-out error; then n_steps search
    steps run on the fitted model."""
    import synth
    valid = sp.copy_valid()
    design = cgs.PolyModel.design(sp)
    g = synth.rng(8, 1)
    held = np.setdiff1d(g.choice(len(valid), n_heldout, replace=False), design)
    rows = np.concatenate([design, held])
    Y = synth.measured_counters(g, _digits(valid[rows], spec.radix), spec.radix, POLY_COUNTERS)
    fits, evals = [], []
    model = None
    for _ in range(repeats):
        if model is not None:
            model.close()
        model = cgs.PolyModel(sp, design, Y[: len(design)], POLY_ORDER)
        fits.append(model.report["fit_ms"])
        evals.append(model.report["eval_ms"])
    T = model.report["n_terms"]
    pred = model.gather_predictions(held.astype(np.uint32))
    truth = Y[len(design):]
    rel_mae = float(np.mean(np.abs(pred - truth) / (np.abs(truth).mean(axis=0) + 1e-30)))
    eval_ms = float(np.median(evals))
    flop = len(valid) * 2.0 * T * POLY_COUNTERS
    achieved = flop / (eval_ms / 1e3) / 1e12
    # the model drives the search like any other
    U, pcs, thr = workload_inputs(n_steps)
    t0 = time.perf_counter()
    _, sess = run_search(cgs, sp, model, U, pcs, expert_settings(cgs, thr), n_steps, timing=False)
    sp.synchronize()
    step_ms = (time.perf_counter() - t0) * 1e3 / n_steps
    sess.close()
    model.close()
    return {
        "design_points": int(len(design)), "subspaces": model.report["n_subspaces"],
        "terms": T, "order": POLY_ORDER, "counters": POLY_COUNTERS,
        "fit_ms_median": float(np.median(fits)), "eval_ms_median": eval_ms,
        "eval_configs_per_s": len(valid) / (eval_ms / 1e3),
        "heldout_configs": int(len(held)), "heldout_rel_mae": rel_mae,
        "search_step_ms": step_ms,
        "eval_roofline": {"kernel": "poly_eval", "bound": "valu", "achieved": achieved,
                          "peak": VALU_FP32_PEAK_T, "unit": "TFLOP/s",
                          "frac": achieved / VALU_FP32_PEAK_T,
                          "flop_per_config": 2 * T * POLY_COUNTERS},
    }


def tuning_path(cgs, n_runs=1000, big_runs=40, big_cap=30000):
    """Alg. 1 (Sect. 3.7) with the evaluation of Sect. 4.1 on a synthetic
    bottleneck-driven kernel: tests until a configuration within 1.1x of the
    best runtime is tested, averaged over n_runs runs, against random
    search's expected (N + 1) / (K + 1).  Models: the measured counters
    themselves (as in Sect. 4.3), a tree fitted on the counters of a random
    20% of the configurations (Sect. 3.4.2) and the least-squares
    polynomials fitted on the three-level design (Sect. 3.4.1).  Space: the
    6-parameter space (11,496 valid configurations), then big_runs runs
    capped at big_cap tests on the 2^24 space.  The measured-counter runs
    also run as batches (cgs_tuning_run_batch: 64 runs at once on the small
    space, all big_runs at once on the big one, which runs only batched);
    each batched run makes the tests of its sequential run."""
    import synth
    out = {}
    for name, spec, key, runs, cap in (("c1", synth.space_c1(), (9, 1), n_runs, None),
                                       ("c2", synth.space_c2(), (9, 2), big_runs, big_cap)):
        sp = cgs.Space.from_spec(spec)
        valid = sp.copy_valid()
        table = synth.kernel_table(synth.rng(*key), _digits(valid, spec.radix), spec.radix)
        rt = table.runtime.astype(np.float64)
        well = rt <= 1.1 * rt.min()
        N, K = len(rt), int(well.sum())
        rec = {"n_valid": N, "well_performing": K, "random_expected": (N + 1) / (K + 1),
               "runs": runs, "cap": cap}
        models = {"measured": cgs.TableModel(sp, table.counters.astype(np.float32))}
        if name == "c1":
            g = synth.rng(10, 1)
            pts = np.sort(g.choice(N, N // 5, replace=False)).astype(np.uint32)
            tree, rep = cgs.ForestModel.fit(sp, pts, table.counters[pts].astype(np.float32),
                                            synth.uniforms_u64(g, len(pts)), 8, 2)
            models["fitted_tree"] = tree
            design = cgs.PolyModel.design(sp)
            models["polynomial"] = cgs.PolyModel(sp, design,
                                                 table.counters[design].astype(np.float32), 2)
        ep = cgs.cgs_expert_params(inst_reaction=0.7, volta=0, reserved=0, cores=1.0, threads=1e9)
        seq_tests = {}
        for mname, model in models.items():
            if cap:
                continue   # the capped runs on the big space run as one batch below
            tests, wall, found_flags = [], [], []
            for r in range(runs):
                U = synth.uniforms_u64(synth.rng(11, r), (cap or 4 * N) + 8)
                sess = cgs.Session(sp)
                t0 = time.perf_counter()
                tested, _, tw = sess.tuning_run(model, table.runtime, table.counters, U,
                                                max_tests=cap, expert=ep)
                wall.append(time.perf_counter() - t0)
                tests.append(tw if tw else len(tested))
                found_flags.append(tw > 0)
                sess.close()
            tests = np.asarray(tests, dtype=np.float64)
            found = [x for x, f in zip(tests, found_flags) if f] if cap else list(tests)
            r = {"ms_per_run": float(np.mean(wall)) * 1e3,
                 "us_per_test": float(np.sum(wall) / tests.sum()) * 1e6}
            if cap:
                # runs stopped at the cap are censored: compare the share of
                # runs that found a well-performing configuration within the
                # cap with random search's probability of doing so
                p_rand = 1.0 - float(np.exp(np.sum(np.log1p(-K / (N - np.arange(cap))))))
                r.update({"found_within_cap": len(found), "share_found": len(found) / runs,
                          "random_share_found": p_rand,
                          "mean_tests_when_found": float(np.mean(found)) if found else None})
            else:
                r.update({"mean_tests": float(tests.mean()), "median_tests": float(np.median(tests)),
                          "improvement": rec["random_expected"] / float(tests.mean())})
            rec[mname] = r
            seq_tests[mname] = tests
        # the measured-counter runs again, many at once (cgs_tuning_run_batch):
        # every run makes the tests of its sequential run
        model = models["measured"]
        bsize = 64 if cap is None else runs
        tests, found_flags, wall = [], [], 0.0
        for b0 in range(0, runs, bsize):
            ids = list(range(b0, min(runs, b0 + bsize)))
            U = np.stack([synth.uniforms_u64(synth.rng(11, r), (cap or 4 * N) + 8) for r in ids])
            sessions = [cgs.Session(sp) for _ in ids]
            batch = cgs.Batch(sessions, [model] * len(ids))
            t0 = time.perf_counter()
            res = batch.tuning_run(table.runtime, table.counters, U, max_tests=cap, expert=ep)
            wall += time.perf_counter() - t0
            batch.close()
            for s in sessions:
                s.close()
            for tested, _, tw in res:
                tests.append(tw if tw else len(tested))
                found_flags.append(tw > 0)
        tests = np.asarray(tests, dtype=np.float64)
        rb = {"batch": bsize, "runs_per_s": runs / wall, "us_per_test": float(wall / tests.sum() * 1e6)}
        if cap:
            found = [x for x, f in zip(tests, found_flags) if f]
            p_rand = 1.0 - float(np.exp(np.sum(np.log1p(-K / (N - np.arange(cap))))))
            rb.update({"found_within_cap": len(found), "share_found": len(found) / runs,
                       "random_share_found": p_rand,
                       "mean_tests_when_found": float(np.mean(found)) if found else None})
        else:
            rb.update({"mean_tests": float(tests.mean()),
                       "equal_to_sequential": bool(np.array_equal(tests, seq_tests["measured"])),
                       "sequential_runs_per_s": 1e3 / rec["measured"]["ms_per_run"]})
        rec["measured_batched"] = rb
        for model in models.values():
            model.close()
        out[name] = rec
        sp.close()
    return out


def cpu_tuning_baseline(n_runs=160):
    """The oracle's Alg. 1 loop, untouched, single thread, on the first
    n_runs runs of the c1 measured-counter workload."""
    import synth
    from threadpoolctl import threadpool_limits

    from oracle import search as SR
    from oracle import space as SP
    from oracle import tuning as TU
    spec = synth.space_c1()
    valid = SP.enumerate_valid(spec.radix, spec.values, spec.constraints)
    digits = SP.digits_of(valid, spec.radix)
    table = synth.kernel_table(synth.rng(9, 1), digits, spec.radix)
    prep = SR.Prepared(valid, digits, None, table.counters, table.counters.astype(np.float32))
    tests = 0
    with threadpool_limits(1):
        t0 = time.perf_counter()
        for r in range(n_runs):
            U = synth.uniforms_u64(synth.rng(11, r), 4 * len(valid) + 8)
            tests += TU.run(prep, table.runtime, table.counters, U, cores=1.0,
                            threads=1e9).tests_to_well
        dt = time.perf_counter() - t0
    return {"value": n_runs / dt, "unit": "runs/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_runs} runs of the 11,496-configuration workload, measured "
                      f"counters as the model ({dt:.1f} s, {tests / dt:.0f} tests/s)"}


def cpu_fit_baseline(spec, sp, n_sample=1000000):
    """The oracle's tree fit, untouched, single thread, on the first
    n_sample points of the same fit workload (same counters and keys)."""
    from threadpoolctl import threadpool_limits

    from oracle import treefit as TF
    valid = sp.copy_valid()
    Y, keys = fit_inputs(spec, valid)
    digits = _digits(valid[:n_sample], spec.radix)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        r = TF.fit(digits, Y[:n_sample], keys[:n_sample], spec.radix, FIT_DEPTH, FIT_MIN_LEAF)
        dt = time.perf_counter() - t0
    return {"value": n_sample / dt, "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_sample} of the 4,813,824 fit points, depth {FIT_DEPTH}, "
                      f"{FIT_COUNTERS} counters ({dt:.1f} s)", "selected_depth": r.depth}


def cpu_baseline(spec, forest, n_steps):
    """The oracle, untouched, on a bounded sample of the workload: the valid
    configurations with raw index below 2^22 (a quarter of the raw space),
    one model evaluation and the same n_steps scored steps (previous pick
    profiled, counter changes from the same counter vectors), single thread.
    Rate: sample x n_steps / (evaluation + steps)."""
    from threadpoolctl import threadpool_limits

    from oracle import expert as E
    from oracle import search as SR
    from oracle import space as SP
    with threadpool_limits(1):
        t0 = time.perf_counter()
        mask = SP.valid_mask(spec.radix, spec.values, spec.constraints, chunk=1 << 21)
        sample = np.flatnonzero(mask[: 1 << 22]).astype(np.uint32)
        del mask
        t1 = time.perf_counter()
        prep = SR.prepare(spec, forest, valid=sample)
        t2 = time.perf_counter()
        U, pcs, thr = workload_inputs(n_steps)
        explored = np.zeros(len(sample), dtype=bool)
        r = SR.step(prep, explored, None, np.zeros(24, np.float32), [int(U[0])])
        prof = r.picks[0]
        t3 = time.perf_counter()
        for i in range(n_steps):
            _, _, d32, _ = E.expert_system(pcs[i], False, CORES_PROFILED, float(thr[i]), 0.7)
            r = SR.step(prep, explored, prof, d32, [int(U[i + 1])])
            prof = r.picks[0]
        t4 = time.perf_counter()
    t_eval, t_steps = t2 - t1, t4 - t3
    rate = len(sample) * n_steps / (t_eval + t_steps)
    cpu_model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {
        "value": rate, "unit": "configs/s", "cores": 1, "kind": "oracle", "cpu_model": cpu_model,
        "sample": (f"valid configurations with raw index < 2^22 of the same space ({len(sample)}): "
                   f"oracle model evaluation {t_eval:.2f} s + {n_steps} scored steps "
                   f"{t_steps:.2f} s; NumPy, one thread (enumeration {t1 - t0:.2f} s and the "
                   f"uniform start not counted)"),
    }


def inference_sweeps(cgs):
    """The perceptron inference of both workloads, untrained weights: the
    12-256-256-24 network over the 2^24 space and the 16-512-512-32 network
    over the 1.07e8 space (model load + two refreshes each)."""
    import synth
    for spec_fn, H, C, key in ((synth.space_c2, 256, 24, (3, 2)), (synth.space_c5, 512, 32, (5, 6))):
        spec = spec_fn()
        sp = cgs.Space.from_spec(spec)
        init = synth.mlp_init(key, len(spec.radix), H, C)
        model = cgs.MLPModel(sp, [init.w[0], init.b[0], init.w[1], init.b[1], init.w[2], init.b[2]])
        for _ in range(2):
            model.refresh()
        log(f"inference {len(spec.radix)}-{H}-{H}-{C}: {sp.n_valid} configs, {model.eval_ms():.3f} ms")
        model.close()
        sp.close()


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mlp", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-online", action="store_true")
    ap.add_argument("--no-neighbourhood", action="store_true")
    ap.add_argument("--no-fit", action="store_true")
    ap.add_argument("--no-poly", action="store_true")
    ap.add_argument("--no-tuning", action="store_true")
    ap.add_argument("--inference-only", action="store_true",
                    help="only the two perceptron inference sweeps (for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the sweep runs on a single MI355X "
              "(multi-GPU sharding is design-only); run with --gpus 1", file=sys.stderr)
        return 2
    K, W = args.steps, args.warmup
    if K < 1:
        print("--steps must be >= 1", file=sys.stderr)
        return 2

    import synth
    from paper_2102_05297_amd import cgs   # fails loudly without the HIP library

    if args.inference_only:
        inference_sweeps(cgs)
        return 0

    spec = synth.space_c2()
    forest = synth.forest_c2(spec)
    t0 = time.perf_counter()
    sp = cgs.Space.from_spec(spec)
    t_enum = time.perf_counter() - t0
    model = cgs.ForestModel.from_spec(sp, forest)
    log(f"space: {sp.n_raw} raw, {sp.n_valid} valid (create {t_enum * 1e3:.1f} ms); "
        f"forest eval {model.eval_ms():.3f} ms")
    U, pcs, thr = workload_inputs(max(K, W))
    eps = expert_settings(cgs, thr)       # per-step inputs, prepared before timing

    # counters entering each step's score (for the algorithmic byte count)
    n_active = []
    for i in range(K):
        ep = cgs.cgs_expert_params(inst_reaction=0.7, volta=0, reserved=0, cores=CORES_PROFILED,
                                   threads=float(thr[i]))
        _, d, _ = cgs.cgs_expert_system(pcs[i], ep)
        n_active.append(int((d.astype(np.float32) != 0).sum()))

    if W > 0:
        run_search(cgs, sp, model, U, pcs, eps, W, timing=False)
        sp.synchronize()
        log(f"warmup: {W} steps done")

    sp.synchronize()
    t_start = time.perf_counter()
    model.refresh()                       # model evaluation inside the timed region
    picks, sess = run_search(cgs, sp, model, U, pcs, eps, K, timing=TIMING_PERIOD)
    sp.synchronize()
    t_total = time.perf_counter() - t_start
    log(f"timed: {K} steps in {t_total * 1e3:.2f} ms")

    n_valid = sp.n_valid
    # step i (1-based) scores every valid configuration except the profile
    # and the i picks so far: n_valid - i
    scored = sum(n_valid - i for i in range(1, K + 1))
    value = scored / t_total

    ms, launches = sess.kernel_times()
    wall = np.asarray(sess.step_wall_s) * 1e3
    kavg = [ms[k] / max(1, launches[k]) for k in range(3)]  # ms per launch
    device_step_ms = sum(kavg)
    # score pass of step j (0 = the uniform start, no active counter): reads
    # the rows of P of its active counters, writes s, reads the explored bits;
    # the timed launches are those of steps 0, k, 2k, ...
    # timed steps: 0, k, 2k, ...; the score-pass totals hold the scored ones
    # only (step 0, the uniform start, reads no prediction)
    timed = [j for j in range(1, K + 1) if j % TIMING_PERIOD == 0]
    assert len(timed) == int(launches[0])
    act = [0] + n_active
    bytes_score = sum(n_valid * (4 + 0.125 + 4.0 * act[j]) for j in timed)
    traffic = pmc_traffic([act[j] for j in timed])
    score_s = ms[0] / 1e3
    achieved = bytes_score / score_s / 1e9 if score_s > 0 else 0.0
    # the whole scored step: score pass as above; weight pass reads s and the
    # explored bits (4 + 1/8 B per configuration) and writes 8 B per block;
    # the draw reads the block sums and one block's scores and explored words
    blk = 1 << max(12, next(b for b in range(12, 21) if (n_valid >> b) < 65536))
    n_blocks = (n_valid + blk - 1) // blk
    bytes_weight = n_valid * (4 + 0.125) + 8 * n_blocks
    bytes_draw = 8 * n_blocks + blk * (4 + 0.125)
    step_bytes = bytes_score / max(1, len(timed)) + bytes_weight + bytes_draw
    step_us = sum(ms[k] / max(1, launches[k]) for k in range(3)) * 1e3
    step_achieved = step_bytes / (step_us / 1e6) / 1e9 if step_us > 0 else 0.0

    # oracle-exact picks: stored oracle trajectory for the same inputs
    golden_path = os.path.join(ROOT, "tests", "golden", "c2_search.json")
    exact = None
    if os.path.exists(golden_path):
        ref = json.load(open(golden_path))["steps"]
        n_chk = min(len(ref), len(picks))
        exact = {"checked": n_chk,
                 "equal": int(sum(ref[i]["pick"] == picks[i] for i in range(n_chk)))}
        log(f"picks equal to the oracle trajectory: {exact['equal']}/{exact['checked']}")

    probe = copy_probe()
    log(f"copy probe: {probe}")

    batch = None
    if not args.no_batch:
        batch = batch_path(cgs)
        log(f"batch: {batch}")

    online = None
    if not args.no_online:
        online = online_path(cgs)
        log(f"online: {online}")

    nbh = None
    if not args.no_neighbourhood:
        nbh = neighbourhood_path(cgs)
        log(f"neighbourhood: {nbh}")

    fit = None
    if not args.no_fit:
        fit = tree_fit_path(cgs, sp, spec)
        log(f"tree fit: {fit}")

    poly = None
    if not args.no_poly:
        poly = poly_path(cgs, sp, spec)
        log(f"poly: {poly}")

    tuning = None
    if not args.no_tuning:
        tuning = tuning_path(cgs)
        log(f"tuning: {tuning}")

    mlp = None
    if not args.no_mlp:
        mlp = mlp_path(cgs, sp, model)
        log(f"mlp: {mlp}")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample) ...")
        cpu = cpu_baseline(spec, forest, K)
        if fit is not None:
            fit["cpu_baseline"] = cpu_fit_baseline(spec, sp)
            log(f"tree fit cpu baseline: {fit['cpu_baseline']}")
        if tuning is not None:
            tuning["cpu_baseline"] = cpu_tuning_baseline()
            log(f"tuning cpu baseline: {tuning['cpu_baseline']}")

    out = {
        "metric": "configs scored/sec per search step (tree vs MLP surrogate) at oracle-exact pick",
        "value": value,
        "unit": "configs/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": t_total * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": ("12-param space, 16,777,216 raw / %d valid configs, forest 16 trees depth 12, "
                         "24 counters, %d sequential steps, 1 draw per step, tree model" % (n_valid, K)),
            "n_raw": sp.n_raw, "n_valid": n_valid, "trees": 16, "depth": 12, "counters": 24,
            "model": "forest (predictions evaluated once per timed run, inside the timed region)",
        },
        "roofline": {
            "kernel": "score_pass",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": bytes_score / max(1, len(timed)),
            "launches": int(launches[0]),
            "avg_us": ms[0] / max(1, launches[0]) * 1e3,
            "timing": "HIP events around every %d-th scored step's kernels" % TIMING_PERIOD,
        },
        # score + weight + draw of one scored step against the same peak
        "step_roofline": {
            "kernels": "score_pass + weight_pass + draw",
            "bound": "hbm",
            "achieved": step_achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": step_achieved / HBM_PEAK_GBS,
            "algorithmic_bytes_per_step": step_bytes,
            "device_us": step_us,
        },
        "step_wall_ms": {"median": float(np.median(wall)), "p10": float(np.percentile(wall, 10)),
                         "p90": float(np.percentile(wall, 90))},
        # N_u over the device time of one step (score + weight + draw averages
        # over the timed steps); the wall-clock value above adds the host side
        "device_rate_per_s": n_valid / (device_step_ms / 1e3) if device_step_ms > 0 else None,
        "kernel_avg_us": {
            "score_pass": ms[0] / max(1, launches[0]) * 1e3,
            "weight_pass": ms[1] / max(1, launches[1]) * 1e3,
            "draw": ms[2] / max(1, launches[2]) * 1e3,
        },
        "tree_eval_in_step_per_s": n_valid / ((model.eval_ms() + t_total * 1e3 / K) / 1e3),
        "mlp": mlp,
        "batch": batch,
        "online": online,
        "neighbourhood": nbh,
        "tree_fit": fit,
        "poly": poly,
        "tuning": tuning,
        "hbm_copy_probe": probe,
        "model_eval_ms": model.eval_ms(),
        "space_create_ms": t_enum * 1e3,
        "mean_active_counters": float(np.mean(n_active)),
        "oracle_exact_picks": exact,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
