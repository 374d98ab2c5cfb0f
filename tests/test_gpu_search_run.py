"""cgs_search_run (the whole one-draw-per-step search of Alg. 1, Sect. 3.7,
driven by the library) against the oracle's steps on a small space: every
pick until the space is exhausted, then CGS_EEMPTY; and the search with no
profiled step."""
import numpy as np
import pytest

import synth
from oracle import expert as E
from oracle import search as SR
from oracle import space as SP
from tests.helpers import cgs

pytestmark = pytest.mark.gpu

RADIX = [3, 4, 2, 5]
VALUES = [[1, 2, 4], [1, 2, 4, 8], [0, 1], [1, 2, 4, 8, 16]]


def _setup(m):
    spec = synth.Space(RADIX, VALUES, [])
    valid = SP.enumerate_valid(spec.radix, spec.values, spec.constraints)
    digits = SP.digits_of(valid, spec.radix)
    table = synth.kernel_table(synth.rng(61), digits, spec.radix)
    P = table.counters
    prep = SR.Prepared(valid, digits, None, P, P.astype(np.float32))
    sp = m.Space.from_spec(spec)
    model = m.TableModel(sp, P.astype(np.float32))
    return valid, prep, sp, model


def _oracle_picks(prep, pcs, thr, U, n_steps):
    explored = np.zeros(len(prep.valid), dtype=bool)
    picks = [SR.step(prep, explored, None, np.zeros(24, np.float32), [int(U[0])],
                     with_fp64=False).picks[0]]
    for i in range(n_steps):
        _, _, d32, _ = E.expert_system(pcs[i], False, 1.0, float(thr[i]), 0.7)
        picks.append(SR.step(prep, explored, picks[-1], d32, [int(U[i + 1])],
                             with_fp64=False).picks[0])
    return picks


def test_search_run_to_exhaustion_equals_the_oracle():
    m = cgs()
    valid, prep, sp, model = _setup(m)
    N = len(valid)
    pcs = synth.profiler_counters(synth.rng(62), N)
    thr = synth.threads_launched(synth.rng(63), N)
    U = synth.uniforms_u64(synth.rng(64), N + 1)
    eps = [m.cgs_expert_params(inst_reaction=0.7, volta=0, reserved=0, cores=1.0,
                               threads=float(x)) for x in thr]
    print(f"search_run: {N} configurations, {N - 1} steps", flush=True)
    raw, val, t_us = m.Session(sp).search_run(model, pcs[:N - 1], eps[:N - 1], U[:N])
    ref = _oracle_picks(prep, pcs, thr, U, N - 1)
    assert val.tolist() == ref
    assert sorted(val.tolist()) == list(range(N))            # every configuration once
    assert raw.tolist() == [int(valid[l]) for l in ref]
    with pytest.raises(m.CgsError) as ei:                     # one draw too many
        m.Session(sp).search_run(model, pcs[:N], eps[:N], U[:N + 1])
    assert ei.value.status == m.EEMPTY


def test_search_run_without_steps():
    m = cgs()
    valid, prep, sp, model = _setup(m)
    U = synth.uniforms_u64(synth.rng(65), 1)
    raw, val, t_us = m.Session(sp).search_run(model, np.zeros((0, 24)), [], U)
    assert val.tolist() == _oracle_picks(prep, None, None, U, 0)
    assert len(t_us) == 0


# 432,432 valid configurations: 106 blocks of 4,096 weights (the last one
# ragged), or 7 blocks of 65,536
WIDE_RADIX = [9, 11, 13, 7, 8, 6]


@pytest.mark.parametrize("block_log2", [12, 16])
def test_search_run_over_many_blocks_equals_the_oracle_and_the_step_calls(block_log2):
    """The search run enqueues its steps ahead of their picks (each step's
    kernels read the configuration to profile from device memory).  Over many
    blocks, with a ragged last block, its picks equal the oracle's; afterwards
    the session is as the same search made by step calls leaves it (scores,
    weights, explored bits, step statistics, a further draw of the last step,
    and a second search run on the same session)."""
    m = cgs()
    spec = synth.Space(WIDE_RADIX, [list(range(1, r + 1)) for r in WIDE_RADIX], [])
    valid = SP.enumerate_valid(spec.radix, spec.values, spec.constraints)
    digits = SP.digits_of(valid, spec.radix)
    P = synth.kernel_table(synth.rng(71), digits, spec.radix).counters
    prep = SR.Prepared(valid, digits, None, P, P.astype(np.float32))
    sp = m.Space.from_spec(spec)
    model = m.TableModel(sp, P.astype(np.float32))
    n_steps = 30
    pcs = synth.profiler_counters(synth.rng(73), n_steps)
    thr = synth.threads_launched(synth.rng(74), n_steps)
    U = synth.uniforms_u64(synth.rng(72), n_steps + 2)
    eps = [m.cgs_expert_params(inst_reaction=0.7, volta=0, reserved=0, cores=1.0,
                               threads=float(x)) for x in thr]
    params = m.cgs_params(gamma=-0.25, w_min=1e-4, block_log2=block_log2, timing=0)
    print(f"search_run over {len(valid)} configurations, block_log2 {block_log2}", flush=True)
    run = m.Session(sp, params)
    raw, val, _ = run.search_run(model, pcs, eps, U[:n_steps + 1])
    assert val.tolist() == _oracle_picks(prep, pcs, thr, U, n_steps)
    assert raw.tolist() == [int(valid[l]) for l in val]

    calls = m.Session(sp, params)
    prof = m.NO_PROFILE
    for i in range(n_steps + 1):
        if i == 0:
            calls.search_step(model, prof)
        else:
            calls.search_step(model, prof, measured=pcs[i - 1], expert=eps[i - 1])
        prof, _ = calls.sample_next(int(U[i]))
    assert (run.copy_scores().view(np.uint32) == calls.copy_scores().view(np.uint32)).all()
    assert (run.copy_weights() == calls.copy_weights()).all()
    assert (run.copy_explored() == calls.copy_explored()).all()
    a, b = run.step_info(), calls.step_info()
    for f in ("total_weight", "n_unexplored", "n_active", "s_min", "s_max"):
        assert getattr(a, f) == getattr(b, f), f
    assert run.sample_next(int(U[n_steps + 1])) == calls.sample_next(int(U[n_steps + 1]))
    # a second search on the same session goes on from its explored set
    _, val2, _ = run.search_run(model, pcs[:5], eps[:5], U[:6])
    prof, got = m.NO_PROFILE, []
    for i in range(6):
        if i == 0:
            calls.search_step(model, prof)
        else:
            calls.search_step(model, prof, measured=pcs[i - 1], expert=eps[i - 1])
        prof, l = calls.sample_next(int(U[i]))
        got.append(l)
    assert val2.tolist() == got
