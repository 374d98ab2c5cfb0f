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
