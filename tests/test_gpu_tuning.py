"""The searcher's outer loop (Alg. 1, Sect. 3.7) on the GPU vs the oracle:
with the same tables and random numbers, every tested configuration, the
profiled flags and the tests to the first well-performing configuration are
equal."""
import numpy as np
import pytest

import synth
from oracle import expert as EX
from oracle import search as SR
from oracle import space as SP
from oracle import tuning as TU
from tests.helpers import cgs

pytestmark = pytest.mark.gpu


def _setup(spec, key):
    valid = SP.enumerate_valid(spec.radix, spec.values, spec.constraints)
    digits = SP.digits_of(valid, spec.radix)
    table = synth.kernel_table(synth.rng(*key), digits, spec.radix)
    P = table.counters
    prep = SR.Prepared(valid, digits, None, P, P.astype(np.float32))
    return valid, table, prep


def _expert(m):
    return m.cgs_expert_params(inst_reaction=0.7, volta=0, reserved=0, cores=1.0, threads=1e9)


def _pair(m, spec, table, prep, seed, n_u, **kw):
    sp = m.Space.from_spec(spec)
    model = m.TableModel(sp, table.counters.astype(np.float32))
    U = synth.uniforms_u64(synth.rng(50, seed), n_u)
    sess = m.Session(sp)
    print(f"loop: seed {seed} {kw}", flush=True)
    tested, prof, tw = sess.tuning_run(model, table.runtime, table.counters, U,
                                       expert=_expert(m), **kw)
    kw_o = dict(kw)
    if "max_tests" in kw_o and kw_o["max_tests"] is None:
        kw_o.pop("max_tests")
    ref = TU.run(prep, table.runtime, table.counters, U, cores=1.0, threads=1e9, **kw_o)
    assert tested.tolist() == ref.tested
    assert prof.tolist() == ref.profiled
    assert tw == ref.tests_to_well
    return ref


@pytest.mark.parametrize("seed", range(8))
def test_c1_runs_equal_the_oracle(seed):
    spec = synth.space_c1()
    valid, table, prep = _setup(spec, (9, 1))
    ref = _pair(cgs(), spec, table, prep, seed, 20000)
    assert ref.tests_to_well > 0


# an iteration's draws go out together (up to 33: the first with the step,
# the rest in one launch); 40 takes the one-at-a-time path
@pytest.mark.parametrize("seed,draws", [(0, 5), (1, 3), (2, 1), (3, 33), (4, 40)])
def test_small_space_runs_to_exhaustion(seed, draws):
    radix = [3, 4, 2, 5, 3]
    values = [[1, 2, 4], [1, 2, 4, 8], [0, 1], [1, 2, 4, 8, 16], [1, 2, 4]]
    spec = synth.Space(radix, values, [])
    valid, table, prep = _setup(spec, (41,))
    ref = _pair(cgs(), spec, table, prep, 100 + seed, 4000, draws=draws, stop_at_well=False)
    assert set(ref.tested) == set(range(len(valid)))


def test_c2_first_iterations_equal_the_oracle():
    spec = synth.space_c2()
    valid, table, prep = _setup(spec, (9, 2))
    _pair(cgs(), spec, table, prep, 7, 200, max_tests=48, stop_at_well=False)


def test_loop_errors():
    m = cgs()
    spec = synth.space_c1()
    valid, table, prep = _setup(spec, (9, 1))
    sp = m.Space.from_spec(spec)
    small = m.TableModel(sp, table.counters[:, :12].astype(np.float32))
    with pytest.raises(m.CgsError) as ei:
        m.Session(sp).tuning_run(small, table.runtime, table.counters, np.arange(100, dtype=np.uint64))
    assert ei.value.status == m.EINVAL
    model = m.TableModel(sp, table.counters.astype(np.float32))
    with pytest.raises(m.CgsError) as ei:
        m.Session(sp).tuning_run(model, table.runtime, table.counters,
                                 synth.uniforms_u64(synth.rng(51), 4), stop_at_well=False,
                                 max_tests=100)
    assert ei.value.status == m.ERANGE
    bad = table.counters[:3].astype(np.float32).copy()
    with pytest.raises(ValueError):
        m.TableModel(sp, bad)


# ---------------------------------------------------- runs of a batch at once
def _batch(m, spec, table, n):
    sp = m.Space.from_spec(spec)
    models = [m.TableModel(sp, table.counters.astype(np.float32)) for _ in range(n)]
    sessions = [m.Session(sp) for _ in range(n)]
    return m.Batch(sessions, models)


def _batch_vs_oracle(spec, key, seeds, n_u, **kw):
    m = cgs()
    valid, table, prep = _setup(spec, key)
    U = np.stack([synth.uniforms_u64(synth.rng(52, s), n_u) for s in seeds])
    b = _batch(m, spec, table, len(seeds))
    print(f"batched loop: seeds {list(seeds)} {kw}", flush=True)
    runs = b.tuning_run(table.runtime, table.counters, U, expert=_expert(m), **kw)
    kw_o = {k: v for k, v in kw.items() if not (k == "max_tests" and v is None)}
    refs = []
    for i, (tested, prof, tw) in enumerate(runs):
        ref = TU.run(prep, table.runtime, table.counters, U[i], cores=1.0, threads=1e9, **kw_o)
        assert tested.tolist() == ref.tested, f"run {i}"
        assert prof.tolist() == ref.profiled, f"run {i}"
        assert tw == ref.tests_to_well, f"run {i}"
        refs.append(ref)
    return refs


def test_batched_c1_runs_equal_the_oracle():
    refs = _batch_vs_oracle(synth.space_c1(), (9, 1), range(12), 20000)
    assert all(r.tests_to_well > 0 for r in refs)
    assert len({len(r.tested) for r in refs}) > 1   # the runs end at different tests


@pytest.mark.parametrize("draws", [1, 3])
def test_batched_small_space_runs_to_exhaustion(draws):
    radix = [3, 4, 2, 5, 3]
    values = [[1, 2, 4], [1, 2, 4, 8], [0, 1], [1, 2, 4, 8, 16], [1, 2, 4]]
    spec = synth.Space(radix, values, [])
    refs = _batch_vs_oracle(spec, (41,), range(200, 205), 4000, draws=draws, stop_at_well=False)
    for r in refs:
        assert sorted(set(r.tested)) == list(range(360))


def test_batched_c2_first_iterations_equal_the_oracle():
    # a mix of run lengths: some runs stop at max_tests, the batch goes on
    _batch_vs_oracle(synth.space_c2(), (9, 2), range(300, 303), 200, max_tests=36,
                     stop_at_well=False)


def test_batched_draws_equal_the_oracle_step():
    """cgs_batch_draw: the further draws of a step, session by session, are
    the picks of the oracle's step with the same random numbers."""
    m = cgs()
    spec = synth.space_c1()
    valid, table, prep = _setup(spec, (9, 1))
    n, k = 3, 4
    b = _batch(m, spec, table, n)
    profiles = [17, 4000, 9000]
    deltas, prof_raw = [], []
    for l in profiles:
        # the oracle's expert system, with the settings of _expert
        _, _, d32, _ = EX.expert_system(table.counters[l], False, 1.0, 1e9, 0.7)
        deltas.append(np.asarray(d32, dtype=np.float32))
        prof_raw.append(int(valid[l]))
    U = synth.uniforms_u64(synth.rng(53), n * (k + 1)).reshape(k + 1, n)
    picks = [[] for _ in range(n)]
    _, val, st = b.step(prof_raw, deltas, U[0])
    assert (st == 0).all()
    for i in range(n):
        picks[i].append(int(val[i]))
    for j in range(1, k + 1):
        _, val, st = b.draw(U[j])
        assert (st == 0).all()
        for i in range(n):
            picks[i].append(int(val[i]))
    for i, l in enumerate(profiles):
        explored = np.zeros(len(valid), dtype=bool)
        ref = SR.step(prep, explored, l, deltas[i], [int(U[j][i]) for j in range(k + 1)],
                      with_fp64=False)
        assert picks[i] == ref.picks, f"session {i}"


def test_batched_loop_errors():
    m = cgs()
    spec = synth.space_c1()
    valid, table, prep = _setup(spec, (9, 1))
    b = _batch(m, spec, table, 2)
    with pytest.raises(m.CgsError) as ei:               # no batch step yet
        b.draw(np.arange(2, dtype=np.uint64))
    assert ei.value.status == m.ESTATE
    with pytest.raises(ValueError):
        b.tuning_run(table.runtime, table.counters, np.arange(6, dtype=np.uint64))
    with pytest.raises(m.CgsError) as ei:               # random numbers run out
        b.tuning_run(table.runtime, table.counters,
                     synth.uniforms_u64(synth.rng(54), 8).reshape(2, 4), stop_at_well=False,
                     max_tests=100)
    assert ei.value.status == m.ERANGE
