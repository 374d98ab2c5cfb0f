"""GPU search step vs the oracle (Sect. 3.6-3.7, Alg. 1): scores bit-exact
against the oracle's float32 chain and within float32 rounding of its
float64 definition; quantised weights, totals and picks bit-exact."""
import numpy as np
import pytest

import synth
from oracle import expert as E
from oracle import sampling as S
from oracle import search as SR
from oracle import space as SP
from tests.helpers import bits_to_bool, cgs

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


def score_tolerance(s64, delta):
    """|s32 - s64| bound: 1e-5 relative, plus the float32 forward-error bound
    of the sum where cancellation makes the relative error meaningless:
    (C + 12) u sum|dpc| (leaf mean, subtraction, addition, division, product
    and C additions, each one rounding of u = 2^-24)."""
    C = len(delta)
    return 1e-5 * np.abs(s64) + (C + 12) * U32 * float(np.abs(np.asarray(delta, np.float64)).sum())


class Pair:
    """The same search run on the GPU and on the oracle."""

    def __init__(self, spec, forest, params=None):
        m = cgs()
        self.m = m
        self.spec = spec
        self.sp = m.Space.from_spec(spec)
        self.model = m.ForestModel.from_spec(self.sp, forest)
        self.sess = m.Session(self.sp, params)
        self.prep = SR.prepare(spec, forest)
        assert (self.sp.copy_valid() == self.prep.valid).all()
        self.explored = np.zeros(len(self.prep.valid), dtype=bool)

    def step(self, profile_l, delta, uniforms, check_scores=True):
        m = self.m
        raw = m.NO_PROFILE if profile_l is None else int(self.prep.valid[profile_l])
        self.sess.search_step(self.model, raw, delta=delta)
        ref = SR.step(self.prep, self.explored, profile_l, delta, uniforms)
        if check_scores:
            at_scoring = self.explored.copy()
            for l in ref.picks:
                if l is not None:
                    at_scoring[l] = False
            un = ~at_scoring
            s = self.sess.copy_scores()
            assert (s[un] == ref.s32[un]).all()
            tol = score_tolerance(ref.s64[un], delta)
            assert (np.abs(s[un].astype(np.float64) - ref.s64[un]) <= tol).all()
            q = self.sess.copy_weights()
            assert (q.astype(np.uint64) == ref.q).all()
        picks = []
        for U in uniforms:
            r = self.sess.sample_next(int(U))
            picks.append(None if r is None else r[1])
            if r is not None:
                assert r[0] == self.prep.valid[r[1]]
        ref_picks = list(ref.picks) + [None] * (len(picks) - len(ref.picks))
        assert picks == ref_picks, (picks, ref.picks)
        info = self.sess.step_info()
        return ref, info


def test_c1_single_step_configuration():
    """The 30,720-configuration space: start from a uniform draw, then one scored step with 12
    bottleneck weights ~ U(-1,1) and one seeded uniform."""
    spec = synth.space_c1()
    pair = Pair(spec, synth.forest_c1(spec))
    g = synth.rng(1, 3)
    U = synth.uniforms_u64(g, 2)
    delta = synth.deltas(g, 1, 12)[0]
    ref0, _ = pair.step(None, np.zeros(12, np.float32), [U[0]])
    ref1, info = pair.step(ref0.picks[0], delta, [U[1]])
    assert info.s_min == np.float32(ref1.s_min) and info.s_max == np.float32(ref1.s_max)
    assert info.total_weight == ref1.total
    assert info.n_unexplored == int((~pair.explored).sum()) + 1


def test_c1_twenty_steps_six_draws_each():
    """Alg. 1 with its default n = 5: n + 1 weighted draws per scoring pass,
    the fastest (here: first) pick profiled next."""
    spec = synth.space_c1()
    pair = Pair(spec, synth.forest_c1(spec))
    g = synth.rng(1, 4)
    U = synth.uniforms_u64(g, 1 + 20 * 6)
    deltas = synth.deltas(g, 20, 12)
    ref, _ = pair.step(None, np.zeros(12, np.float32), [U[0]])
    prof = ref.picks[0]
    for i in range(20):
        ref, _ = pair.step(prof, deltas[i], U[1 + 6 * i: 7 + 6 * i], check_scores=(i % 5 == 0))
        prof = ref.picks[0]
    ex = bits_to_bool(pair.sess.copy_explored(), len(pair.prep.valid))
    assert (ex == pair.explored).all()


def test_zero_delta_is_uniform():
    spec = synth.space_c1()
    pair = Pair(spec, synth.forest_c1(spec))
    U = synth.uniforms_u64(synth.rng(1, 5), 8)
    pair.step(None, np.zeros(12, np.float32), U[:1])
    # a profiled configuration but no bottleneck: still uniform, profile excluded
    ref, info = pair.step(5, np.zeros(12, np.float32), U[1:])
    assert info.n_active == 0
    un = ~pair.explored
    for l in ref.picks:
        un[l] = True
    assert (ref.q[un] == 1 << 23).all() and (ref.q[~un] == 0).all()


def test_exhaustion_and_single_remaining():
    """Tiny space: draws until nothing is left; the last unexplored
    configuration is always the pick; then CGS_EEMPTY."""
    spec = synth.Space([3, 2], [[1, 2, 4], [1, 2]], [("DIV", 0, 1, 0, 0)])
    forest = synth.random_forest(synth.rng(60), spec.radix, 2, 2, 3)
    pair = Pair(spec, forest)
    n = len(pair.prep.valid)
    U = synth.uniforms_u64(synth.rng(61), n + 2)
    d = synth.deltas(synth.rng(62), 1, 3)[0]
    ref, _ = pair.step(None, np.zeros(3, np.float32), U[:1])
    ref, _ = pair.step(ref.picks[0], d, U[1:])
    assert ref.picks[-1] is None and ref.picks[-2] is not None
    assert pair.sess.sample_next(123) is None


def test_sample_before_step_is_a_state_error():
    m = cgs()
    spec = synth.space_c1()
    sp = m.Space.from_spec(spec)
    sess = m.Session(sp)
    with pytest.raises(m.CgsError) as ei:
        sess.sample_next(1)
    assert ei.value.status == m.ESTATE


def test_measured_counters_path_matches_oracle_expert_system():
    """dPC from measured Table 1 counters through the library's expert system
    equals the oracle's (24-counter model)."""
    m = cgs()
    spec = synth.space_c1()
    forest = synth.random_forest(synth.rng(70), spec.radix, 4, 6, 24)
    pair = Pair(spec, forest)
    pcs = synth.profiler_counters(synth.rng(71), 3)
    thr = synth.threads_launched(synth.rng(72), 3)
    U = synth.uniforms_u64(synth.rng(73), 4)
    ref, _ = pair.step(None, np.zeros(24, np.float32), U[:1])
    prof = ref.picks[0]
    for i in range(3):
        ep = m.cgs_expert_params(inst_reaction=0.7, volta=0, reserved=0, cores=1920.0,
                                 threads=float(thr[i]))
        _, _, d32, _ = E.expert_system(pcs[i], False, 1920.0, float(thr[i]), 0.7)
        pair.sess.search_step(pair.model, int(pair.prep.valid[prof]), measured=pcs[i], expert=ep)
        ref = SR.step(pair.prep, pair.explored, prof, d32, [U[1 + i]])
        assert (pair.sess.copy_scores()[~pair.explored] == ref.s32[~pair.explored]).all()
        r = pair.sess.sample_next(int(U[1 + i]))
        assert r[1] == ref.picks[0]
        prof = ref.picks[0]


@pytest.mark.parametrize("block_log2", [12, 16])
def test_block_size_and_ragged_tail(block_log2):
    """Explicit 2^12- and 2^16-configuration weight blocks (4 and 64 weights
    per draw thread) over a space whose valid count (498,750) is neither a
    multiple of the block nor of 4."""
    m = cgs()
    spec = synth.space_batch(63)
    forest = synth.random_forest(synth.rng(63, 2), spec.radix, 4, 8, 6)
    p = m.cgs_default_params()
    p.block_log2 = block_log2
    pair = Pair(spec, forest, p)
    n = len(pair.prep.valid)
    assert n % 4096 != 0 and n % 4 != 0
    g = synth.rng(1, 6)
    U = synth.uniforms_u64(g, 5)
    ref, _ = pair.step(None, np.zeros(6, np.float32), U[:1])
    ref, _ = pair.step(ref.picks[0], synth.deltas(g, 1, 6)[0], U[1:])


def test_sampled_timing_counts_and_leaves_picks_unchanged():
    """timing = 3 times launched steps 0, 3, 6, 9 (and their further draws;
    the score pass of step 0, the uniform start, is not a scored pass); the
    picks stay those of the oracle."""
    m = cgs()
    spec = synth.space_c1()
    p = m.cgs_default_params()
    p.timing = 3
    pair = Pair(spec, synth.forest_c1(spec), p)
    g = synth.rng(1, 7)
    U = synth.uniforms_u64(g, 1 + 9 * 2)
    deltas = synth.deltas(g, 9, 12)
    ref, _ = pair.step(None, np.zeros(12, np.float32), [U[0]], check_scores=False)
    for i in range(9):
        ref, info = pair.step(ref.picks[0], deltas[i], U[1 + 2 * i: 3 + 2 * i], check_scores=False)
    ms, n = pair.sess.kernel_times()
    # the uniform start's score pass reads no prediction and is not counted
    assert n.tolist() == [3, 4, 1 + 3 * 2, 0]
    assert (ms[:3] > 0).all()
    assert info.device_ms > 0        # step 9 is timed
    # no timing: zeros
    plain = Pair(spec, synth.forest_c1(spec))
    plain.step(None, np.zeros(12, np.float32), [U[0]], check_scores=False)
    ms, n = plain.sess.kernel_times()
    assert n.tolist() == [0, 0, 0, 0] and plain.sess.step_info().device_ms == 0.0
