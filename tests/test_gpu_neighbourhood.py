"""GPU neighbourhood-restricted steps vs the oracle (Sect. 3.7, footnote to
the scoring line of Alg. 1): candidates, scores, quantised weights, totals
and picks bit-exact."""
import numpy as np
import pytest

import synth
from oracle import neighbourhood as NB
from oracle import search as SR
from tests.helpers import bits_to_bool, cgs

pytestmark = pytest.mark.gpu


class NbPair:
    """The same search (full and restricted steps) on the GPU and on the
    oracle."""

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

    def start(self, U):
        self.sess.search_step(self.model, self.m.NO_PROFILE)
        ref = SR.step(self.prep, self.explored, None, np.zeros(self.model.n_counters, np.float32),
                      [U], with_fp64=False)
        assert self.sess.sample_next(int(U))[1] == ref.picks[0]
        return ref.picks[0]

    def nb_step(self, profile_l, delta, uniforms, radius, check=True):
        raw = int(self.prep.valid[profile_l])
        self.sess.search_step_neighbourhood(self.model, raw, radius, delta=delta)
        ref = NB.step(self.prep, self.spec.radix, self.explored, profile_l, delta, uniforms, radius)
        if check:
            idx, sc, q = self.sess.copy_neighbourhood()
            assert idx.tolist() == ref.cand.tolist()
            assert (sc == ref.s32).all()
            assert (q.astype(np.uint64) == ref.q).all()
            info = self.sess.step_info()
            assert info.n_unexplored == len(ref.cand)
            if len(ref.cand):
                assert info.s_min == np.float32(ref.s_min) and info.s_max == np.float32(ref.s_max)
        picks = []
        for U in uniforms:
            r = self.sess.sample_next(int(U))
            picks.append(None if r is None else r[1])
            if r is not None:
                assert r[0] == self.prep.valid[r[1]]
        ref_picks = list(ref.picks) + [None] * (len(picks) - len(ref.picks))
        assert picks == ref_picks, (picks, ref.picks)
        return ref

    def check_explored(self):
        ex = bits_to_bool(self.sess.copy_explored(), len(self.prep.valid))
        assert (ex == self.explored).all()


def test_c1_restricted_steps_all_radii():
    """The 30,720-configuration space: a uniform start, then 12 restricted
    steps (radius 1, 2, 3 in turn, 3 draws each, the first pick profiled
    next)."""
    spec = synth.space_c1()
    pair = NbPair(spec, synth.forest_c1(spec))
    g = synth.rng(1, 8)
    U = synth.uniforms_u64(g, 1 + 12 * 3)
    deltas = synth.deltas(g, 12, 12)
    prof = pair.start(U[0])
    for i in range(12):
        ref = pair.nb_step(prof, deltas[i], U[1 + 3 * i: 4 + 3 * i], 1 + i % 3)
        prof = next((p for p in ref.picks if p is not None), prof)
    pair.check_explored()


def test_restricted_then_full_steps_interleave():
    """Full and restricted steps share the explored set; a full step after
    restricted ones is the oracle's full step."""
    spec = synth.space_c1()
    pair = NbPair(spec, synth.forest_c1(spec))
    g = synth.rng(1, 9)
    U = synth.uniforms_u64(g, 20)
    deltas = synth.deltas(g, 6, 12)
    prof = pair.start(U[0])
    for i in range(3):
        ref = pair.nb_step(prof, deltas[i], U[1 + 2 * i: 3 + 2 * i], 2)
        prof = ref.picks[0]
        pair.sess.search_step(pair.model, int(pair.prep.valid[prof]), delta=deltas[3 + i])
        rf = SR.step(pair.prep, pair.explored, prof, deltas[3 + i], [U[10 + i]], with_fp64=False)
        s = pair.sess.copy_scores()
        un = ~pair.explored
        un[rf.picks[0]] = True
        assert (s[un] == rf.s32[un]).all()
        assert pair.sess.sample_next(int(U[10 + i]))[1] == rf.picks[0]
        prof = rf.picks[0]
    pair.check_explored()


def test_ragged_space_radius_two():
    """A 498,750-configuration space (8-14 parameters, constraints): radius-2
    steps with 4 draws each."""
    spec = synth.space_batch(63)
    forest = synth.random_forest(synth.rng(63, 2), spec.radix, 4, 8, 6)
    pair = NbPair(spec, forest)
    g = synth.rng(1, 10)
    U = synth.uniforms_u64(g, 1 + 6 * 4)
    deltas = synth.deltas(g, 6, 6)
    prof = pair.start(U[0])
    for i in range(6):
        ref = pair.nb_step(prof, deltas[i], U[1 + 4 * i: 5 + 4 * i], 2)
        prof = ref.picks[0]
    pair.check_explored()


def test_exhausting_a_neighbourhood():
    """Radius 1 around one profile: draw until nothing is left (the last
    draw answers empty), then a new restricted step on it has no candidate."""
    spec = synth.space_c1()
    pair = NbPair(spec, synth.forest_c1(spec))
    U = synth.uniforms_u64(synth.rng(1, 11), 60)
    prof = pair.start(U[0])
    d = synth.deltas(synth.rng(1, 12), 1, 12)[0]
    ref = pair.nb_step(prof, d, U[1:40], 1)
    assert ref.picks[-1] is None
    ref = pair.nb_step(prof, d, U[40:42], 1)
    assert len(ref.cand) == 0 and pair.sess.sample_next(5) is None
    pair.check_explored()


def test_restricted_step_errors():
    m = cgs()
    spec = synth.space_c1()
    sp = m.Space.from_spec(spec)
    model = m.ForestModel.from_spec(sp, synth.forest_c1(spec))
    sess = m.Session(sp)
    raw = int(sp.copy_valid()[0])
    d = np.zeros(12, np.float32)
    for radius in (0, 4):
        with pytest.raises(m.CgsError) as ei:
            sess.search_step_neighbourhood(model, raw, radius, delta=d)
        assert ei.value.status == m.EINVAL
    with pytest.raises(m.CgsError) as ei:
        sess.search_step_neighbourhood(model, m.NO_PROFILE, 1, delta=d)
    assert ei.value.status == m.EINVAL
    sess.search_step_neighbourhood(model, raw, 1, delta=d)
    with pytest.raises(m.CgsError) as ei:
        sess.copy_scores()
    assert ei.value.status == m.ESTATE
    # six parameters of 16 values: 70,965 neighbours at radius 3, too many
    big = m.Space([16] * 6, [list(range(16))] * 6, [])
    bm = m.ForestModel.from_spec(big, synth.random_forest(synth.rng(94), [16] * 6, 1, 2, 2))
    bs = m.Session(big)
    bs.search_step_neighbourhood(bm, 12345, 2, delta=np.zeros(2, np.float32))
    with pytest.raises(m.CgsError) as ei:
        bs.search_step_neighbourhood(bm, 12345, 3, delta=np.zeros(2, np.float32))
    assert ei.value.status == m.ERANGE
    # a single one-valued parameter: empty neighbourhood
    one = m.Space([1], [[3]], [])
    om = m.ForestModel(one, np.zeros((1, 0), np.uint8), np.zeros((1, 0), np.uint8),
                       np.ones((1, 1, 2), np.float32))
    with pytest.raises(m.CgsError) as ei:
        m.Session(one).search_step_neighbourhood(om, 0, 1, delta=np.zeros(2, np.float32))
    assert ei.value.status == m.EEMPTY


def test_restricted_steps_are_timed_in_their_own_slot():
    m = cgs()
    spec = synth.space_c1()
    p = m.cgs_default_params()
    p.timing = 1
    pair = NbPair(spec, synth.forest_c1(spec), p)
    U = synth.uniforms_u64(synth.rng(1, 13), 8)
    prof = pair.start(U[0])
    d = synth.deltas(synth.rng(1, 14), 1, 12)[0]
    pair.nb_step(prof, d, U[1:3], 2, check=False)
    ms, n = pair.sess.kernel_times()
    # the uniform start's score pass reads no prediction and is not counted;
    # its weight pass and draw are
    assert n.tolist() == [0, 1, 3, 1] and ms[3] > 0
