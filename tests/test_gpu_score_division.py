"""The score pass's division (Sect. 3.6 score equation, t = (x - a) / (a + x)
per counter) against the oracle's float32 chain, bit for bit, on adversarial
predictions: divisors a + x with all-ones significands, x == a, x one or a
few ulps from a, subnormal and zero x, x at 2^59 and above (the library
refuses negative and non-finite predictions), -0; and profiles whose a is
tiny (below 2^-36), huge (above 2^59) or zero."""
import numpy as np
import pytest

import synth
from oracle import search as SR
from oracle import space as SP
from tests.helpers import cgs

pytestmark = pytest.mark.gpu

RADIX = [16, 16, 16, 8]   # 32,768 valid configurations, no constraints
C = 24
P_IN, P_OUT = 5000, 20000  # profiles: every a in range / some a outside it


def _predictions():
    g = np.random.default_rng(2102)
    n = int(np.prod(RADIX))
    P = np.exp(g.uniform(np.log(1e-3), np.log(1e6), size=(n, C))).astype(np.float32)
    a_in = np.array([2.0 ** -36, 1.0, np.nextafter(np.float32(2.0), np.float32(0.0)), 2.0 ** 59,
                     3.0, 0.1, 1e-10, 1e10, 5e17, 0.75, 1.5, 2.0 ** -20] * 2, np.float32)
    P[P_IN] = a_in
    a_out = P[P_OUT].copy()
    a_out[3] = 1e-12          # below 2^-36
    a_out[11] = 1e18          # above 2^59
    a_out[17] = 0.0           # the counter is skipped
    P[P_OUT] = a_out
    # configurations 0 .. 8191: adversarial x against both profiles' a, all
    # within the sequence's range
    for l in range(8192):
        if l in (P_IN, P_OUT):
            continue
        for c in range(C):
            a = np.float32(P[P_IN, c] if l % 2 == 0 else P[P_OUT, c])
            kind = (l // 2 + 7 * c) % 8
            if kind == 0:
                x = a
            elif kind == 1:                      # a few ulps from a
                x = np.float32(a) + np.float32(((l % 9) - 4)) * np.spacing(np.float32(a))
            elif kind == 2:                      # a + x with an all-ones significand
                e = np.floor(np.log2(max(float(a), 1e-30))) + 1 + (l % 3)
                x = np.float32(np.float32((2.0 - 2.0 ** -23) * 2.0 ** e) - a)
            elif kind == 3:
                x = np.float32(1e-42)            # subnormal
            elif kind == 4:
                x = np.float32(0.0)
            elif kind == 5:
                x = np.float32(2.0 ** 59)
            elif kind == 6:
                x = np.float32(a) * np.float32(0.5)
            else:
                x = np.float32(a) * np.float32(2.0)
            P[l, c] = min(max(np.float32(x), np.float32(0.0)), np.float32(2.0 ** 59))
    # configurations 8192 .. 12287: out-of-range x scattered over waves
    for l in range(8192, 12288, 37):
        P[l, l % C] = [1e18, 6e17, -0.0, 3e38][l % 4]
    return P


def test_scores_equal_the_float32_chain_on_adversarial_predictions():
    m = cgs()
    spec = synth.Space(RADIX, [list(range(1, r + 1)) for r in RADIX], [])
    valid = SP.enumerate_valid(spec.radix, spec.values, spec.constraints)
    digits = SP.digits_of(valid, spec.radix)
    P = _predictions()
    prep = SR.Prepared(valid, digits, None, P.astype(np.float64), P)
    sp = m.Space.from_spec(spec)
    model = m.TableModel(sp, P)
    sess = m.Session(sp)
    explored = np.zeros(len(valid), dtype=bool)
    g = np.random.default_rng(5)
    U = synth.uniforms_u64(synth.rng(81), 3)
    sess.search_step(model, m.NO_PROFILE)
    SR.step(prep, explored, None, np.zeros(C, np.float32), [int(U[0])], with_fp64=False)
    sess.sample_next(int(U[0]))
    for i, prof in enumerate((P_IN, P_OUT)):
        delta = g.uniform(-1.0, 1.0, size=C).astype(np.float32)
        print(f"profile {prof}", flush=True)
        sess.search_step(model, int(valid[prof]), delta=delta)
        ref = SR.step(prep, explored, prof, delta, [int(U[i + 1])], with_fp64=False)
        at_scoring = explored.copy()
        for l in ref.picks:
            if l is not None:
                at_scoring[l] = False
        un = ~at_scoring
        s = sess.copy_scores()
        same = s[un].view(np.uint32) == ref.s32[un].view(np.uint32)
        both_nan = np.isnan(s[un]) & np.isnan(ref.s32[un])
        assert (same | both_nan).all(), np.flatnonzero(~(same | both_nan))[:10]
        q = sess.copy_weights()
        assert (q.astype(np.uint64) == ref.q).all()
        _, l = sess.sample_next(int(U[i + 1]))
        assert l == ref.picks[0]
