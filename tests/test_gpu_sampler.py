"""The device scan + inverse-CDF search on caller-given integer weights vs
the oracle's draw rule (Sect. 3.7, Alg. 1), bit-exact."""
import numpy as np
import pytest

import synth
from oracle import sampling as S
from tests.helpers import cgs

pytestmark = pytest.mark.gpu


def _space():
    m = cgs()
    return m, m.Space([2], [[0, 1]], [])


@pytest.mark.parametrize("n", [1, 7, 4096, 4097, 100003])
def test_single_draws_bit_exact(n):
    m, sp = _space()
    g = np.random.default_rng(n)
    q = g.integers(0, 1 << 31, n, dtype=np.uint64)
    q[g.random(n) < 0.3] = 0
    q[-1] = max(q[-1], 1)
    U = synth.uniforms_u64(synth.rng(80, n), 300)
    U[:3] = [0, np.iinfo(np.uint64).max, 1 << 63]
    for u in U:
        got = sp.sample_weights(q.astype(np.uint32), [u])[0]
        assert got == S.pick(q, int(u))


def test_draws_with_removal_until_empty():
    m, sp = _space()
    g = np.random.default_rng(3)
    q = g.integers(1, 1000, 50, dtype=np.uint64)
    q[::7] = 0
    U = synth.uniforms_u64(synth.rng(81), 60)
    got = sp.sample_weights(q.astype(np.uint32), U)
    ref = S.draws(q, [int(u) for u in U])
    ref = [-1 if r is None else r for r in ref] + [-1] * (60 - len(ref))
    assert got.tolist() == ref


def test_large_uniform_closed_form():
    """5M equal weights: the pick is floor(U * n / 2^64) (closed form)."""
    m, sp = _space()
    n = 5_000_000
    q = np.full(n, 1 << 23, dtype=np.uint32)
    for u in synth.uniforms_u64(synth.rng(82), 50):
        assert sp.sample_weights(q, [u])[0] == (int(u) * n) >> 64


def test_many_blocks_per_draw_thread():
    """20M weights: 4883 blocks of 4096, so each draw thread scans a run of 5
    block sums in two load rounds."""
    m, sp = _space()
    g = np.random.default_rng(5)
    n = 20_000_000
    q = g.integers(0, 1 << 31, n, dtype=np.uint64)
    q[g.random(n) < 0.5] = 0
    U = synth.uniforms_u64(synth.rng(83), 12)
    U[:2] = [0, np.iinfo(np.uint64).max]
    q32 = q.astype(np.uint32)
    for u in U:
        assert sp.sample_weights(q32, [u])[0] == S.pick(q, int(u))
