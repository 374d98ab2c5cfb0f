"""The sampler entry point that allocates no device memory
(cgs_sample_weights_noalloc): on two calls in a row, the second smaller, its
picks equal those of cgs_sample_weights and the oracle's draws with removal
(Alg. 1) on the same weights and uniforms, bit for bit; sizes above its
limit are refused before any device work."""
import numpy as np
import pytest

import synth
from oracle import sampling as S
from tests.helpers import cgs

pytestmark = pytest.mark.gpu

LIMIT = 1 << 22


def _weights(n, seed):
    g = np.random.default_rng(seed)
    q = g.integers(0, 1 << 31, n, dtype=np.uint64)
    q[g.random(n) < 0.3] = 0
    q[-1] = max(q[-1], 1)
    return q


def _oracle(q, U):
    ref = S.draws(q, [int(u) for u in U])
    return [-1 if r is None else r for r in ref] + [-1] * (len(U) - len(ref))


def test_two_calls_in_a_row_match_the_allocating_sampler_and_the_oracle():
    m = cgs()
    sp = m.Space([2], [[0, 1]], [])
    for n, seed in ((3_000_017, 1), (100_003, 2)):   # the second call is smaller
        q = _weights(n, seed)
        U = synth.uniforms_u64(synth.rng(90, seed), 40)
        U[:3] = [0, np.iinfo(np.uint64).max, 1 << 63]
        got = sp.sample_weights_noalloc(q.astype(np.uint32), U)
        assert got.tolist() == sp.sample_weights(q.astype(np.uint32), U).tolist()
        assert got.tolist() == _oracle(q, U)


def test_draws_until_empty_after_a_larger_call():
    """A small call after a large one reads none of the large call's leftovers:
    its picks run out exactly when its weights do."""
    m = cgs()
    sp = m.Space([2], [[0, 1]], [])
    big = np.full(LIMIT, 7, np.uint32)                 # the largest size allowed
    U = synth.uniforms_u64(synth.rng(91), 4)
    assert sp.sample_weights_noalloc(big, U).tolist() == _oracle(big.astype(np.uint64), U)
    q = np.random.default_rng(3).integers(1, 1000, 50, dtype=np.uint64)
    q[::7] = 0
    U = synth.uniforms_u64(synth.rng(92), 60)
    got = sp.sample_weights_noalloc(q.astype(np.uint32), U)
    assert got.tolist() == _oracle(q, U)
    assert got.tolist() == sp.sample_weights(q.astype(np.uint32), U).tolist()


def test_sizes_and_arguments():
    m = cgs()
    sp = m.Space([2], [[0, 1]], [])
    with pytest.raises(m.CgsError) as ei:
        sp.sample_weights_noalloc(np.ones(LIMIT + 1, np.uint32), [5])
    assert ei.value.status == m.ERANGE
    assert sp.sample_weights_noalloc(np.zeros(0, np.uint32), [1, 2]).tolist() == [-1, -1]
    assert sp.sample_weights_noalloc(np.zeros(9, np.uint32), [1]).tolist() == [-1]
