"""GPU enumeration + constraint pruning vs the oracle: bit-exact masks and
valid lists (Sect. 1; TS of Alg. 1)."""
import hashlib

import numpy as np
import pytest

import synth
from oracle import space as SP
from tests.helpers import bits_to_bool, cgs, golden, random_small_space

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed", range(40))
def test_random_small_spaces_bit_exact(seed):
    m = cgs()
    g = np.random.default_rng(1000 + seed)
    radix, values, cons = random_small_space(g)
    sp = m.Space(radix, values, cons)
    brute = SP.enumerate_bruteforce(radix, values, cons)
    assert sp.n_raw == int(np.prod(radix))
    assert sp.n_valid == len(brute)
    assert sp.copy_valid().tolist() == brute
    mask = bits_to_bool(sp.copy_mask(), sp.n_raw)
    assert np.flatnonzero(mask).tolist() == brute


def test_c1_full():
    m = cgs()
    spec = synth.space_c1()
    sp = m.Space.from_spec(spec)
    ref_mask = SP.valid_mask(spec.radix, spec.values, spec.constraints)
    assert (sp.copy_mask() == SP.mask_words(ref_mask)).all()
    assert (sp.copy_valid() == np.flatnonzero(ref_mask)).all()


@pytest.mark.parametrize("name", ["c2", "c5"] + [f"batch{s}" for s in (0, 7, 21, 40, 63)])
def test_full_size_against_stored_oracle_hash(name):
    m = cgs()
    spec = {"c2": synth.space_c2, "c5": synth.space_c5}.get(name)
    spec = spec() if spec else synth.space_batch(int(name[5:]))
    ref = golden("space_counts.json")[name]
    sp = m.Space.from_spec(spec)
    assert sp.n_raw == ref["n_raw"] and sp.n_valid == ref["n_valid"]
    v = sp.copy_valid()
    assert hashlib.sha256(v.astype("<u4").tobytes()).hexdigest() == ref["sha256_valid_u32le"]
    # the bitmask agrees with the list
    words = sp.copy_mask()
    assert int(np.unpackbits(words.view(np.uint8)).sum()) == sp.n_valid


def test_no_constraints_all_valid_and_radix_one():
    m = cgs()
    sp = m.Space([3, 1, 5, 1], [[1, 2, 3], [7], [0, 1, 2, 3, 4], [-2]], [])
    assert sp.n_raw == 15 and sp.n_valid == 15
    assert sp.copy_valid().tolist() == list(range(15))


def test_empty_space():
    m = cgs()
    sp = m.Space([4, 4], [[1, 2, 4, 8], [1, 2, 4, 8]], [("PROD_LE", 0, 1, 0, 0)])
    assert sp.n_valid == 0
    sess = m.Session(sp)
    model = m.ForestModel(sp, np.zeros((1, 1), np.uint8), np.zeros((1, 1), np.uint8),
                          np.ones((1, 2, 3), np.float32))
    with pytest.raises(m.CgsError) as ei:
        sess.search_step(model, m.NO_PROFILE)
    assert ei.value.status == m.EEMPTY


def test_monotone_chain_over_31_binary_parameters():
    """2^31 raw configurations; LE(v_j, v_{j+1}) for all j keeps exactly the 32
    non-decreasing 0/1 sequences 0..01..1 (closed form)."""
    m = cgs()
    n = 31
    cons = [("LE", j, j + 1, 0, 0) for j in range(n - 1)]
    sp = m.Space([2] * n, [[0, 1]] * n, cons[:32])
    assert len(cons) <= 32
    expect = sorted((1 << t) - 1 for t in range(n + 1))   # t trailing ones
    assert sp.n_raw == 1 << 31 and sp.n_valid == 32
    assert sp.copy_valid().tolist() == expect


def test_near_2_32_raw_configurations():
    """15 * 16^7 = 4,026,531,840 raw configurations; v_1 .. v_6 forced to 0 by
    v_j * v_j <= 0 leaves the 15 * 16 configurations k = d0 * 16^7 + d7."""
    m = cgs()
    radix = [15] + [16] * 7
    values = [list(range(1, 16))] + [list(range(16))] * 7
    cons = [("PROD_LE", j, j, 0, 0) for j in range(1, 7)]
    sp = m.Space(radix, values, cons)
    assert sp.n_raw == 15 * 16 ** 7
    expect = sorted(d0 * 16 ** 7 + d7 for d0 in range(15) for d7 in range(16))
    assert sp.copy_valid().tolist() == expect
    assert int(np.unpackbits(sp.copy_mask().view(np.uint8)).sum()) == 240


def test_host_decode_and_valid_index():
    m = cgs()
    spec = synth.space_c1()
    sp = m.Space.from_spec(spec)
    v = sp.copy_valid()
    for k in [0, 1, 777, spec.n_raw - 1] + v[::997].tolist():
        assert sp.decode(k).tolist() == SP.decode(int(k), spec.radix)
    for l in range(0, len(v), 991):
        assert sp.valid_index(int(v[l])) == l
    invalid = sorted(set(range(spec.n_raw)) - set(v.tolist()))[:5]
    for k in invalid:
        assert sp.valid_index(k) == -1
