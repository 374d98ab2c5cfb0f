"""The C-ABI library: loads, exports every declared symbol, validates
arguments on the host, and its host-side expert system equals the oracle
bit for bit.  No GPU work is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle import expert as E

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cgs.h")


def _cgs():
    from paper_2102_05297_amd import cgs
    return cgs


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cgs_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    cgs = _cgs()
    lib = ctypes.CDLL(cgs.library_path())
    names = declared_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(cgs.EXPORTS) == names


def test_version_and_defaults():
    cgs = _cgs()
    assert cgs.cgs_version() >= 1
    p = cgs.cgs_default_params()
    assert p.gamma == np.float32(-0.25) and p.w_min == np.float32(1e-4) and p.block_log2 == 0
    e = cgs.cgs_default_expert_params()
    assert e.inst_reaction == 0.7 and e.volta == 0


def test_host_argument_validation():
    cgs = _cgs()
    with pytest.raises(cgs.CgsError) as ei:
        cgs.Space([], [], [])
    assert ei.value.status == cgs.ERANGE
    with pytest.raises(cgs.CgsError) as ei:
        cgs.Space([17], [list(range(17))], [])
    assert ei.value.status == cgs.ERANGE
    with pytest.raises(cgs.CgsError) as ei:
        cgs.Space([3], [[1, 1, 2]], [])
    assert ei.value.status == cgs.EINVAL
    with pytest.raises(cgs.CgsError) as ei:
        cgs.Space([2], [[0, 1 << 20]], [])
    assert ei.value.status == cgs.ERANGE
    with pytest.raises(cgs.CgsError) as ei:
        cgs.Space([16] * 8 + [2], [list(range(16))] * 8 + [[0, 1]], [])
    assert ei.value.status == cgs.ERANGE          # 2^33 raw configurations
    with pytest.raises(cgs.CgsError) as ei:
        cgs.Space([2, 2], [[0, 1], [0, 1]], [("DIV", 0, 2, 0, 0)])
    assert ei.value.status == cgs.EINVAL
    with pytest.raises(cgs.CgsError) as ei:
        cgs.Space([2, 2], [[0, 1], [0, 1]], [(9, 0, 1, 0, 0)])
    assert ei.value.status == cgs.EINVAL


def _cases():
    pcs = synth.profiler_counters(synth.rng(901), 300)
    thr = synth.threads_launched(synth.rng(902), 300)
    return pcs, thr


def test_expert_system_matches_oracle_bit_for_bit():
    cgs = _cgs()
    pcs, thr = _cases()
    for i in range(len(pcs)):
        for volta in (0, 1):
            for ir in (0.7, 0.5):
                ep = cgs.cgs_expert_params(inst_reaction=ir, volta=volta, reserved=0,
                                           cores=1920.0, threads=float(thr[i]))
                B, d, dt = cgs.cgs_expert_system(pcs[i], ep)
                oB, od, _, odt = E.expert_system(pcs[i], bool(volta), 1920.0, float(thr[i]), ir)
                assert (B == oB).all(), (i, B, oB)
                assert (d == od).all(), (i, d, od)
                assert dt == odt


def test_expert_system_hand_cases_through_the_library():
    import json
    cgs = _cgs()
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "expert_hand_computed.json")))
    for case in g["cases"]:
        pc = np.zeros(24)
        for k, v in case["pc"].items():
            pc[g["counters"].index(k)] = v
        ep = cgs.cgs_expert_params(inst_reaction=case["inst_reaction"], volta=int(case["volta"]),
                                   reserved=0, cores=float(case["cores"]),
                                   threads=float(case["threads"]))
        B, d, dt = cgs.cgs_expert_system(pc, ep)
        for k, v in case["delta"].items():
            assert abs(d[g["counters"].index(k)] - v) < 1e-12
        for k, v in case["B"].items():
            assert abs(B[g["bottlenecks"].index(k)] - v) < 1e-12
        assert abs(dt - case["delta_threads"]) < 1e-12


def test_expert_system_rejects_bad_input():
    cgs = _cgs()
    pc = np.zeros(24)
    pc[3] = np.nan
    with pytest.raises(cgs.CgsError) as ei:
        cgs.cgs_expert_system(pc)
    assert ei.value.status == cgs.EINVAL
