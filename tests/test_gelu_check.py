"""Host check of the perceptron kernels' GELU (paper_2102_05297_amd/csrc/gelu.h,
tests/gelu_check.cpp): its tail polynomial stays within the oracle's
TAIL_LOG2_ERR of log2 Phi(-x) on [0, 6] in float32 evaluation, and the whole
GELU within the oracle's per-value bound, against a long double
reference."""
import os
import shutil
import subprocess

import pytest

from oracle import mlp as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_gelu_tail_within_the_oracle_bound(tmp_path):
    exe = str(tmp_path / "gelu_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-pthread",
                    "-I" + os.path.join(ROOT, "paper_2102_05297_amd", "csrc"),
                    os.path.join(ROOT, "tests", "gelu_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout
    # the bound the check asserts is the one the oracle's intervals assume
    assert f"(bound {M.TAIL_LOG2_ERR:.3e})" in r.stdout, r.stdout
