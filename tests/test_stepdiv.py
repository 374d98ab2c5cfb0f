"""Host check of the fixed-divisor division used by the score
normalisation (paper_2102_05297_amd/csrc/stepdiv.h): bit-equal to IEEE
float32 division for every numerator significand with 160 divisor
significands (adversarial and random), both signs, two scales, and for
zeros, tiny, huge and non-finite operands (tests/stepdiv_check.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_fixed_divisor_division_is_correctly_rounded(tmp_path):
    exe = str(tmp_path / "stepdiv_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-pthread",
                    "-I" + os.path.join(ROOT, "paper_2102_05297_amd", "csrc"),
                    os.path.join(ROOT, "tests", "stepdiv_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe, "64"], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "mismatches 0" in r.stdout, r.stdout
