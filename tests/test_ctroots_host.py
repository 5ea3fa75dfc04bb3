"""Host check of the compile-time roots of unity that the radix-29 and -31
stages of the mixed-radix passes use (qva_ctroots.h): every W_R^j of the
radices 2..31 within 3 ulp of long-double cos and sin (the angle is rounded
twice before the series), and the constexpr table equal to the function."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_compile_time_roots(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "ctroots_host")
    subprocess.run([cxx, "-std=c++17", "-O2", "-I", os.path.join(ROOT, "paper_2110_03963_amd", "csrc"),
                    os.path.join(ROOT, "tests", "ctroots_host.cpp"), "-o", exe], check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    worst_ulps, table = float(out[0]), float(out[1])
    assert worst_ulps <= 3.0, worst_ulps
    assert table == 0.0
