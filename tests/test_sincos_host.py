"""Accuracy of the kernels' sin/cos (series after reduction by quarter turns).

The same source the kernels inline is compiled for the host with hipcc and
compared with long double sinl/cosl on uniform arguments up to 1e12 and on
arguments next to multiples of pi/2.  Bound: 1.6e-16 absolute on sin, cos
and exp(-i x) (the phase factor's error as a complex number), and exact
results for 0 and tiny arguments.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def report(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("sincos") / "sincos_host")
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "paper_2110_03963_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "sincos_host.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    rows = {}
    for line in out.strip().splitlines():
        name, cnt, es, ec, ee = line.split()
        rows[name] = (int(cnt), float(es), float(ec), float(ee))
    return rows


def test_uniform_ranges(report):
    for span in ["1", "4", "100", "10000", "1e+07", "1e+10", "1e+12"]:
        cnt, es, ec, ee = report[f"uniform_{span}"]
        assert cnt == 400000
        assert es <= 1.6e-16 and ec <= 1.6e-16 and ee <= 1.6e-16, (span, es, ec, ee)


def test_near_quarter_turns(report):
    _, es, ec, ee = report["near_half_pi_multiples"]
    assert es <= 1.6e-16 and ec <= 1.6e-16 and ee <= 1.6e-16, (es, ec, ee)


def test_special_arguments(report):
    _, es, ec, ee = report["special"]
    assert es <= 1.6e-16 and ec <= 1.6e-16
