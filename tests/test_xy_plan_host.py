"""The parity-mixer planner (xy_layer_plan), compiled for the host.

For rings over all qubits, two interleaved rings (the two-position encoding of
the paper's portfolio example) and random pair lists at n = 2..33, every pair
must be applied exactly once, inside its pass's tile, at most kMaxXyOps per
pass, and after every earlier pair sharing a qubit with it (the factors that
do not commute keep their order).
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def test_xy_planner_keeps_factor_order(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "xy_plan_host")
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "paper_2110_03963_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "xy_plan_host.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    words = out.stdout.split()
    assert words[0] == "ok" and int(words[1]) == 32 * 22
