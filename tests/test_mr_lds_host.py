"""Host check of the mixed-radix planner's LDS padding choice (no GPU).

The low group's DFT stages run in LDS; when a power-of-two radix comes after
the odd radices (e.g. 3496 = 23 19 8 for N = C(26, 13)), its stage reads at a
stride of 8 elements and the lanes of a quarter-wave fall on the same banks.
The planner then pads the LDS slots (one element after every 16).  Checked
here: the choice for known factorisations, and that the cost model counts
the 8-way conflict of a stride-8 stage.
"""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("mrlds") / "mr_lds_host")
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "paper_2110_03963_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "mr_lds_host.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True)
    return out


def _run(exe, *Ns):
    res = subprocess.run([exe, *map(str, Ns)], capture_output=True, text=True, check=True)
    rows = {}
    for line in res.stdout.split("\n"):
        if line.strip():
            n, pad, c0, c1 = line.split()
            rows[int(n)] = (pad, int(c0), int(c1))
    return rows


def test_padding_choice(exe):
    rows = _run(exe, 10400600, 155117520, 460288, 11907000, 2704156, 6000, 3003, 30)
    # a power-of-two radix after larger odd ones: padded
    for N in (10400600, 155117520, 460288):
        assert rows[N][0] == "1", (N, rows[N])
        assert 3 * rows[N][2] <= 2 * rows[N][1]
    # odd radices last (lane strides coprime to 16): left unpadded
    for N in (11907000, 2704156, 6000, 3003, 30):
        assert rows[N][0] == "0", (N, rows[N])


def test_stride_eight_stage_cost(exe):
    """N = 8 * 23 * 19 * 7 = 24472 plans its low group of 3496 = 23 19 8 (the
    last stage reads 8 consecutive elements per lane: lane stride 8, two
    granules per quarter-wave, an 8-way conflict), padded; its padded cost is
    at most that of stages without conflicts."""
    rows = _run(exe, 24472)
    pad, c0, c1 = rows[24472]
    assert pad == "1"
    # stage costs without the conflict: 16-lane quarters at one lane per granule
    assert c1 < c0
