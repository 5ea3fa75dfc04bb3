"""Host check of bench.py's HBM-traffic bookkeeping (no GPU): counter values
from synthetic rocprofv3 CSVs are matched to plan launches in dispatch order,
scaled by the calibration copy, averaged per kernel label, and a launch that
meets a kernel of the wrong family is an error."""

import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

CALIB_KIB = bench.CALIB_ELEMS * 8 / 1024.0


def _csv(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "pmc_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, ["Agent_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, value) in enumerate(rows):
            w.writerow({"Agent_Id": "Agent 1", "Dispatch_Id": i + 1, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": value})


def _plan(path):
    seg = {"workload": "w", "call": "grad", "N": 1024, "runs": 2, "launches": [
        {"label": "xpass_kernel<4, XMODE_FIRST>", "kind": 1, "dispatches": 1, "bytes": 24 * 1024},
        {"label": "grad_dif<5>", "kind": 22, "dispatches": 2, "bytes": 64 * 1024},
        {"label": "grad_reduce", "kind": 25, "dispatches": 2, "bytes": 100.0}]}
    with open(path, "w") as fh:
        json.dump({"segments": [seg]}, fh)


XP = "void qva::(anonymous namespace)::xpass_kernel<4, 71>(qva::XPassParams)"
FP = "void qva::(anonymous namespace)::fftpass_kernel<5, 32>(qva::FftPassParams)"
SR = "qva::(anonymous namespace)::slot_reduce_kernel(double const*, long, double*)"
GF = "qva::(anonymous namespace)::grad_finalize_kernel(double const*, int, int, int, double*, double*)"
COPY = "__amd_rocclr_copyBuffer"


def test_write_traffic_matches_launches(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "t.json"))
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(tmp_path / "t.md"))
    run = [(XP, 8.0), (FP, 16.0), (FP, 16.0), (SR, 0.5), (GF, 0.25)]
    # the copy reads half its bytes on FETCH (scale 2) and all on WRITE (scale 1)
    _csv(str(tmp_path / "f"), "FETCH_SIZE", [(COPY, CALIB_KIB / 2), ("torch_fill", 99.0)] + run + run)
    _csv(str(tmp_path / "w"), "WRITE_SIZE", [(COPY, CALIB_KIB), ("torch_fill", 99.0)] + run + run)
    _plan(str(tmp_path / "plan.json"))
    assert bench.write_traffic(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "plan.json")) == 0
    data = json.load(open(tmp_path / "t.json"))
    k = data["workloads"][0]["kernels"]
    assert k["xpass_kernel<4, XMODE_FIRST>"]["fetch_bytes"] == 8 * 1024 * 2
    assert k["xpass_kernel<4, XMODE_FIRST>"]["write_bytes"] == 8 * 1024
    assert k["grad_dif<5>"]["bytes_per_launch"] == (2 * 16 * 2 + 2 * 16) * 1024
    assert k["grad_dif<5>"]["launches_per_call"] == 1
    assert k["grad_reduce"]["fetch_bytes"] == round((0.5 + 0.25) * 1024 * 2)
    assert data["calibration"]["fetch_scale"] == 2.0 and data["calibration"]["write_scale"] == 1.0
    assert os.path.exists(tmp_path / "t.md")


def test_write_traffic_rejects_misaligned_dispatches(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "t.json"))
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(tmp_path / "t.md"))
    run = [(FP, 8.0), (FP, 16.0), (FP, 16.0), (SR, 0.5), (GF, 0.25)]  # first launch is not an xpass
    _csv(str(tmp_path / "f"), "FETCH_SIZE", [(COPY, CALIB_KIB)] + run + run)
    _csv(str(tmp_path / "w"), "WRITE_SIZE", [(COPY, CALIB_KIB)] + run + run)
    _plan(str(tmp_path / "plan.json"))
    with pytest.raises(RuntimeError, match="met dispatch"):
        bench.write_traffic(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "plan.json"))
    _csv(str(tmp_path / "f"), "FETCH_SIZE", [(COPY, CALIB_KIB)] + run)
    with pytest.raises(RuntimeError, match="count mismatch"):
        bench.write_traffic(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "plan.json"))
