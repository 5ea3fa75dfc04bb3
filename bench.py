"""Benchmark of the QVA state-evolution hot path on one MI355X.

A step is one fused evolution of the QAOA MaxCut workload (n = 28 qubits,
2^28 complex128 amplitudes, random 3-regular graph with weights ~ U(0,1),
p = 8 layers): psi_0, p x (phase + hypercube mixer), <Q>.  Inputs are seeded
synthetic data resident in HBM before the timed region.

Prints one JSON line: layer-applications/s, the roofline of the dominant
kernel (per-launch HIP events over the timed steps), the CPU oracle timed on
a bounded sample (rank 0, N = 1 only), and secondary measurements of the
other workloads (QWOA circulant mixer, adjoint gradient vs finite
differences) under "extras".

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-extras]
"""

from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "layer-applications/s and HBM GB/s vs peak; adjoint gradients/s vs finite-diff"
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "xpass_traffic_qaoa_n28.json")
CSRC = os.path.join(ROOT, "paper_2110_03963_amd", "csrc")
# Sources the hypercube-mixer passes are built and launched from: a stored
# traffic measurement holds only while these are unchanged.
TRAFFIC_SOURCES = [os.path.join(CSRC, f) for f in
                   ("qva_xmix.hip", "qva_tile.h", "qva_passes.h", "qva_device.h", "qva_internal.h",
                    "qva_plan.h", "qva_api.hip")]
CALIB_ELEMS = 1 << 27  # calibration copy: 2^27 float64 = 1 GiB read + 1 GiB written


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class HipEvents:
    """hipEvent_t handles through the HIP runtime (timing-enabled)."""

    def __init__(self, count: int):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                 ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.ev = []
        for _ in range(count):
            h = ctypes.c_void_p()
            if self.hip.hipEventCreate(ctypes.byref(h)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.ev.append(h.value)
        self.array = (ctypes.c_void_p * count)(*self.ev)

    def slice(self, start: int):
        return ctypes.cast(ctypes.byref(self.array, ctypes.sizeof(ctypes.c_void_p) * start),
                           ctypes.POINTER(ctypes.c_void_p))

    def elapsed_ms(self, a: int, b: int) -> float:
        ms = ctypes.c_float()
        if self.hip.hipEventElapsedTime(ctypes.byref(ms), self.ev[a], self.ev[b]) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return ms.value

    def close(self):
        for h in self.ev:
            self.hip.hipEventDestroy(h)


MODE_NAMES = {1: "XMODE_FIRST", 2: "XMODE_MIDDLE", 3: "XMODE_BOUNDARY", 4: "XMODE_LAST",
              5: "XMODE_LAST_STORE"}
# xpass_kernel's second template argument (pass flag bits) per mode, as the
# profiler prints it.
XMODE_FLAGS = {"XMODE_FIRST": 71, "XMODE_MIDDLE": 68, "XMODE_BOUNDARY": 92, "XMODE_LAST": 164,
               "XMODE_LAST_STORE": 228, "XMODE_FIRST_Z": 327, "XMODE_BOUNDARY_Z": 348}


def kernel_name(kind: int, col_bits: int) -> str:
    from paper_2110_03963_amd import _lib

    if kind in MODE_NAMES:
        return f"xpass_kernel<{col_bits}, {MODE_NAMES[kind]}>"
    name = _lib.PASS_KINDS[kind]
    if name.startswith(("fft_", "grad_", "xy")) and name not in ("grad_reduce", "grad_whole"):
        return f"{name}<{col_bits}>"
    return name


def source_digest(*paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def plan_of(lib, prob, p: int, for_grad: bool, flags: int):
    from paper_2110_03963_amd import _lib

    n = lib.qva_plan(prob.cstruct(), p, int(for_grad), flags, None, 0)
    infos = (_lib.QvaPassInfo * n)()
    lib.qva_plan(prob.cstruct(), p, int(for_grad), flags, infos, n)
    return list(infos)


def per_kernel_profile(run_timed, infos, steps: int):
    """Run `steps` timed executions of a plan and aggregate the per-launch
    event durations by kernel."""
    import torch

    npl = len(infos)
    evs = HipEvents(2 * npl * steps)
    for s in range(steps):
        run_timed(evs.slice(2 * npl * s), 2 * npl)
    torch.cuda.synchronize()
    per: dict[str, dict] = {}
    for s in range(steps):
        for i, info in enumerate(infos):
            name = kernel_name(info.kind, info.col_bits)
            d = per.setdefault(name, {"launches": 0, "ms": 0.0, "bytes": 0.0})
            d["launches"] += 1
            d["ms"] += evs.elapsed_ms(2 * (s * npl + i), 2 * (s * npl + i) + 1)
            d["bytes"] += info.bytes
    evs.close()
    return per


def roofline_of(per: dict, steps: int) -> dict:
    name, d = max(per.items(), key=lambda kv: kv[1]["ms"])
    avg_ms = d["ms"] / d["launches"]
    bpl = d["bytes"] / d["launches"]
    achieved = bpl / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": name,
            "launches_per_step": d["launches"] // steps, "avg_launch_ms": round(avg_ms, 4),
            "algorithmic_bytes_per_launch": bpl}


def profiler_label(name: str) -> str | None:
    """Map a profiler kernel name to the names used here: xpass kernels to
    kernel_name()'s form, the runtime's device-to-device copy to "copy"."""
    import re

    if "copyBuffer" in name:
        return "copy"
    m = re.search(r"xpass_kernel<(\d+), (\d+)>", name)
    if m:
        flags = int(m.group(2))
        for mode, v in XMODE_FLAGS.items():
            if v == flags:
                return f"xpass_kernel<{m.group(1)}, {mode}>"
    for short in ("phase_kernel", "init_uniform_kernel"):
        if f"::{short}(" in name:
            return short
    return None


def read_counter_csv(folder: str, counter: str) -> dict:
    """Per-dispatch values of one counter from rocprofv3's counter_collection
    CSV(s) under `folder`: {label: [value, ...]} (values in the counter's
    unit, KiB for FETCH_SIZE / WRITE_SIZE)."""
    import csv
    import glob

    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {folder}")
    out: dict[str, list] = {}
    for fn in files:
        with open(fn, newline="") as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                label = profiler_label(row.get("Kernel_Name", ""))
                if label:
                    out.setdefault(label, []).append(float(row["Counter_Value"]))
    return out


VALU_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64")


def valu_summary(counter_dir: str, stats_csv: str) -> int:
    """Vector-ALU load of each kernel: per-dispatch means of the SQ_INSTS_VALU*
    counters (wave instructions, whole GPU) from a `rocprofv3 --pmc` run, with
    the kernel's average duration from a `--kernel-trace --stats` run of the
    same command.  FP64 flops = 64 lanes x (add + mul + 2 fma); the issue time
    of the VALU instructions is 4 cycles per wave instruction (16 lanes per
    SIMD) spread over 1024 SIMDs at 2.4 GHz; both are shown against the
    kernel's duration (FP64 vector peak 78.6 TFLOP/s)."""
    import csv
    import glob
    import re

    def key(name: str) -> str:
        m = re.search(r"(\w+_kernel<[^>]*>|\w+_kernel)\(", name.replace("(anonymous namespace)::", ""))
        return m.group(1) if m else name[:60]

    vals: dict = {}
    for fn in glob.glob(os.path.join(counter_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(fn, newline="") as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") in VALU_COUNTERS:
                    vals.setdefault(key(row["Kernel_Name"]), {}).setdefault(row["Counter_Name"], []).append(
                        float(row["Counter_Value"]))
    dur = {}
    with open(stats_csv, newline="") as fh:
        for row in csv.DictReader(fh):
            dur[key(row["Name"])] = float(row["AverageNs"]) * 1e-9
    rows = []
    for k, cs in vals.items():
        if k not in dur or "SQ_INSTS_VALU" not in cs:
            continue
        m = {c: sum(v) / len(v) for c, v in cs.items()}
        t = dur[k]
        flops = 64.0 * (m.get("SQ_INSTS_VALU_ADD_F64", 0) + m.get("SQ_INSTS_VALU_MUL_F64", 0)
                        + 2 * m.get("SQ_INSTS_VALU_FMA_F64", 0))
        issue = m["SQ_INSTS_VALU"] * 4 / (1024 * 2.4e9)
        rows.append({"kernel": k, "dispatches": len(cs["SQ_INSTS_VALU"]), "avg_ms": round(t * 1e3, 4),
                     "valu_wave_instructions": round(m["SQ_INSTS_VALU"]),
                     "fp64_tflops": round(flops / t / 1e12, 2), "fp64_frac_of_peak": round(flops / t / 78.6e12, 3),
                     "valu_issue_ms": round(issue * 1e3, 4), "valu_issue_frac": round(issue / t, 3)})
    rows.sort(key=lambda r: -r["avg_ms"] * r["dispatches"])
    print(json.dumps(rows, indent=1))
    return 0


def pmc_pass() -> int:
    """The program profiled by the two counter runs: one calibration copy of
    known size, one standalone phase (reads psi and q, writes psi), then two
    fused n = 28, p = 8 evolutions as in the timed step."""
    import torch

    import paper_2110_03963_amd as qva
    from paper_2110_03963_amd import _lib
    from workloads import CONFIG_SEEDS, maxcut_qualities_device, qaoa_maxcut_workload

    lib = qva.load_library()
    n, p = 28, 8
    wl = qaoa_maxcut_workload(n, p, graph="regular3", weighted=True, seed=CONFIG_SEEDS["qaoa_n28"],
                              build_q=False)
    src = torch.ones(CALIB_ELEMS, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    q = maxcut_qualities_device(n, wl.edges, wl.weights, "cuda")
    psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    qva.init_uniform(psi)
    qva.phase(psi, q, 0.3)
    prob = qva.Problem(q, "x")
    g = torch.tensor(wl.gammas, dtype=torch.float64, device="cuda")
    t = torch.tensor(wl.ts, dtype=torch.float64, device="cuda")
    ws = torch.empty(max(prob.workspace_bytes(p), 16), dtype=torch.uint8, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    for _ in range(2):
        _lib.check("qva_evolve", lib.qva_evolve(prob.cstruct(), g.data_ptr(), t.data_ptr(), p,
                                                psi.data_ptr(), out.data_ptr(), out.data_ptr() + 8,
                                                _lib.QVA_EVOLVE_SKIP_FINAL_STATE, ws.data_ptr(),
                                                ws.numel(), stream))
    torch.cuda.synchronize()
    log(f"pmc pass done: f={out[0].item():.15f}")
    return 0


def write_traffic(fetch_dir: str, write_dir: str) -> int:
    """Turn the FETCH_SIZE and WRITE_SIZE runs of pmc_pass into HBM bytes per
    launch of each xpass kernel, each counter scaled by what it reads on the
    calibration copy (known bytes), and store them with the sources' digest."""
    fetch = read_counter_csv(fetch_dir, "FETCH_SIZE")
    write = read_counter_csv(write_dir, "WRITE_SIZE")
    calib_kib = CALIB_ELEMS * 8 / 1024.0
    if "copy" not in fetch or "copy" not in write:
        raise RuntimeError("calibration copy not found in the counter runs")
    f_copy, w_copy = max(fetch["copy"]), max(write["copy"])
    ff, fw = calib_kib / f_copy, calib_kib / w_copy
    n = 28
    amps = 1 << n
    kernels = {}
    for label in sorted(set(fetch) & set(write)):
        if not label.startswith("xpass_kernel"):
            continue
        fb = sum(fetch[label]) / len(fetch[label]) * 1024 * ff
        wb = sum(write[label]) / len(write[label]) * 1024 * fw
        kernels[label] = {"fetch_bytes": round(fb), "write_bytes": round(wb),
                          "bytes_per_launch": round(fb + wb), "dispatches": len(fetch[label]),
                          "fetch_bytes_per_amplitude": round(fb / amps, 3),
                          "write_bytes_per_amplitude": round(wb / amps, 3)}
    check = {}
    if "phase_kernel" in fetch and "phase_kernel" in write:
        check = {"phase_kernel_fetch_bytes_per_amplitude":
                 round(max(fetch["phase_kernel"]) * 1024 * ff / amps, 3),
                 "phase_kernel_write_bytes_per_amplitude":
                 round(max(write["phase_kernel"]) * 1024 * fw / amps, 3),
                 "expected": "24 read (psi 16 + q 8), 16 written"}
    data = {"source_digest": source_digest(*TRAFFIC_SOURCES), "workload": "qaoa_maxcut_n28_p8",
            "calibration": {"kernel": "__amd_rocclr_copyBuffer", "bytes_each_way": CALIB_ELEMS * 8,
                            "fetch_kib_read": f_copy, "write_kib_read": w_copy,
                            "fetch_scale": ff, "write_scale": fw, **check},
            "commands": ["timeout -s KILL 150 rocprofv3 --pmc FETCH_SIZE --output-format csv "
                         "-d gpurun_out/pmc_fetch -o pmc -- python3 -u bench.py --pmc-pass",
                         "timeout -s KILL 150 rocprofv3 --pmc WRITE_SIZE --output-format csv "
                         "-d gpurun_out/pmc_write -o pmc -- python3 -u bench.py --pmc-pass",
                         "python bench.py --write-traffic gpurun_out/pmc_fetch gpurun_out/pmc_write"],
            "kernels": kernels}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(json.dumps(data, indent=1, sort_keys=True))
    return 0


def time_calls(fn, warmup: int, steps: int) -> float:
    """Mean milliseconds per call of fn() between torch events."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def attainable_rate(n: int, groups, two: bool = False) -> dict | None:
    """The streaming probe (probe/stream_probe.hip, built with the library) over
    the tile geometries `groups` [(C, k)]: the same element -> index map and the
    same 40 bytes per amplitude as a boundary pass (two=True: two vectors and q,
    72 bytes per amplitude, as a backward boundary pass), no arithmetic.  Runs
    as a child process; None when the probe is not built."""
    import subprocess

    exe = os.path.join(ROOT, "paper_2110_03963_amd", "stream_probe")
    if not os.path.exists(exe):
        return None
    args = [exe] + (["-2"] if two else []) + [str(n)] + [str(x) for g in groups for x in g]
    res = subprocess.run(args, capture_output=True, text=True, timeout=120)
    if res.returncode != 0:
        return None
    rows = [json.loads(line) for line in res.stdout.splitlines() if line.startswith("{")]
    ms = sum(r["ms"] for r in rows) / len(rows)
    bpa = 72.0 if two else 40.0
    return {"GBps": round(bpa * (1 << n) / (ms * 1e-3) / 1e9, 1), "probe_ms": round(ms, 4),
            "geometries": [{"C": r["C"], "k": r["k"], "GBps": r["GBps"]} for r in rows],
            "command": " ".join(["paper_2110_03963_amd/stream_probe"] + args[1:])}


def cpu_baseline(wl) -> dict:
    """The oracle (single-threaded C) on one layer of the same n = 28 instance."""
    import oracle

    t0 = time.perf_counter()
    oracle.evolve("x", wl.q, wl.gammas[:1], wl.ts[:1])
    dt = time.perf_counter() - t0
    return {"value": round(1.0 / dt, 5), "unit": "layer-applications/s", "cores": 1, "kind": "oracle",
            "sample": f"one layer (phase + hypercube mixer + <Q>) of the same n=28 instance at full "
                      f"size: {dt:.1f} s on 1 host core ({platform.processor() or 'cpu'}); "
                      f"value = 1 layer / that time",
            "host_cpus": os.cpu_count()}


# ------------------------------------------------------------------ extras
def extra_qwoa(lib, steps: int, kind: str = "ring", constrained: bool = False) -> dict:
    """QWOA portfolio over all subsets of 26 assets, p = 6; ring mixer
    (transform passes) or complete graph (closed-form passes).  constrained:
    only the C(26, 13) = 10,400,600 subsets of exactly 13 assets (N not a
    power of two: Bluestein's transform for the ring, the closed form for the
    complete graph)."""
    import torch

    import paper_2110_03963_amd as qva
    from paper_2110_03963_amd import _lib
    from workloads import CONFIG_SEEDS, qwoa_portfolio_workload

    from workloads import qwoa_constrained_workload

    n, p = 26, 6
    if constrained:
        wl = qwoa_constrained_workload(n, 13, p, seed=CONFIG_SEEDS["qwoa_n26"], lambda_kind=kind)
    else:
        wl = qwoa_portfolio_workload(n, p, seed=CONFIG_SEEDS["qwoa_n26"], lambda_kind=kind)
    prob = qva.Problem(torch.from_numpy(wl.q).cuda(), "circulant", None, kind)
    g = torch.tensor(wl.gammas, device="cuda")
    t = torch.tensor(wl.ts, device="cuda")
    psi = torch.empty(prob.N, dtype=torch.complex128, device="cuda")
    ws = torch.empty(max(prob.workspace_bytes(p), 16), dtype=torch.uint8, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    flags = _lib.QVA_EVOLVE_SKIP_FINAL_STATE
    stream = torch.cuda.current_stream().cuda_stream

    def run():
        _lib.check("qva_evolve", lib.qva_evolve(prob.cstruct(), g.data_ptr(), t.data_ptr(), p,
                                                psi.data_ptr(), out.data_ptr(), out.data_ptr() + 8,
                                                flags, ws.data_ptr(), ws.numel(), stream))

    ms = time_calls(run, 2, steps)
    infos = plan_of(lib, prob, p, False, flags)

    def run_timed(ev, nev):
        _lib.check("qva_evolve_timed",
                   lib.qva_evolve_timed(prob.cstruct(), g.data_ptr(), t.data_ptr(), p, psi.data_ptr(),
                                        out.data_ptr(), out.data_ptr() + 8, flags, ws.data_ptr(),
                                        ws.numel(), ev, nev, stream))

    per = per_kernel_profile(run_timed, infos, steps)
    plan_bytes = sum(i.bytes for i in infos)
    name = f"qwoa_portfolio_m26_k13_p6_{kind}" if constrained else f"qwoa_portfolio_n26_p6_{kind}"
    return {"workload": name, "N": prob.N, "ms_per_evolve": round(ms, 4),
            "layer_applications_per_s": round(p / (ms * 1e-3), 2), "launches": len(infos),
            "effective_GBps": round(plan_bytes / (ms * 1e-3) / 1e9, 1),
            "f": out[0].item(), "roofline": roofline_of(per, steps),
            "per_kernel_ms_per_evolve": {k: round(v["ms"] / steps, 4) for k, v in sorted(per.items())}}


def extra_adjoint(lib, reps: int, workload: str = "qaoa") -> dict:
    """Adjoint gradient against 4p central-difference and 2p+1 forward-difference
    evaluations of the same fused forward on the same GPU.  Workloads: weighted
    3-regular MaxCut n = 30, p = 12 (24 params), the QWOA portfolio over 2^26
    subsets with the complete-graph mixer, p = 6 (closed-form passes), or the
    constrained portfolio (13 of 26 assets, N = 10,400,600) with the ring,
    p = 6 (Bluestein's transform)."""
    import numpy as np
    import torch

    import paper_2110_03963_amd as qva
    from paper_2110_03963_amd import _lib
    from workloads import (CONFIG_SEEDS, maxcut_qualities_device, qaoa_maxcut_workload,
                           qwoa_constrained_workload, qwoa_portfolio_workload)

    if workload == "qaoa":
        n, p = 30, 12
        wl = qaoa_maxcut_workload(n, p, graph="regular3", weighted=True, seed=CONFIG_SEEDS["grad_n30"],
                                  build_q=False)
        q = maxcut_qualities_device(n, wl.edges, wl.weights, "cuda")
        prob = qva.Problem(q, "x")
        name = "adjoint_qaoa_maxcut_n30_p12"
        h_t = 1e-5
    elif workload == "qwoa_constrained_ring":
        n, p = 26, 6
        wl = qwoa_constrained_workload(n, 13, p, seed=CONFIG_SEEDS["qwoa_n26"], lambda_kind="ring")
        prob = qva.Problem(torch.from_numpy(wl.q).cuda(), "circulant", None, "ring")
        name = "adjoint_qwoa_portfolio_m26_k13_p6_ring"
        h_t = 1e-5
    else:
        n, p = 26, 6
        wl = qwoa_portfolio_workload(n, p, seed=CONFIG_SEEDS["qwoa_n26"], lambda_kind="complete")
        prob = qva.Problem(torch.from_numpy(wl.q).cuda(), "circulant", None, "complete")
        name = "adjoint_qwoa_portfolio_n26_p6_complete"
        h_t = 1e-5 / (1 << n)  # f oscillates in t at frequency N (e^{-i t N})
    g = torch.tensor(wl.gammas, device="cuda")
    t = torch.tensor(wl.ts, device="cuda")
    psi = torch.empty(prob.N, dtype=torch.complex128, device="cuda")
    chi = torch.empty(prob.N, dtype=torch.complex128, device="cuda")
    wsg = torch.empty(max(prob.workspace_bytes(p, True), 256), dtype=torch.uint8, device="cuda")
    wse = torch.empty(max(prob.workspace_bytes(p), 16), dtype=torch.uint8, device="cuda")
    f = torch.empty((), dtype=torch.float64, device="cuda")
    dg = torch.empty(p, dtype=torch.float64, device="cuda")
    dt = torch.empty(p, dtype=torch.float64, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    flags = _lib.QVA_EVOLVE_SKIP_FINAL_STATE

    def adjoint():
        _lib.check("qva_grad", lib.qva_grad(prob.cstruct(), g.data_ptr(), t.data_ptr(), p, psi.data_ptr(),
                                            chi.data_ptr(), f.data_ptr(), dg.data_ptr(), dt.data_ptr(),
                                            wsg.data_ptr(), wsg.numel(), stream))

    gp = torch.empty(p, dtype=torch.float64, device="cuda")
    tp = torch.empty(p, dtype=torch.float64, device="cuda")

    def forward():
        _lib.check("qva_evolve", lib.qva_evolve(prob.cstruct(), gp.data_ptr(), tp.data_ptr(), p,
                                                psi.data_ptr(), out.data_ptr(), out.data_ptr() + 8,
                                                flags, wse.data_ptr(), wse.numel(), stream))

    h = 1e-5
    fd_vals = torch.empty(4 * p, dtype=torch.float64, device="cuda")

    def central():
        # 4p fused forward evaluations f(theta +- h e_k), results kept on device
        for k in range(2 * p):
            for sgn in (1.0, -1.0):
                gp.copy_(g)
                tp.copy_(t)
                (gp if k < p else tp)[k % p] += sgn * (h if k < p else h_t)
                forward()
                fd_vals[2 * k + (0 if sgn > 0 else 1)] = out[0]

    def forward_diff():
        for k in range(2 * p + 1):
            gp.copy_(g)
            tp.copy_(t)
            if k < 2 * p:
                (gp if k < p else tp)[k % p] += h if k < p else h_t
            forward()

    ms_adj = time_calls(adjoint, 1, reps)
    ms_cfd = time_calls(central, 1, reps)
    ms_ffd = time_calls(forward_diff, 0, reps)
    adj = torch.cat([dg, dt]).cpu().numpy()
    fdv = fd_vals.cpu().numpy()
    # the step actually taken: (x + h) - (x - h), exact in double (the t step
    # of the complete graph, 1e-5 / N, is only a few hundred ulps of t)
    x = np.concatenate([np.asarray(wl.gammas, np.float64), np.asarray(wl.ts, np.float64)])
    hs = np.array([h] * p + [h_t] * p)
    cfd = (fdv[0::2] - fdv[1::2]) / ((x + hs) - (x - hs))
    rel = float(np.max(np.abs(adj - cfd)) / np.max(np.abs(adj)))
    infos = plan_of(lib, prob, p, True, 0)

    def run_timed(ev, nev):
        _lib.check("qva_grad_timed",
                   lib.qva_grad_timed(prob.cstruct(), g.data_ptr(), t.data_ptr(), p, psi.data_ptr(),
                                      chi.data_ptr(), f.data_ptr(), dg.data_ptr(), dt.data_ptr(),
                                      wsg.data_ptr(), wsg.numel(), ev, nev, stream))

    per = per_kernel_profile(run_timed, infos, 1)
    plan_bytes = sum(i.bytes for i in infos)
    roof = roofline_of(per, 1)
    if workload == "qaoa" and roof["kernel"].startswith("grad_bound<"):
        # the streaming probe over the backward boundary passes' tiles, 72 B/amp
        geoms = sorted({(i.col_bits, i.group_first) for i in infos if i.kind == 20})
        att = attainable_rate(prob.n, geoms, two=True)
        if att:
            roof["attainable"] = att
            roof["frac_of_attainable"] = round(roof["achieved"] / att["GBps"], 4)
    return {"workload": name, "params": 2 * p,
            "ms_per_adjoint_gradient": round(ms_adj, 2),
            "adjoint_gradients_per_s": round(1e3 / ms_adj, 3),
            "ms_per_central_fd_gradient": round(ms_cfd, 2),
            "ms_per_forward_fd_gradient": round(ms_ffd, 2),
            "speedup_vs_central_fd": round(ms_cfd / ms_adj, 2),
            "speedup_vs_forward_fd": round(ms_ffd / ms_adj, 2),
            "max_rel_diff_adjoint_vs_central_fd": rel, "fd_steps": {"gamma": h, "t": h_t},
            "f": f.item(), "launches": len(infos),
            "effective_GBps": round(plan_bytes / (ms_adj * 1e-3) / 1e9, 1),
            "roofline": roof,
            "per_kernel_ms": {k: round(v["ms"], 3) for k, v in sorted(per.items())}}


def extra_exqaoa(lib, steps: int) -> dict:
    """Extended QAOA on the n = 28, p = 8 weighted 3-regular MaxCut instance of
    the headline (42 edges: one Z_u Z_v term and one angle per edge and layer,
    p (1 + 42) = 344 parameters): the fused forward and the adjoint gradient,
    beside the plain QAOA forward of the same instance."""
    import numpy as np
    import torch

    import paper_2110_03963_amd as qva
    from paper_2110_03963_amd import _lib
    from workloads import CONFIG_SEEDS, exqaoa_maxcut_workload, maxcut_qualities_device

    n, p = 28, 8
    wl = exqaoa_maxcut_workload(n, p, seed=CONFIG_SEEDS["qaoa_n28"], build_q=False)
    E = len(wl.supports)
    q = maxcut_qualities_device(n, wl.edges, wl.weights, "cuda")
    prob = qva.Problem(q, "x", terms=(wl.supports, wl.coefs))
    plain = qva.Problem(q, "x")
    g = torch.tensor(np.ascontiguousarray(wl.gammas).ravel(), device="cuda")
    g1 = torch.tensor(np.ascontiguousarray(wl.gammas.mean(axis=1)), device="cuda")
    t = torch.tensor(wl.ts, device="cuda")
    psi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    chi = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    wse = torch.empty(max(prob.workspace_bytes(p), plain.workspace_bytes(p), 16), dtype=torch.uint8,
                      device="cuda")
    wsg = torch.empty(max(prob.workspace_bytes(p, True), 256), dtype=torch.uint8, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    f = torch.empty((), dtype=torch.float64, device="cuda")
    dg = torch.empty(p * E, dtype=torch.float64, device="cuda")
    dt = torch.empty(p, dtype=torch.float64, device="cuda")
    flags = _lib.QVA_EVOLVE_SKIP_FINAL_STATE
    stream = torch.cuda.current_stream().cuda_stream

    def forward(pr, gg):
        _lib.check("qva_evolve", lib.qva_evolve(pr.cstruct(), gg.data_ptr(), t.data_ptr(), p,
                                                psi.data_ptr(), out.data_ptr(), out.data_ptr() + 8,
                                                flags, wse.data_ptr(), wse.numel(), stream))

    def adjoint():
        _lib.check("qva_grad", lib.qva_grad(prob.cstruct(), g.data_ptr(), t.data_ptr(), p, psi.data_ptr(),
                                            chi.data_ptr(), f.data_ptr(), dg.data_ptr(), dt.data_ptr(),
                                            wsg.data_ptr(), wsg.numel(), stream))

    ms_fwd = time_calls(lambda: forward(prob, g), 2, steps)
    f_ex = out[0].item()
    ms_plain = time_calls(lambda: forward(plain, g1), 2, steps)
    ms_adj = time_calls(adjoint, 1, max(2, steps // 4))
    infos = plan_of(lib, prob, p, False, flags)

    def run_timed(ev, nev):
        _lib.check("qva_evolve_timed",
                   lib.qva_evolve_timed(prob.cstruct(), g.data_ptr(), t.data_ptr(), p, psi.data_ptr(),
                                        out.data_ptr(), out.data_ptr() + 8, flags, wse.data_ptr(),
                                        wse.numel(), ev, nev, stream))

    per = per_kernel_profile(run_timed, infos, steps)
    ginfos = plan_of(lib, prob, p, True, 0)

    def grad_timed(ev, nev):
        _lib.check("qva_grad_timed",
                   lib.qva_grad_timed(prob.cstruct(), g.data_ptr(), t.data_ptr(), p, psi.data_ptr(),
                                      chi.data_ptr(), f.data_ptr(), dg.data_ptr(), dt.data_ptr(),
                                      wsg.data_ptr(), wsg.numel(), ev, nev, stream))

    gper = per_kernel_profile(grad_timed, ginfos, 1)

    def zname(per):  # the phase passes of this plan are the Z-string variants
        out = {}
        for k, v in per.items():
            for a, b in (("XMODE_FIRST>", "XMODE_FIRST_Z>"), ("XMODE_BOUNDARY>", "XMODE_BOUNDARY_Z>"),
                         ("grad_bound<", "grad_bound_z<"), ("grad_final<", "grad_final_z<")):
                k = k.replace(a, b)
            out[k] = v
        return out

    per, gper = zname(per), zname(gper)
    plan_bytes = sum(i.bytes for i in infos)
    gplan_bytes = sum(i.bytes for i in ginfos)
    return {"workload": "exqaoa_maxcut_n28_p8_regular3", "terms": E, "params": p * (E + 1),
            "ms_per_evolve": round(ms_fwd, 3), "layer_applications_per_s": round(p / (ms_fwd * 1e-3), 2),
            "ms_per_evolve_plain_qaoa_same_instance": round(ms_plain, 3),
            "ms_per_adjoint_gradient": round(ms_adj, 2),
            "effective_GBps_evolve": round(plan_bytes / (ms_fwd * 1e-3) / 1e9, 1),
            "effective_GBps_gradient": round(gplan_bytes / (ms_adj * 1e-3) / 1e9, 1),
            "f": f_ex, "f_gradient_call": f.item(),
            "roofline_evolve": roofline_of(per, steps), "roofline_gradient": roofline_of(gper, 1),
            "per_kernel_ms_per_evolve": {k: round(v["ms"] / steps, 4) for k, v in sorted(per.items())},
            "per_kernel_ms_per_gradient": {k: round(v["ms"], 3) for k, v in sorted(gper.items())}}


def extra_qaoaz(lib, steps: int) -> dict:
    """QAOAz portfolio over all 2^26 subsets (the QWOA portfolio's q, gammas
    and ts), the parity mixer on the ring of all 26 qubits, psi0 = |D^26_13>,
    p = 6: the fused forward and the adjoint gradient.  Each call starts from
    a fresh copy of psi0 (outside the timed interval: events bracket the
    library call alone)."""
    import numpy as np
    import torch

    import paper_2110_03963_amd as qva
    from paper_2110_03963_amd import _lib
    from workloads import CONFIG_SEEDS, dicke_state_device, qaoaz_portfolio_workload

    n, k, p = 26, 13, 6
    wl = qaoaz_portfolio_workload(n, k, p, seed=CONFIG_SEEDS["qwoa_n26"])
    q = torch.from_numpy(wl.q).cuda()
    psi0 = dicke_state_device(n, k, "cuda")
    pairs = qva.parity_ring_pairs(range(n))
    prob = qva.Problem(q, "xy", pairs=pairs, psi0=psi0)
    g = torch.tensor(wl.gammas, device="cuda")
    t = torch.tensor(wl.ts, device="cuda")
    psi = torch.empty_like(psi0)
    chi = torch.empty_like(psi0)
    wse = torch.empty(max(prob.workspace_bytes(p), 16), dtype=torch.uint8, device="cuda")
    wsg = torch.empty(max(prob.workspace_bytes(p, True), 256), dtype=torch.uint8, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    f = torch.empty((), dtype=torch.float64, device="cuda")
    dg = torch.empty(p, dtype=torch.float64, device="cuda")
    dt = torch.empty(p, dtype=torch.float64, device="cuda")
    flags = _lib.QVA_EVOLVE_SKIP_FINAL_STATE
    stream = torch.cuda.current_stream().cuda_stream

    def forward():
        _lib.check("qva_evolve", lib.qva_evolve(prob.cstruct(), g.data_ptr(), t.data_ptr(), p, psi.data_ptr(),
                                                out.data_ptr(), out.data_ptr() + 8, flags, wse.data_ptr(),
                                                wse.numel(), stream))

    def adjoint():
        _lib.check("qva_grad", lib.qva_grad(prob.cstruct(), g.data_ptr(), t.data_ptr(), p, psi.data_ptr(),
                                            chi.data_ptr(), f.data_ptr(), dg.data_ptr(), dt.data_ptr(),
                                            wsg.data_ptr(), wsg.numel(), stream))

    def timed(fn, reps):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        psi.copy_(psi0)
        fn()  # warm-up
        for e0, e1 in evs:
            psi.copy_(psi0)
            e0.record()
            fn()
            e1.record()
        torch.cuda.synchronize()
        return sum(e0.elapsed_time(e1) for e0, e1 in evs) / reps

    ms_fwd = timed(forward, steps)
    f_fwd = out[0].item()
    ms_adj = timed(adjoint, max(2, steps // 2))
    infos = plan_of(lib, prob, p, False, flags)

    def run_timed(ev, nev):
        psi.copy_(psi0)
        _lib.check("qva_evolve_timed",
                   lib.qva_evolve_timed(prob.cstruct(), g.data_ptr(), t.data_ptr(), p, psi.data_ptr(),
                                        out.data_ptr(), out.data_ptr() + 8, flags, wse.data_ptr(),
                                        wse.numel(), ev, nev, stream))

    per = per_kernel_profile(run_timed, infos, steps)
    ginfos = plan_of(lib, prob, p, True, 0)

    def grad_timed(ev, nev):
        psi.copy_(psi0)
        _lib.check("qva_grad_timed",
                   lib.qva_grad_timed(prob.cstruct(), g.data_ptr(), t.data_ptr(), p, psi.data_ptr(),
                                      chi.data_ptr(), f.data_ptr(), dg.data_ptr(), dt.data_ptr(),
                                      wsg.data_ptr(), wsg.numel(), ev, nev, stream))

    gper = per_kernel_profile(grad_timed, ginfos, 1)
    plan_bytes = sum(i.bytes for i in infos)
    gplan_bytes = sum(i.bytes for i in ginfos)
    G = sum(1 for i in infos if i.kind in (42, 43)) // p
    return {"workload": "qaoaz_portfolio_m26_k13_p6_ring", "pairs": len(pairs), "passes_per_layer": G,
            "ms_per_evolve": round(ms_fwd, 3), "layer_applications_per_s": round(p / (ms_fwd * 1e-3), 2),
            "ms_per_adjoint_gradient": round(ms_adj, 3),
            "effective_GBps_evolve": round(plan_bytes / (ms_fwd * 1e-3) / 1e9, 1),
            "effective_GBps_gradient": round(gplan_bytes / (ms_adj * 1e-3) / 1e9, 1),
            "f": f_fwd, "f_gradient_call": f.item(),
            "roofline_evolve": roofline_of(per, steps), "roofline_gradient": roofline_of(gper, 1),
            "per_kernel_ms_per_evolve": {kk: round(v["ms"] / steps, 4) for kk, v in sorted(per.items())},
            "per_kernel_ms_per_gradient": {kk: round(v["ms"], 3) for kk, v in sorted(gper.items())}}


def extra_batch(lib) -> dict:
    """512 independent QAOA MaxCut instances (n ~ U{12..22}, p ~ U{1..8},
    G(n, 0.4), weights U(0,1)): f and the adjoint gradient of every instance
    plus a gradient step, replayed as one captured HIP graph; compared with
    one qva_grad call per instance."""
    import torch

    import paper_2110_03963_amd as qva
    from paper_2110_03963_amd import _lib
    from paper_2110_03963_amd.autotune import time_batch_grad, tune_batch
    from workloads import CONFIG_SEEDS, batched_workloads, maxcut_qualities_device

    wls = batched_workloads(512, seed=CONFIG_SEEDS["batch512"], build_q=False)
    qs = [maxcut_qualities_device(w.n, w.edges, w.weights, "cuda") for w in wls]
    gs = [w.gammas for w in wls]
    ts = [w.ts for w in wls]
    tune = tune_batch(qs, gs, ts, reps=2)
    b = qva.Batch(qs, gs, ts, align=tune["align"])
    ms_eager = time_batch_grad(b, reps=3)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        b.grad()
        b.sgd(1e-3)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms_graph = e0.elapsed_time(e1) / reps
    # one qva_grad per instance, back to back
    probs = [qva.Problem(q, "x") for q in qs]
    psi = torch.empty(1 << 22, dtype=torch.complex128, device="cuda")
    chi = torch.empty_like(psi)
    ws = torch.empty(max(max(pr.workspace_bytes(w.p, True) for pr, w in zip(probs, wls)), 256),
                     dtype=torch.uint8, device="cuda")
    gd = [torch.tensor(w.gammas, device="cuda") for w in wls]
    td = [torch.tensor(w.ts, device="cuda") for w in wls]
    fo = torch.empty(512, dtype=torch.float64, device="cuda")
    dg = torch.empty(8, dtype=torch.float64, device="cuda")
    dt = torch.empty(8, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream

    def per_instance():
        for i, (pr, w) in enumerate(zip(probs, wls)):
            _lib.check("qva_grad", lib.qva_grad(pr.cstruct(), gd[i].data_ptr(), td[i].data_ptr(), w.p,
                                                psi.data_ptr(), chi.data_ptr(), fo.data_ptr() + 8 * i,
                                                dg.data_ptr(), dt.data_ptr(), ws.data_ptr(), ws.numel(), st))

    ms_single = time_calls(per_instance, 1, 2)
    total_bytes = 0.0
    for pr, w in zip(probs, wls):
        total_bytes += sum(i.bytes for i in plan_of(lib, pr, w.p, True, 0))
    return {"workload": "batch512_qaoa_maxcut_n12-22_p1-8", "instances": 512,
            "amplitudes": int(sum(1 << w.n for w in wls)),
            "autotune": tune, "rounds": b.rounds, "launches_per_batch": b.launches, "tiles": b.tiles,
            "ms_per_batch_graph_replay": round(ms_graph, 3),
            "ms_per_batch_eager": round(ms_eager, 3),
            "instance_gradients_per_s": round(512 / (ms_graph * 1e-3), 1),
            "ms_per_batch_one_call_per_instance": round(ms_single, 3),
            "speedup_vs_one_call_per_instance": round(ms_single / ms_graph, 2),
            "effective_GBps": round(total_bytes / (ms_graph * 1e-3) / 1e9, 1)}


# Secondary measurements: name -> fn(lib, steps).
EXTRAS = {
    "qwoa_circulant": lambda lib, steps: extra_qwoa(lib, max(3, steps // 2)),
    "qwoa_complete": lambda lib, steps: extra_qwoa(lib, max(3, steps // 2), "complete"),
    "qwoa_constrained_ring": lambda lib, steps: extra_qwoa(lib, max(3, steps // 2), "ring", True),
    "qwoa_constrained_complete": lambda lib, steps: extra_qwoa(lib, max(3, steps // 2), "complete", True),
    "adjoint_vs_fd": lambda lib, steps: extra_adjoint(lib, 2),
    "adjoint_qwoa_complete": lambda lib, steps: extra_adjoint(lib, 3, "qwoa_complete"),
    "adjoint_qwoa_constrained_ring": lambda lib, steps: extra_adjoint(lib, 3, "qwoa_constrained_ring"),
    "batched": lambda lib, steps: extra_batch(lib),
    "exqaoa": lambda lib, steps: extra_exqaoa(lib, max(3, steps // 2)),
    "qaoaz": lambda lib, steps: extra_qaoaz(lib, max(3, steps // 2)),
}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--pmc-pass", action="store_true",
                    help="run the short program profiled by the HBM-traffic counter runs")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="store per-launch HBM traffic from the two counter runs' CSV output")
    ap.add_argument("--valu-summary", nargs=2, metavar=("COUNTER_DIR", "KERNEL_STATS_CSV"),
                    help="per-kernel VALU load from a --pmc SQ_INSTS_VALU* run and a --stats run")
    ap.add_argument("--extra", choices=sorted(EXTRAS),
                    help="run one secondary measurement alone and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.write_traffic:
        return write_traffic(*args.write_traffic)
    if args.valu_summary:
        return valu_summary(*args.valu_summary)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the sharded multi-GPU path is a design, not part of this build)", file=sys.stderr)
        return 2
    if args.pmc_pass:
        return pmc_pass()
    if args.extra:
        import torch

        import paper_2110_03963_amd as qva

        if not torch.cuda.is_available():
            print("bench.py needs a GPU", file=sys.stderr)
            return 1
        print(json.dumps({args.extra: EXTRAS[args.extra](qva.load_library(), args.steps)}), flush=True)
        return 0

    import torch

    import paper_2110_03963_amd as qva
    from paper_2110_03963_amd import _lib
    from workloads import CONFIG_SEEDS, qaoa_maxcut_workload

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    lib = qva.load_library()
    dev = torch.device("cuda:0")

    n, p = 28, 8
    t_gen = time.perf_counter()
    wl = qaoa_maxcut_workload(n, p, graph="regular3", weighted=True, seed=CONFIG_SEEDS["qaoa_n28"])
    log(f"workload n={n} p={p} generated in {time.perf_counter() - t_gen:.1f}s")
    q = torch.from_numpy(wl.q).to(dev)
    prob = qva.Problem(q, "x")
    g = torch.tensor(wl.gammas, dtype=torch.float64, device=dev)
    t = torch.tensor(wl.ts, dtype=torch.float64, device=dev)
    psi = torch.empty(1 << n, dtype=torch.complex128, device=dev)
    ws = torch.empty(max(prob.workspace_bytes(p), 16), dtype=torch.uint8, device=dev)
    out = torch.empty(2, dtype=torch.float64, device=dev)
    flags = _lib.QVA_EVOLVE_SKIP_FINAL_STATE  # the workload's output is <Q>
    stream = torch.cuda.current_stream().cuda_stream

    def step():
        _lib.check("qva_evolve", lib.qva_evolve(prob.cstruct(), g.data_ptr(), t.data_ptr(), p,
                                                psi.data_ptr(), out.data_ptr(), out.data_ptr() + 8,
                                                flags, ws.data_ptr(), ws.numel(), stream))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    f_val, norm_val = out[0].item(), out[1].item()
    value = p * args.steps / (ms_total * 1e-3)
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step, f={f_val:.15f}, norm={norm_val:.15f}")

    # per-launch timing of the same plan (HIP events on the same stream)
    infos = plan_of(lib, prob, p, False, flags)

    def run_timed(ev, nev):
        _lib.check("qva_evolve_timed",
                   lib.qva_evolve_timed(prob.cstruct(), g.data_ptr(), t.data_ptr(), p, psi.data_ptr(),
                                        out.data_ptr(), out.data_ptr() + 8, flags, ws.data_ptr(),
                                        ws.numel(), ev, nev, stream))

    per = per_kernel_profile(run_timed, infos, args.steps)
    roofline = roofline_of(per, args.steps)
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        entry = tr.get("kernels", {}).get(roofline["kernel"])
        if tr.get("source_digest") == source_digest(*TRAFFIC_SOURCES) and entry:
            roofline["traffic"] = entry["bytes_per_launch"]
    # the attainable rate of the dominant kernel's access pattern (its tile
    # geometries, the same bytes, no arithmetic), from the streaming probe
    geoms = sorted({(i.col_bits, i.group_first) for i in infos
                    if kernel_name(i.kind, i.col_bits) == roofline["kernel"] and i.col_bits >= 3})
    att = attainable_rate(n, geoms) if geoms else None
    if att:
        roofline["attainable"] = att
        roofline["frac_of_attainable"] = round(roofline["achieved"] / att["GBps"], 4)
    plan_bytes = sum(i.bytes for i in infos)

    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "layer-applications/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "qaoa_maxcut_n28_p8", "n_qubits": n, "p": p,
                   "graph": "random 3-regular, weights U(0,1)", "quality": "weighted cut",
                   "seed": CONFIG_SEEDS["qaoa_n28"], "output": "<Q> (final state not stored)"},
        "roofline": roofline,
        "plan": {"launches": len(infos), "algorithmic_bytes": plan_bytes,
                 "effective_GBps": round(plan_bytes / (ms_step * 1e-3) / 1e9, 1),
                 "per_kernel_ms_per_step": {k: round(v["ms"] / args.steps, 4)
                                            for k, v in sorted(per.items())}},
        "f": f_val,
        "norm": norm_val,
        "device": torch.cuda.get_device_name(0),
    }
    del psi, ws, q, prob
    torch.cuda.empty_cache()
    if not args.no_extras:
        extras = {}
        for name, fn in EXTRAS.items():
            log(f"extra: {name} ...")
            try:
                extras[name] = fn(lib, args.steps)
            except Exception as exc:  # reported, not fatal: the headline line still prints
                extras[name] = {"error": repr(exc)}
            torch.cuda.empty_cache()
        result["extras"] = extras
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on one layer ...")
        result["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
