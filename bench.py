"""Benchmark of the QVA state-evolution hot path on one MI355X.

A step is one fused evolution of the QAOA MaxCut workload (n = 28 qubits,
2^28 complex128 amplitudes, random 3-regular graph with weights ~ U(0,1),
p = 8 layers): psi_0, p x (phase + hypercube mixer), <Q>.  Inputs are seeded
synthetic data resident in HBM before the timed region.

Prints one JSON line: layer-applications/s, the roofline of the dominant
kernel (per-launch HIP events over the timed steps), and the CPU oracle timed
on a bounded sample (rank 0, N = 1 only).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-extras]
"""

from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import math
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

KIND_NAMES = {0: "whole", 1: "first", 2: "middle", 3: "boundary", 4: "last", 5: "last_store",
              6: "init", 7: "expect", 8: "reduce"}


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

    def elapsed_ms(self, a: int, b: int) -> float:
        ms = ctypes.c_float()
        if self.hip.hipEventElapsedTime(ctypes.byref(ms), self.ev[a], self.ev[b]) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return ms.value

    def close(self):
        for h in self.ev:
            self.hip.hipEventDestroy(h)


def kernel_symbol(kind: int, col_bits: int) -> str:
    mode = {1: "XMODE_FIRST", 2: "XMODE_MIDDLE", 3: "XMODE_BOUNDARY", 4: "XMODE_LAST",
            5: "XMODE_LAST_STORE"}.get(kind)
    if mode is None:
        return KIND_NAMES[kind]
    return f"xpass_kernel<{col_bits}, {mode}>"


def source_digest(*paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(wl) -> dict:
    """The oracle (single-threaded C) on one layer of the same n = 28 instance."""
    import oracle

    t0 = time.perf_counter()
    oracle.evolve("x", wl.q, wl.gammas[:1], wl.ts[:1])
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "layer-applications/s", "cores": 1, "kind": "oracle",
            "sample": f"one layer (phase + hypercube mixer + <Q>) of the same n=28 instance, "
                      f"full size, {dt:.1f} s on 1 host core ({platform.processor() or 'cpu'})"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the sharded multi-GPU path is a design, not part of this build)", file=sys.stderr)
        return 2

    import numpy as np
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
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] workload n={n} p={p} generated in {t_gen:.1f}s", file=sys.stderr, flush=True)
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
    t_wall = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    f_val, norm_val = out[0].item(), out[1].item()
    value = p * args.steps / (ms_total * 1e-3)
    print(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step, f={f_val:.15f}, "
          f"norm={norm_val:.15f}", file=sys.stderr, flush=True)

    # ---- per-launch timing of the same plan (HIP events on the same stream)
    npl = lib.qva_plan(prob.cstruct(), p, 0, flags, None, 0)
    infos = (_lib.QvaPassInfo * npl)()
    lib.qva_plan(prob.cstruct(), p, 0, flags, infos, npl)
    evs = HipEvents(2 * npl * args.steps)
    for s in range(args.steps):
        arr = ctypes.cast(ctypes.byref(evs.array, ctypes.sizeof(ctypes.c_void_p) * 2 * npl * s),
                          ctypes.POINTER(ctypes.c_void_p))
        _lib.check("qva_evolve_timed",
                   lib.qva_evolve_timed(prob.cstruct(), g.data_ptr(), t.data_ptr(), p,
                                        psi.data_ptr(), out.data_ptr(), out.data_ptr() + 8, flags,
                                        ws.data_ptr(), ws.numel(), arr, 2 * npl, stream))
    torch.cuda.synchronize()
    per_kernel: dict[str, dict] = {}
    for s in range(args.steps):
        for i in range(npl):
            info = infos[i]
            name = kernel_symbol(info.kind, info.col_bits)
            d = per_kernel.setdefault(name, {"launches": 0, "ms": 0.0, "bytes": 0.0})
            d["launches"] += 1
            d["ms"] += evs.elapsed_ms(2 * (s * npl + i), 2 * (s * npl + i) + 1)
            d["bytes"] += info.bytes
    evs.close()
    dom_name, dom = max(per_kernel.items(), key=lambda kv: kv[1]["ms"])
    avg_ms = dom["ms"] / dom["launches"]
    bytes_per_launch = dom["bytes"] / dom["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    plan_bytes = sum(infos[i].bytes for i in range(npl))
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        digest = source_digest(os.path.join(ROOT, "paper_2110_03963_amd", "csrc", "qva_xmix.hip"))
        if tr.get("source_digest") == digest and tr.get("kernel") == dom_name:
            traffic = tr.get("bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dom_name, "launches_per_step": dom["launches"] // args.steps,
                "avg_launch_ms": round(avg_ms, 4),
                "algorithmic_bytes_per_launch": bytes_per_launch}

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
        "plan": {"launches": npl, "algorithmic_bytes": plan_bytes,
                 "effective_GBps": round(plan_bytes / (ms_step * 1e-3) / 1e9, 1),
                 "per_kernel_ms_per_step": {k: round(v["ms"] / args.steps, 4)
                                            for k, v in sorted(per_kernel.items())}},
        "f": f_val,
        "norm": norm_val,
        "device": torch.cuda.get_device_name(0),
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on one layer ...", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(wl)
        result["cpu_baseline"]["host_cpus"] = os.cpu_count()
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
