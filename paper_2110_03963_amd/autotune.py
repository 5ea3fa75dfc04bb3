"""Autotuning: the batched engine's launch plan, and the split of the
strided qubit groups (how many qubits each tile pass handles above the
contiguous 12).

Batched plans:

The batched gradient groups the passes of all instances into rounds; how
instances are aligned to rounds (all start together, all finish together, or
start rounds spread to even out the tiles per round) changes how well each
launch fills the GPU, and so does splitting the instances into lanes,
independent sequences of rounds on streams of their own whose launches
overlap.  `tune_batch` times each (alignment, lanes) candidate on the actual
instances and caches the winner in a JSON file keyed by the batch's shape
(the multiset of (n, p)), the device name and the library version.

Cache file: $QVA_TUNE_CACHE, else ~/.cache/qva/tune.json.
"""

from __future__ import annotations

import ctypes
import hashlib
import json
import os

import torch

from . import _lib
from .qva import Batch

CANDIDATES = ("start", "end", "spread")


def cache_path() -> str:
    p = os.environ.get("QVA_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "qva", "tune.json")


def batch_signature(ns, ps) -> str:
    shape = sorted(zip(ns, ps))
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    ver = _lib.load().qva_version().decode()
    h = hashlib.sha256(json.dumps([shape, dev, ver]).encode()).hexdigest()[:24]
    return f"batch-{h}"


def _load(path: str) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path: str, data: dict) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_batch_grad(batch: Batch, reps: int = 3, warmup: int = 1) -> float:
    """Mean milliseconds of one batched gradient (events on the current stream)."""
    for _ in range(warmup):
        batch.grad()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        batch.grad()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


LANE_CANDIDATES = (1, 2, 3, 4)


def tune_batch(qs, gammas, ts, *, candidates=CANDIDATES, lanes=LANE_CANDIDATES, reps: int = 2,
               use_cache: bool = True, path: str | None = None) -> dict:
    """Pick the round alignment and the lane count (independent sequences of
    rounds on their own streams, qva_batch_create_lanes) with the shortest
    batched gradient.

    Returns {"align": best, "lanes": best, "ms": {"align/lanes": time},
    "cached": bool}.
    """
    path = path or cache_path()
    ns = [int(q.numel()).bit_length() - 1 for q in qs]
    ps = [len(g) for g in gammas]
    key = batch_signature(ns, ps)
    data = _load(path) if use_cache else {}
    if use_cache and key in data and data[key].get("align") in candidates and data[key].get("lanes") in lanes:
        out = dict(data[key])
        out["cached"] = True
        return out
    times = {}
    for align in candidates:
        for nl in lanes:
            b = Batch(qs, gammas, ts, align=align, lanes=nl)
            times[f"{align}/{nl}"] = time_batch_grad(b, reps=reps)
            del b
            torch.cuda.empty_cache()
    best = min(times, key=times.get)
    align, nl = best.split("/")
    entry = {"align": align, "lanes": int(nl), "ms": times}
    if use_cache:
        data = _load(path)
        data[key] = entry
        _store(path, data)
    return dict(entry, cached=False)


# ------------------------------------------------------------- group splits
MAX_HIGH = 9  # qubits per strided group (a tile keeps >= 8 contiguous amplitudes)


def split_candidates(n: int) -> list[tuple[int, ...]]:
    """Splits of the n - 12 qubits above the contiguous group into strided
    groups of 1..9 qubits, from qubit 12 upward: every split into the fewest
    groups whose sizes differ by at most 2, and every split into one group
    more whose sizes differ by at most 1 (more passes, longer rows)."""
    rem = n - 12
    if rem <= 0:
        return [()]
    out = []

    def comps(total, parts, lo, hi):
        if parts == 1:
            if lo <= total <= hi:
                yield (total,)
            return
        for first in range(lo, min(hi, total) + 1):
            for rest in comps(total - first, parts - 1, lo, hi):
                yield (first,) + rest

    fewest = -(-rem // MAX_HIGH)
    for parts, spread in ((fewest, 2), (fewest + 1, 1)):
        if parts > rem:
            continue
        for c in comps(rem, parts, 1, MAX_HIGH):
            if max(c) - min(c) <= spread:
                out.append(c)
    return out


def get_split(n: int) -> tuple[int, ...]:
    lib = _lib.load()
    arr = (ctypes.c_int * 32)()
    cnt = lib.qva_get_group_split(n, arr, 32)
    return tuple(arr[:max(cnt, 0)])


def set_split(n: int, split) -> None:
    lib = _lib.load()
    if split is None or len(split) == 0:
        _lib.check("qva_set_group_split", lib.qva_set_group_split(n, None, 0))
        return
    arr = (ctypes.c_int * len(split))(*split)
    _lib.check("qva_set_group_split", lib.qva_set_group_split(n, arr, len(split)))


def _device_key() -> list:
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    arch = torch.cuda.get_device_properties(0).gcnArchName if torch.cuda.is_available() else ""
    return [dev, arch, torch.version.hip, _lib.load().qva_version().decode()]


def split_signature(call: str, mixer: str, n: int) -> str:
    h = hashlib.sha256(json.dumps([call, mixer, n] + _device_key()).encode()).hexdigest()[:24]
    return f"split-{call}-{mixer}-n{n}-{h}"


def _time_call(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    ts = sorted(a.elapsed_time(b) for a, b in ev)
    return ts[len(ts) // 2]


def tune_split(problem, gammas, ts, *, call: str = "evolve", candidates=None, reps: int = 3,
               use_cache: bool = True, path: str | None = None) -> dict:
    """Time problem's qva_evolve (call="evolve") or qva_grad (call="grad")
    under every candidate split of its qubits (split_candidates), keep the
    fastest in effect (qva_set_group_split) and cache it in the JSON file
    keyed by (call, mixer, n, device, arch, ROCm, library version).

    Returns {"split": best, "default": default split, "ms": {split: median ms},
    "cached": bool}."""
    from .qva import evolve, grad

    n = problem.n
    path = path or cache_path()
    key = split_signature(call, problem.mixer, n)
    default = tuple(get_split(n)) if n > 12 else ()
    if use_cache:
        data = _load(path)
        if key in data:
            out = dict(data[key])
            set_split(n, out["split"])
            out["cached"] = True
            return out
    cands = candidates or split_candidates(n)
    before = get_split(n)
    times = {}
    try:
        for c in cands:
            set_split(n, c)
            if call == "grad":
                fn = lambda: grad(problem, gammas, ts)  # noqa: E731
            else:
                fn = lambda: evolve(problem, gammas, ts, store=False)  # noqa: E731
            times[c] = _time_call(fn, reps)
    finally:
        set_split(n, before)
    best = min(times, key=times.get)
    set_split(n, best)
    entry = {"split": list(best), "default": list(default),
             "ms": {",".join(map(str, c)): round(t, 4) for c, t in times.items()}}
    if use_cache:
        data = _load(path)
        data[key] = entry
        _store(path, data)
    return dict(entry, cached=False)


def apply_cached_splits(call: str = "evolve", mixer: str = "x", path: str | None = None) -> dict:
    """Put into effect every cached split of (call, mixer) for this device
    and library; returns {n: split}."""
    data = _load(path or cache_path())
    applied = {}
    for n in range(13, 34):
        key = split_signature(call, mixer, n)
        if key in data:
            set_split(n, data[key]["split"])
            applied[n] = tuple(data[key]["split"])
    return applied


# ---------------------------------------------------- batched launch profile
def batch_launch_profile(batch: Batch, full_workgroups: int = 4096) -> dict:
    """Per-launch events over one batched gradient: each launch's duration,
    the gaps between launches, and the time the launches take beyond
    streaming their bytes at the rate of the batch's large launches (those
    with >= full_workgroups workgroups, which fill the GPU many times over):
    the idle tail of launches too small, or too ragged at their end, to fill
    the 256 compute units."""
    import statistics

    lib = _lib.load()
    count = batch.launches
    info = []
    for i in range(count):
        r, w, b = ctypes.c_int(), ctypes.c_int64(), ctypes.c_double()
        _lib.check("qva_batch_launch_info",
                   lib.qva_batch_launch_info(batch._plan, i, ctypes.byref(r), ctypes.byref(w), ctypes.byref(b)))
        info.append((r.value, w.value, b.value))
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
    hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
    evs = []
    for _ in range(2 * count):
        h = ctypes.c_void_p()
        if hip.hipEventCreate(ctypes.byref(h)) != 0:
            raise RuntimeError("hipEventCreate failed")
        evs.append(h.value)
    arr = (ctypes.c_void_p * len(evs))(*evs)
    stream = torch.cuda.current_stream().cuda_stream
    batch.grad()  # warm-up
    torch.cuda.synchronize()
    _lib.check("qva_batch_grad_timed",
               lib.qva_batch_grad_timed(batch._plan, batch.workspace.data_ptr(), batch.workspace.numel(),
                                        arr, len(evs), stream))
    torch.cuda.synchronize()

    def ms(a, b):
        x = ctypes.c_float()
        if hip.hipEventElapsedTime(ctypes.byref(x), evs[a], evs[b]) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return x.value

    dur = [ms(2 * i, 2 * i + 1) for i in range(count)]
    gaps = [ms(2 * i + 1, 2 * i + 2) for i in range(count - 1)]
    total = ms(0, 2 * count - 1)
    for h in evs:
        hip.hipEventDestroy(h)
    big = [b / (d * 1e-3) for (r, w, b), d in zip(info, dur) if w >= full_workgroups and d > 0]
    rate = statistics.median(big) if big else None
    tail = sum(max(0.0, d - b / rate * 1e3) for (r, w, b), d in zip(info, dur)) if rate else None
    rounds = {}
    for (r, w, b), d in zip(info, dur):
        x = rounds.setdefault(r, [0.0, 0, 0.0])
        x[0] += d
        x[1] += w
        x[2] += b
    return {"launches": count, "ms_total": round(total, 3), "ms_in_launches": round(sum(dur), 3),
            "ms_between_launches": round(sum(gaps), 3),
            "full_launch_GBps": round(rate / 1e9, 1) if rate else None,
            "ms_beyond_full_rate": round(tail, 3) if tail is not None else None,
            "idle_tail_fraction": round((tail + sum(gaps)) / total, 4) if tail is not None else None,
            "rounds": {r: {"ms": round(v[0], 4), "workgroups": v[1], "GBps": round(v[2] / (v[0] * 1e-3) / 1e9, 1)}
                       for r, v in sorted(rounds.items())}}
