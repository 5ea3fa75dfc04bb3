"""Autotuning of the batched engine's launch plan.

The batched gradient groups the passes of all instances into rounds; how
instances are aligned to rounds (all start together, all finish together, or
start rounds spread to even out the tiles per round) changes how well each
launch fills the GPU.  `tune_batch` times each candidate on the actual
instances and caches the winner in a JSON file keyed by the batch's shape
(the multiset of (n, p)), the device name and the library version.

Cache file: $QVA_TUNE_CACHE, else ~/.cache/qva/tune.json.
"""

from __future__ import annotations

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


def tune_batch(qs, gammas, ts, *, candidates=CANDIDATES, reps: int = 2, use_cache: bool = True,
               path: str | None = None) -> dict:
    """Pick the round alignment with the shortest batched gradient.

    Returns {"align": best, "ms": {candidate: time}, "cached": bool}.
    """
    path = path or cache_path()
    ns = [int(q.numel()).bit_length() - 1 for q in qs]
    ps = [len(g) for g in gammas]
    key = batch_signature(ns, ps)
    data = _load(path) if use_cache else {}
    if use_cache and key in data and data[key].get("align") in candidates:
        out = dict(data[key])
        out["cached"] = True
        return out
    times = {}
    for align in candidates:
        b = Batch(qs, gammas, ts, align=align)
        times[align] = time_batch_grad(b, reps=reps)
        del b
        torch.cuda.empty_cache()
    best = min(times, key=times.get)
    entry = {"align": best, "ms": times}
    if use_cache:
        data = _load(path)
        data[key] = entry
        _store(path, data)
    return dict(entry, cached=False)
