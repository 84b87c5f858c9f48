"""Tile-shape autotuner: picks items_per_thread (elements per thread per
tile; 256 threads per workgroup) for a call by timing every shape the
library has a kernel for, and caches the choice in a JSON file keyed by
device, algorithm, dtype, op, mode and a size class.

Cache file: $DR_TUNE_CACHE, else ~/.cache/paper_2406_00158_amd/tune.json.
The tuner never runs while a stream is being captured into a graph: tune
first (one eager call), then capture.
"""
from __future__ import annotations

import ctypes
import json
import math
import os

import torch

from . import binding as B

CANDIDATES = (16, 32, 64)
_cache: dict | None = None


def cache_path() -> str:
    p = os.environ.get("DR_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2406_00158_amd", "tune.json")


def _load() -> dict:
    global _cache
    if _cache is None:
        try:
            with open(cache_path()) as f:
                _cache = json.load(f)
        except (OSError, ValueError):
            _cache = {}
    return _cache


def _save() -> None:
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(_cache, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def size_class(n_segments: int, total: int) -> str:
    """Coarse bucket: log2 of the total length and of the segment count."""
    return f"n2^{max(0, int(math.log2(max(total, 1))))}_m2^{max(0, int(math.log2(max(n_segments, 1))))}"


def key(algo: int, view: B.dr_view, out_dtype: int, table: B.Table, extra: str = "") -> str:
    name = torch.cuda.get_device_name(table.device)
    return "|".join([name, str(algo), str(view.in_dtype), str(view.op), str(out_dtype), str(table.mode),
                     size_class(table.n_segments, table.total_length), extra])


def supported(algo: int, view: B.dr_view, out_dtype: int) -> list[int]:
    out = []
    for items in CANDIDATES:
        t = B.make_tuning(items)
        if B.lib().dr_tuning_supported(algo, ctypes.byref(view), out_dtype, ctypes.byref(t)):
            out.append(items)
    return out


def tune(algo: int, view: B.dr_view, out_dtype: int, table: B.Table, call, reps: int = 5,
         extra: str = "") -> B.dr_tuning | None:
    """Return the fastest tuning for `call(tuning)`, timing it on `table`'s
    device the first time this (algo, view, size class) is seen. `call`
    must run the operation once with the given tuning."""
    k = key(algo, view, out_dtype, table, extra)
    cache = _load()
    if k in cache:
        return B.make_tuning(cache[k]["items"])
    if torch.cuda.is_current_stream_capturing():
        return None   # never time inside a capture: defaults apply
    cands = supported(algo, view, out_dtype)
    if len(cands) <= 1:
        cache[k] = {"items": cands[0] if cands else 16, "ms": None}
        _save()
        return B.make_tuning(cache[k]["items"])
    stream = torch.cuda.current_stream(table.device)
    best, best_ms, results = None, float("inf"), {}
    for items in cands:
        tu = B.make_tuning(items)
        call(tu)   # warm-up (and plan)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            call(tu)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        results[items] = ms
        if ms < best_ms:
            best, best_ms = items, ms
    cache[k] = {"items": best, "ms": best_ms, "all": {str(i): v for i, v in results.items()}}
    _save()
    return B.make_tuning(best)
