"""Launch-shape autotuner: picks the workgroup size (block_threads), the
elements per thread per tile (items_per_thread) and, for scans, the form
(reduce-then-scan or the single-pass look-back) of a call by timing every
shape the library has a kernel for, and caches the choice in a JSON file
keyed by device, algorithm, dtype, op, mode and a size class.

Search space: block_threads in BLOCKS x items_per_thread in ITEMS x the
scan forms in SCAN_FORMS, cut to what dr_tuning_supported accepts (the
look-back scan is built at 256, 512 and 1024 threads; every other kernel
at 256).

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

BLOCKS = (256, 512, 1024)
ITEMS = (4, 8, 16, 32, 64)
SCAN_FORMS = (("two_pass", B.DR_TUNE_TWO_PASS), ("look_back", B.DR_TUNE_TILE_PER_BLOCK))
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


def form_name(flags: int) -> str:
    for name, f in SCAN_FORMS:
        if flags == f:
            return name
    return "default" if flags == 0 else f"flags {flags}"


def label(t: B.dr_tuning) -> str:
    """`256x32/look_back`: block_threads x items_per_thread / form."""
    return f"{t.block_threads}x{t.items_per_thread}/{form_name(t.flags)}"


def candidates(algo: int, view: B.dr_view, out_dtype: int) -> list[B.dr_tuning]:
    """Every (block_threads, items_per_thread, form) the library has a
    kernel for, for this call."""
    forms = SCAN_FORMS if algo in (B.DR_ALGO_SCAN, B.DR_ALGO_SCAN_REDUCE) else (("default", 0),)
    out = []
    for block in BLOCKS:
        for items in ITEMS:
            for _, fl in forms:
                t = B.dr_tuning(block, items, fl, 0)
                if B.lib().dr_tuning_supported(algo, ctypes.byref(view), out_dtype, ctypes.byref(t)):
                    out.append(t)
    return out


def _from_entry(e: dict) -> B.dr_tuning:
    return B.dr_tuning(int(e.get("block_threads", 256)), int(e["items"]), int(e.get("flags", 0)), 0)


def tune(algo: int, view: B.dr_view, out_dtype: int, table: B.Table, call, reps: int = 5,
         extra: str = "") -> B.dr_tuning | None:
    """Return the fastest tuning for `call(tuning)`, timing it on `table`'s
    device the first time this (algo, view, size class) is seen. `call`
    must run the operation once with the given tuning. The cache entry
    (`entry(...)`) keeps every candidate's time."""
    k = key(algo, view, out_dtype, table, extra)
    cache = _load()
    if k in cache:
        return _from_entry(cache[k])
    if torch.cuda.is_current_stream_capturing():
        return None   # never time inside a capture: defaults apply
    cands = candidates(algo, view, out_dtype)
    if not cands:
        return None
    if len(cands) == 1:
        t = cands[0]
        cache[k] = {"block_threads": t.block_threads, "items": t.items_per_thread, "flags": t.flags,
                    "label": label(t), "ms": None}
        _save()
        return t
    stream = torch.cuda.current_stream(table.device)
    best, best_ms, results = None, float("inf"), {}
    for tu in cands:
        call(tu)   # warm-up (and plan)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            call(tu)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        results[label(tu)] = ms
        if ms < best_ms:
            best, best_ms = tu, ms
    cache[k] = {"block_threads": best.block_threads, "items": best.items_per_thread, "flags": best.flags,
                "label": label(best), "ms": best_ms, "all": results}
    _save()
    return best


def entry(algo: int, view: B.dr_view, out_dtype: int, table: B.Table, extra: str = "") -> dict | None:
    """The cached choice (and every candidate's time) for this call, if tuned."""
    return _load().get(key(algo, view, out_dtype, table, extra))
