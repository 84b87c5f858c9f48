"""The serial oracle run on every host core: the CPU baseline the benchmark
times next to the GPU (TEST INFRASTRUCTURE, like the rest of oracle/).

Each call cuts its work into one contiguous piece per thread and runs the
oracle's own C functions (oracle.c, through ``oracle``) on the pieces in a
thread pool; ctypes releases the interpreter lock for the duration of a C
call, so the pieces run in parallel. The pieces are joined in order:

  * for_each and the adjoint: independent pieces;
  * reduce (one range): the pieces' binary64 partials added with math.fsum,
    their int64 partials exactly;
  * scan (one range): every piece's total first (a reduce), then every piece
    scanned with the total of the pieces before it as its initial value;
  * BATCH calls: groups of whole ranges, one group per thread.

The results equal the serial oracle's (integers) or lie within its own
rounding (binary64); the benchmark uses them for timing only.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle as O


def threads() -> int:
    """Host threads the twin uses: every core this process may run on."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return max(1, os.cpu_count() or 1)


_POOL = None


def _pool() -> ThreadPoolExecutor:
    global _POOL
    if _POOL is None:
        _POOL = ThreadPoolExecutor(max_workers=threads())
    return _POOL


def _bounds(n: int, parts: int) -> list[tuple[int, int]]:
    step = -(-n // parts) if n else 0
    return [(o, min(o + step, n)) for o in range(0, n, step)] if n else []


def _groups(lengths: list[int], parts: int) -> list[tuple[int, int]]:
    """Consecutive ranges [k0, k1) of about equal element counts."""
    total = sum(lengths)
    target = total / parts if parts else total
    out, k0, acc = [], 0, 0
    for k, n in enumerate(lengths):
        acc += n
        if acc >= target * (len(out) + 1) and k + 1 < len(lengths):
            out.append((k0, k + 1))
            k0 = k + 1
    out.append((k0, len(lengths)))
    return out


def for_each(x: np.ndarray, y, in_dtype: int, op: int, out_dtype: int, alpha: float = 0.0) -> np.ndarray:
    out = np.empty(x.shape[0], dtype=O._NP_DTYPE[out_dtype])

    def piece(b):
        lo, hi = b
        out[lo:hi] = O.for_each([x[lo:hi]], [y[lo:hi]] if y is not None else None, in_dtype, op, out_dtype,
                                alpha=alpha)[0]
    list(_pool().map(piece, _bounds(x.shape[0], threads())))
    return out


def reduce(x: np.ndarray, y, in_dtype: int, op: int, alpha: float = 0.0):
    def piece(b):
        lo, hi = b
        return O.reduce([x[lo:hi]], [y[lo:hi]] if y is not None else None, in_dtype, op, alpha=alpha)[0][0]
    parts = list(_pool().map(piece, _bounds(x.shape[0], threads())))
    return int(sum(int(p) for p in parts)) if in_dtype == O.I32 else math.fsum(parts)


def scan(x: np.ndarray, in_dtype: int, out_dtype=None) -> np.ndarray:
    """Inclusive sum scan of the identity view over one range."""
    if out_dtype is None:
        out_dtype = O.I64 if in_dtype == O.I32 else O.F64
    bounds = _bounds(x.shape[0], threads())
    totals = list(_pool().map(lambda b: O.reduce([x[b[0]:b[1]]], None, in_dtype, O.IDENTITY)[0][0], bounds))
    carries, run = [], 0
    for t in totals:
        carries.append(run)
        run = run + (int(t) if in_dtype == O.I32 else float(t))
    out = np.empty(x.shape[0], dtype=O._NP_DTYPE[out_dtype])

    def piece(i):
        lo, hi = bounds[i]
        out[lo:hi] = O.scan_ex([x[lo:hi]], None, in_dtype, O.IDENTITY, O.SUM, init=carries[i],
                               out_dtype=out_dtype)[0]
    list(_pool().map(piece, range(len(bounds))))
    return out


def _batch(fn, lengths: list[int]):
    groups = _groups(lengths, threads())
    return list(_pool().map(fn, groups))


def scan_batch(x: np.ndarray, lengths: list[int], reverse: bool = False) -> None:
    """Per-range inclusive sum scans (BATCH), binary64 references."""
    offs = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)

    def piece(g):
        k0, k1 = g
        O.scan(O_split(x, offs, k0, k1), None, O.F32, O.IDENTITY, mode=O.BATCH, reverse=reverse)
    _batch(piece, lengths)


def reduce_batch(x: np.ndarray, y: np.ndarray, lengths: list[int]) -> None:
    offs = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)

    def piece(g):
        k0, k1 = g
        O.reduce(O_split(x, offs, k0, k1), O_split(y, offs, k0, k1), O.F32, O.MUL, mode=O.BATCH)
    _batch(piece, lengths)


def reduce_grad_batch(x: np.ndarray, y: np.ndarray, lengths: list[int], g: np.ndarray, which: int) -> None:
    offs = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)

    def piece(gr):
        k0, k1 = gr
        O.reduce_grad(O_split(x, offs, k0, k1), O_split(y, offs, k0, k1), O.F32, O.MUL, g[k0:k1], which,
                      mode=O.BATCH)
    _batch(piece, lengths)


def O_split(a: np.ndarray, offs: np.ndarray, k0: int, k1: int) -> list[np.ndarray]:
    return [a[offs[k]:offs[k + 1]] for k in range(k0, k1)]
