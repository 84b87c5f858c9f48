"""ctypes front end of plain_loops.c: plain serial binary32 / int64 loops
over the benchmark's operations, timed beside the oracle to separate the
cost of its binary64 reference arithmetic. TIMING BASELINE ONLY (test
infrastructure; nothing is checked against these loops)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "plain_loops.c")
_LIB = os.path.join(_HERE, "libplain.so")
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-Wall", "-Wextra",
                        "-fPIC", "-shared", "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        P, i64, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
        L.plain_triad.argtypes = [i64, P, P, P, ctypes.c_float]
        for f in ("plain_dot_f32", "plain_dot_bf16"):
            getattr(L, f).argtypes = [i64, P, P]
            getattr(L, f).restype = d
        for f in ("plain_sumsq_f32", "plain_sumsq_bf16"):
            getattr(L, f).argtypes = [i64, P]
            getattr(L, f).restype = d
        for f in ("plain_scan_i32_i64", "plain_scan_i32_i32", "plain_scan_f32"):
            getattr(L, f).argtypes = [i64, P, P]
        L.plain_scan_f32_batch.argtypes = [i64, P, P, P, ctypes.c_int]
        L.plain_dot_f32_batch.argtypes = [i64, P, P, P, P]
        L.plain_bcast_mul_batch.argtypes = [i64, P, P, P, P, P, P]
        _lib = L
    return _lib


def ptr(a: np.ndarray) -> int:
    return a.ctypes.data
