"""ctypes front end of the plain serial CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product package. It shares no
code with the GPU library; both sides take their inputs from
``paper_2406_00158_amd.inputs`` and nothing else.

Every function takes a list of per-segment numpy arrays (one list per zipped
input) and returns numpy arrays; see oracle.c for the definitions and the
paper passages they follow.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

I32, F32, BF16, F64, I64 = 0, 1, 2, 3, 4
IDENTITY, SQUARE, MUL, AXPY = 0, 1, 2, 3
CONCAT, BATCH = 0, 1
SUM, MAX, MIN = 0, 1, 2
ARITY = {IDENTITY: 1, SQUARE: 1, MUL: 2, AXPY: 2}

_NP_DTYPE = {I32: np.int32, F32: np.float32, BF16: np.uint16, F64: np.float64, I64: np.int64}


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc -O2 -ffp-contract=off)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
                        "-Wall", "-Wextra", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        override = os.environ.get("ORACLE_LIB")   # a separately built copy (mutation checks)
        _lib = ctypes.CDLL(override if override else build())
        PP = ctypes.POINTER(ctypes.c_void_p)
        I64P = ctypes.POINTER(ctypes.c_int64)
        DP = ctypes.POINTER(ctypes.c_double)
        i, d, i64 = ctypes.c_int, ctypes.c_double, ctypes.c_int64
        _lib.oracle_for_each.argtypes = [i, PP, PP, PP, I64P, i, i, d, i]
        _lib.oracle_reduce.argtypes = [i, PP, PP, I64P, i, i, d, i, i64, d, I64P, DP, DP]
        _lib.oracle_scan.argtypes = [i, PP, PP, PP, PP, I64P, i, i, d, i, i, i]
        _lib.oracle_reduce_grad.argtypes = [i, PP, PP, PP, I64P, i, i, d, i, DP, i]
        _lib.oracle_reduce_ex.argtypes = [i, PP, PP, I64P, i, i, d, i, i, i, i64, d, I64P, DP]
        _lib.oracle_scan_ex.argtypes = [i, PP, PP, PP, PP, I64P, i, i, d, i, i, i, i, i, i, i64, d]
        _lib.oracle_black_scholes.argtypes = [i, PP, PP, PP, PP, PP, PP, I64P, d]
        for f in ("oracle_for_each", "oracle_reduce", "oracle_scan", "oracle_reduce_grad"):
            getattr(_lib, f).restype = i
    return _lib


def _ptrs(arrays):
    if arrays is None:
        return None
    return (ctypes.c_void_p * max(1, len(arrays)))(*[a.ctypes.data for a in arrays])


def _prep(segs, dtype):
    want = _NP_DTYPE[dtype]
    out = []
    for a in segs:
        a = np.ascontiguousarray(a)
        if a.dtype != want:
            raise TypeError(f"segment dtype {a.dtype} does not match {want}")
        out.append(a)
    return out


def _lengths(segs):
    return (ctypes.c_int64 * max(1, len(segs)))(*[a.shape[0] for a in segs])


def _check(rc):
    if rc != 0:
        raise ValueError(f"oracle rejected the arguments (code {rc})")


def for_each(in0, in1, in_dtype, op, out_dtype, alpha=0.0):
    """Per-segment output arrays of op(in0, in1) in out_dtype."""
    in0 = _prep(in0, in_dtype)
    in1 = _prep(in1, in_dtype) if in1 is not None else None
    outs = [np.empty(a.shape[0], dtype=_NP_DTYPE[out_dtype]) for a in in0]
    _check(lib().oracle_for_each(len(in0), _ptrs(in0), _ptrs(in1), _ptrs(outs), _lengths(in0),
                                 in_dtype, op, float(alpha), out_dtype))
    return outs


def reduce(in0, in1, in_dtype, op, mode=CONCAT, init=0, alpha=0.0):
    """(results, abs_sums). Integer inputs: int64 results, abs_sums None.
    Floating inputs: binary64 results and the sum of |v| per result."""
    in0 = _prep(in0, in_dtype)
    in1 = _prep(in1, in_dtype) if in1 is not None else None
    nres = len(in0) if mode == BATCH else 1
    if in_dtype == I32:
        res = np.zeros(max(1, nres), dtype=np.int64)
        _check(lib().oracle_reduce(len(in0), _ptrs(in0), _ptrs(in1), _lengths(in0), in_dtype, op,
                                   float(alpha), mode, int(init), 0.0,
                                   res.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), None, None))
        return res[:nres], None
    res = np.zeros(max(1, nres), dtype=np.float64)
    mag = np.zeros(max(1, nres), dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    _check(lib().oracle_reduce(len(in0), _ptrs(in0), _ptrs(in1), _lengths(in0), in_dtype, op,
                               float(alpha), mode, 0, float(init), None,
                               res.ctypes.data_as(dp), mag.ctypes.data_as(dp)))
    return res[:nres], mag[:nres]


def scan(in0, in1, in_dtype, op, mode=CONCAT, reverse=False, out_dtype=None, alpha=0.0,
         want_abs=False):
    """Per-segment scan outputs (and, for floating inputs with want_abs, the
    per-segment running sums of |v|)."""
    in0 = _prep(in0, in_dtype)
    in1 = _prep(in1, in_dtype) if in1 is not None else None
    if out_dtype is None:
        out_dtype = I64 if in_dtype == I32 else F64
    outs = [np.empty(a.shape[0], dtype=_NP_DTYPE[out_dtype]) for a in in0]
    absp = [np.empty(a.shape[0], dtype=np.float64) for a in in0] if want_abs else None
    _check(lib().oracle_scan(len(in0), _ptrs(in0), _ptrs(in1), _ptrs(outs), _ptrs(absp),
                             _lengths(in0), in_dtype, op, float(alpha), mode, int(bool(reverse)),
                             out_dtype))
    return (outs, absp) if want_abs else outs


def reduce_grad(in0, in1, in_dtype, op, g, which, mode=CONCAT, alpha=0.0):
    """Per-segment binary64 gradient of the reduce result(s) with respect to
    input ``which`` (0 or 1), given upstream gradients ``g``."""
    in0 = _prep(in0, in_dtype)
    in1 = _prep(in1, in_dtype) if in1 is not None else None
    g = np.ascontiguousarray(np.atleast_1d(np.asarray(g, dtype=np.float64)))
    outs = [np.empty(a.shape[0], dtype=np.float64) for a in in0]
    _check(lib().oracle_reduce_grad(len(in0), _ptrs(in0), _ptrs(in1), _ptrs(outs), _lengths(in0),
                                    in_dtype, op, float(alpha), mode,
                                    g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), which))
    return outs


def _init_args(in_dtype, init):
    """(has_init, init_i, init_f) for the C calls; init None = the
    operator's identity."""
    if init is None:
        return 0, 0, 0.0
    if in_dtype == I32:
        return 1, int(init), 0.0
    return 1, 0, float(init)


def reduce_ex(in0, in1, in_dtype, op, combine, mode=CONCAT, init=None, alpha=0.0):
    """Per-result reduce with operator `combine` (SUM, MAX, MIN): int64 for
    I32 inputs, binary64 otherwise."""
    in0 = _prep(in0, in_dtype)
    in1 = _prep(in1, in_dtype) if in1 is not None else None
    nres = len(in0) if mode == BATCH else 1
    has, ii, ff = _init_args(in_dtype, init)
    ri = np.zeros(max(1, nres), dtype=np.int64)
    rf = np.zeros(max(1, nres), dtype=np.float64)
    _check(lib().oracle_reduce_ex(len(in0), _ptrs(in0), _ptrs(in1), _lengths(in0), in_dtype, op, float(alpha),
                                  mode, combine, has, ii, ff,
                                  ri.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  rf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return (ri if in_dtype == I32 else rf)[:nres]


def scan_ex(in0, in1, in_dtype, op, combine, mode=CONCAT, reverse=False, exclusive=False, init=None,
            out_dtype=None, alpha=0.0, want_abs=False):
    """Per-segment outputs of the scan with operator `combine`, optional
    init and exclusive form (and, for floating sums with want_abs, the
    running sums of |v| including |init|)."""
    in0 = _prep(in0, in_dtype)
    in1 = _prep(in1, in_dtype) if in1 is not None else None
    if out_dtype is None:
        out_dtype = I64 if in_dtype == I32 else F64
    has, ii, ff = _init_args(in_dtype, init)
    outs = [np.empty(a.shape[0], dtype=_NP_DTYPE[out_dtype]) for a in in0]
    absp = [np.empty(a.shape[0], dtype=np.float64) for a in in0] if want_abs else None
    _check(lib().oracle_scan_ex(len(in0), _ptrs(in0), _ptrs(in1), _ptrs(outs), _ptrs(absp), _lengths(in0),
                                in_dtype, op, float(alpha), mode, int(bool(reverse)), out_dtype, combine,
                                int(bool(exclusive)), has, ii, ff))
    return (outs, absp) if want_abs else outs


def black_scholes(S, K, T, V, r):
    """Per-segment (call, put) binary64 prices of European options for the
    binary32 arrays S (spot), K (strike), T (years), V (volatility) and the
    rate r."""
    S, K, T, V = (_prep(a, F32) for a in (S, K, T, V))
    calls = [np.empty(a.shape[0], dtype=np.float64) for a in S]
    puts = [np.empty(a.shape[0], dtype=np.float64) for a in S]
    _check(lib().oracle_black_scholes(len(S), _ptrs(S), _ptrs(K), _ptrs(T), _ptrs(V), _ptrs(calls), _ptrs(puts),
                                      _lengths(S), float(r)))
    return calls, puts

