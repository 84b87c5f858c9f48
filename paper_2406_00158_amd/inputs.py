"""Seeded synthetic inputs for the segmented for_each / transform_reduce /
inclusive_scan path.

This module only draws numbers and splits lengths: it holds none of the
arithmetic of the method (no sums, scans or views). Both the CPU oracle's
tests and the GPU parity tests take their inputs from here, so the two sides
see the same stored values and share nothing else.

Workload shapes follow the paper's benchmarks (section 5.1: dot product,
reduce, inclusive scan and stream over a block-distributed vector, section
4.2) at the sizes of the five workloads used throughout this package:

  * ``tiny``      2^20 FP32 pairs U[-1,1), 4 unequal segments (40/25/20/15 %),
                  plus int32 U{0..100} for the scan.
  * ``triad``     stream triad a = b + 3c and dot(b, c), FP32, 2^28, 8 equal
                  segments.
  * ``scan``      int32 U{0..100} over 2^30 in 16 Dirichlet(1) segments, and
                  FP32 N(0,1) over 2^28 in its own 16 Dirichlet(1) segments.
  * ``precision`` 2^29 values from a 50/50 mixture of |N(0,1)| and
                  lognormal(0, 4) with random signs, stored FP32 and BF16.
  * ``batch``     10,000 ragged FP32 N(0,1) ranges, log-uniform lengths
                  rescaled to a total of 2^28.

Every generator takes an explicit seed (numpy PCG64); the default seeds are
1000 + the workload number (1..5).
"""
from __future__ import annotations

import math
import os

import numpy as np

SEED_TINY = 1001
SEED_TRIAD = 1002
SEED_SCAN = 1003
SEED_PRECISION = 1004
SEED_BATCH = 1005


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# Segment lengths
# ---------------------------------------------------------------------------

def lengths_block(n: int, p: int) -> list[int]:
    """Block partition of a distributed vector (section 4.2.1): p segments of
    ceil(n/p) elements, the last ones shorter (possibly empty)."""
    if p <= 0:
        raise ValueError("p must be positive")
    b = -(-n // p) if n else 0
    out = []
    left = n
    for _ in range(p):
        take = min(b, left)
        out.append(take)
        left -= take
    return out


def lengths_fractions(n: int, fracs: list[float]) -> list[int]:
    """floor(f * n) for every fraction but the last; the last takes the rest."""
    out = [int(math.floor(f * n)) for f in fracs[:-1]]
    out.append(n - sum(out))
    if out[-1] < 0:
        raise ValueError("fractions exceed 1")
    return out


def lengths_dirichlet(n: int, m: int, alpha: float, seed: int) -> list[int]:
    """Segment sizes from a Dirichlet(alpha) draw, rounded by largest
    remainder so that they sum to n exactly."""
    g = rng(seed)
    p = g.dirichlet([alpha] * m)
    raw = p * n
    base = np.floor(raw).astype(np.int64)
    rem = n - int(base.sum())
    order = np.argsort(-(raw - base), kind="stable")
    base[order[:rem]] += 1
    return [int(v) for v in base]


def lengths_loguniform(count: int, max_len: int, total: int, seed: int,
                       rescale: bool = True) -> list[int]:
    """Ragged range lengths: floor(exp(U(0, ln(max_len + 1)))), then (when
    ``rescale``) scaled so the lengths sum to ``total`` exactly: rounded,
    clamped to >= 1, the difference put into the longest range."""
    g = rng(seed)
    raw = np.floor(np.exp(g.uniform(0.0, math.log(max_len + 1), size=count)))
    raw = np.maximum(raw, 1.0)
    if not rescale:
        return [int(v) for v in raw]
    scaled = np.maximum(np.rint(raw * (total / raw.sum())), 1).astype(np.int64)
    diff = total - int(scaled.sum())
    k = int(np.argmax(scaled))
    scaled[k] += diff
    if scaled[k] < 1:
        raise ValueError("cannot rescale lengths to the requested total")
    return [int(v) for v in scaled]


def split(arr: np.ndarray, lengths: list[int]) -> list[np.ndarray]:
    """Views of consecutive pieces of ``arr`` with the given lengths."""
    out, o = [], 0
    for n in lengths:
        out.append(arr[o:o + n])
        o += n
    if o != arr.shape[0]:
        raise ValueError("lengths do not cover the array")
    return out


# ---------------------------------------------------------------------------
# Values
# ---------------------------------------------------------------------------

def uniform_f32(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return rng(seed).uniform(lo, hi, size=n).astype(np.float32)


def normal_f32(n: int, seed: int) -> np.ndarray:
    return rng(seed).standard_normal(size=n, dtype=np.float32)


def ints_0_100(n: int, seed: int) -> np.ndarray:
    """int32 uniform on {0, ..., 100} (both ends included)."""
    return rng(seed).integers(0, 100, size=n, endpoint=True, dtype=np.int32)


def mixture_f32(n: int, seed: int) -> np.ndarray:
    """50/50 mixture of |N(0,1)| and lognormal(0, 4), times an independent
    random sign: per element one binary32 standard normal z and two random
    bits, b0 choosing |z| or exp(4 z), b1 the sign. Block b of 2^24
    elements draws from its own PCG64 stream seeded by (seed, b), so the
    blocks are generated on several threads and the values do not depend
    on how many."""
    out = np.empty(n, dtype=np.float32)
    block = 1 << 24

    def fill(o: int) -> None:
        g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, o // block])))
        m = min(block, n - o)
        z = g.standard_normal(size=m, dtype=np.float32)
        bits = g.integers(0, 4, size=m, dtype=np.uint8)
        mag = np.where(bits & 1, np.abs(z), np.exp(np.float32(4.0) * z))
        out[o:o + m] = np.where(bits & 2, -mag, mag)

    starts = range(0, n, block)
    if len(starts) > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=min(len(starts), os.cpu_count() or 1, 16)) as ex:
            list(ex.map(fill, starts))
    else:
        for o in starts:
            fill(o)
    return out


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to bfloat16 (round to nearest, ties to even) and
    return the 16-bit patterns as uint16. NaN stays a quiet NaN."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    lsb = (b >> np.uint32(16)) & np.uint32(1)
    # uint32 arithmetic wraps only for NaN patterns, which are set below
    rounded = (b + np.uint32(0x7FFF) + lsb) >> np.uint32(16)
    out = rounded.astype(np.uint16)
    nan = np.isnan(x)
    if nan.any():
        out[nan] = ((b[nan] >> np.uint32(16)) | np.uint32(0x40)).astype(np.uint16)
    return out


def bf16_to_f32(bits: np.ndarray) -> np.ndarray:
    """The FP32 value of each bfloat16 pattern (exact)."""
    return (bits.astype(np.uint32) << np.uint32(16)).view(np.float32)


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

TINY_N = 1 << 20
TINY_FRACS = [0.40, 0.25, 0.20, 0.15]


def tiny(n: int = TINY_N, seed: int = SEED_TINY) -> dict:
    """2^20 FP32 x, y U[-1,1) and int32 U{0..100}, 4 unequal segments."""
    return {
        "lengths": lengths_fractions(n, TINY_FRACS),
        "x": uniform_f32(n, seed),
        "y": uniform_f32(n, seed + 100),
        "k": ints_0_100(n, seed + 200),
    }


TRIAD_N = 1 << 28
TRIAD_SEGMENTS = 8
TRIAD_SCALAR = 3.0


def triad(n: int = TRIAD_N, segments: int = TRIAD_SEGMENTS, seed: int = SEED_TRIAD) -> dict:
    """Stream triad inputs: b, c FP32 U[-1,1), equal segments, s = 3."""
    return {
        "lengths": lengths_block(n, segments),
        "b": uniform_f32(n, seed),
        "c": uniform_f32(n, seed + 100),
        "s": TRIAD_SCALAR,
    }


SCAN_INT_N = 1 << 30
SCAN_FP_N = 1 << 28
SCAN_SEGMENTS = 16


def scan_int(n: int = SCAN_INT_N, segments: int = SCAN_SEGMENTS, seed: int = SEED_SCAN) -> dict:
    return {"lengths": lengths_dirichlet(n, segments, 1.0, seed),
            "k": ints_0_100(n, seed + 100)}


def scan_fp(n: int = SCAN_FP_N, segments: int = SCAN_SEGMENTS, seed: int = SEED_SCAN) -> dict:
    return {"lengths": lengths_dirichlet(n, segments, 1.0, seed + 1),
            "x": normal_f32(n, seed + 200)}


PRECISION_N = 1 << 29
PRECISION_SEGMENTS = 8


def precision(n: int = PRECISION_N, segments: int = PRECISION_SEGMENTS,
              seed: int = SEED_PRECISION) -> dict:
    x = mixture_f32(n, seed)
    y = mixture_f32(n, seed + 100)
    return {"lengths": lengths_block(n, segments), "x": x, "y": y,
            "x_bf16": bf16_bits(x), "y_bf16": bf16_bits(y)}


BATCH_RANGES = 10_000
BATCH_MAX_LEN = 1 << 20
BATCH_TOTAL = 1 << 28


def batch(count: int = BATCH_RANGES, total: int = BATCH_TOTAL, max_len: int = BATCH_MAX_LEN,
          seed: int = SEED_BATCH) -> dict:
    lengths = lengths_loguniform(count, max_len, total, seed)
    n = sum(lengths)
    return {"lengths": lengths, "x": normal_f32(n, seed + 100),
            "y": normal_f32(n, seed + 200)}


OPTIONS_N = 1 << 28
OPTIONS_SEGMENTS = 8
OPTIONS_RATE = 0.02
SEED_OPTIONS = 1006


def options(n: int = OPTIONS_N, segments: int = OPTIONS_SEGMENTS, seed: int = SEED_OPTIONS) -> dict:
    """European options for the Black-Scholes for_each: binary32 spot S and
    strike K U[10, 50), time to expiry T U[0.1, 2) years, volatility
    V U[0.1, 0.5), one risk-free rate; equal segments."""
    g = rng(seed)
    return {"lengths": lengths_block(n, segments),
            "S": g.uniform(10.0, 50.0, size=n).astype(np.float32),
            "K": g.uniform(10.0, 50.0, size=n).astype(np.float32),
            "T": g.uniform(0.1, 2.0, size=n).astype(np.float32),
            "V": g.uniform(0.1, 0.5, size=n).astype(np.float32),
            "r": OPTIONS_RATE}
