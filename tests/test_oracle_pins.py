"""Pins for the CPU oracle: it is checked against things other than itself
(hand-worked examples of the paper's algorithms, closed forms, brute force
in exact rational arithmetic, correctly rounded sums, numpy's float32
arithmetic, invariants of the segmented model). CPU only."""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from paper_2406_00158_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.jsonl")
U64 = 2.0 ** -53

OPS = {"identity": O.IDENTITY, "square": O.SQUARE, "mul": O.MUL, "axpy": O.AXPY}


def _load_golden():
    with open(GOLDEN) as f:
        return [json.loads(line) for line in f if line.strip()]


def _rand_segmentation(n, rng, max_segments=12, empty_prob=0.2):
    """Random split of n elements into segments, with empty ones sprinkled in."""
    k = int(rng.integers(1, max_segments + 1))
    cuts = sorted(int(c) for c in rng.integers(0, n + 1, size=k - 1))
    lengths = [b - a for a, b in zip([0] + cuts, cuts + [n])]
    out = []
    for L in lengths:
        if rng.random() < empty_prob:
            out.append(0)
        out.append(L)
    return out


# ---------------------------------------------------------------------------
# Hand-worked examples of the paper's algorithms (tests/golden)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", _load_golden(), ids=lambda c: c["name"])
def test_golden_worked_examples(case):
    mode = O.BATCH if case.get("mode") == "batch" else O.CONCAT
    algo = case["algo"]
    if algo == "for_each":
        a = [np.array(s, dtype=np.float32) for s in case["segments"]]
        b = [np.array(s, dtype=np.float32) for s in case["segments_b"]]
        out = O.for_each(a, b, O.F32, OPS[case["op"]], O.F32, alpha=case["alpha"])
        assert [o.tolist() for o in out] == case["expect"]
        return
    segs = [np.array(s, dtype=np.int32) for s in case["segments"]]
    if algo == "scan":
        out = O.scan(segs, None, O.I32, O.IDENTITY, mode=mode, reverse=case.get("reverse", False))
        assert [o.tolist() for o in out] == case["expect"]
        steps = case.get("steps")
        if steps:
            # the fixture's own intermediate steps agree with the paper's recipe
            assert [list(itertools.accumulate(s)) for s in case["segments"]] == steps["local"]
            assert [loc[-1] for loc in steps["local"]] == steps["totals"]
            assert list(itertools.accumulate(steps["totals"])) == steps["scanned_totals"]
            assert [0] + steps["scanned_totals"][:-1] == steps["offsets"]
    elif algo == "reduce":
        b = [np.array(s, dtype=np.int32) for s in case["segments_b"]] if "segments_b" in case else None
        res, _ = O.reduce(segs, b, O.I32, OPS[case["op"]], mode=mode, init=case.get("init", 0))
        assert res.tolist() == case["expect"]
        # the FP path agrees on the same small integers
        fs = [s.astype(np.float32) for s in segs]
        fb = [s.astype(np.float32) for s in b] if b is not None else None
        resf, _ = O.reduce(fs, fb, O.F32, OPS[case["op"]], mode=mode, init=case.get("init", 0))
        assert resf.tolist() == [float(v) for v in case["expect"]]


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------

def test_scan_of_ones_is_iota_under_any_segmentation():
    rng = np.random.default_rng(7)
    n = 100_003
    ones = np.ones(n, dtype=np.int32)
    for _ in range(5):
        lens = _rand_segmentation(n, rng)
        out = O.scan(I.split(ones, lens), None, O.I32, O.IDENTITY)
        assert np.array_equal(np.concatenate(out), np.arange(1, n + 1, dtype=np.int64))
        rev = O.scan(I.split(ones, lens), None, O.I32, O.IDENTITY, reverse=True)
        assert np.array_equal(np.concatenate(rev), np.arange(n, 0, -1, dtype=np.int64))


def test_scan_of_constant():
    n, c = 50_000, 37
    x = np.full(n, c, dtype=np.int32)
    out = O.scan(I.split(x, [n // 3, 0, n - n // 3]), None, O.I32, O.IDENTITY)
    assert np.array_equal(np.concatenate(out), c * np.arange(1, n + 1, dtype=np.int64))


def test_int32_wrap_output_is_int64_mod_2_32():
    # constant 2^30 overflows int32 after two elements
    n = 10
    x = np.full(n, 1 << 30, dtype=np.int32)
    out = O.scan([x], None, O.I32, O.IDENTITY, out_dtype=O.I32)[0]
    want = [((k + 1) * (1 << 30) + 2 ** 31) % 2 ** 32 - 2 ** 31 for k in range(n)]
    assert out.tolist() == want


def test_sum_of_arithmetic_sequence():
    n = 1 << 20
    x = np.arange(n, dtype=np.int32)
    res, _ = O.reduce(I.split(x, I.lengths_fractions(n, I.TINY_FRACS)), None, O.I32, O.IDENTITY,
                      init=5)
    assert int(res[0]) == n * (n - 1) // 2 + 5
    # FP: i is exact in float32 below 2^24, and so is the sum in binary64
    xf = x.astype(np.float32)
    resf, mag = O.reduce(I.split(xf, I.lengths_fractions(n, I.TINY_FRACS)),
                         I.split(np.ones(n, np.float32), I.lengths_fractions(n, I.TINY_FRACS)),
                         O.F32, O.MUL)
    assert resf[0] == n * (n - 1) / 2 and mag[0] == n * (n - 1) / 2


def test_fp_scan_of_ones_is_exact():
    n = 1 << 18
    x = np.ones(n, dtype=np.float32)
    out = O.scan(I.split(x, I.lengths_block(n, 7)), None, O.F32, O.IDENTITY)
    assert np.array_equal(np.concatenate(out), np.arange(1, n + 1, dtype=np.float64))


def test_sum_of_squares_closed_form():
    n = 3000
    x = np.arange(1, n + 1, dtype=np.int32)
    res, _ = O.reduce([x[:1000], x[1000:]], None, O.I32, O.SQUARE)
    assert int(res[0]) == n * (n + 1) * (2 * n + 1) // 6


# ---------------------------------------------------------------------------
# Brute force on tiny inputs, exact rational arithmetic
# ---------------------------------------------------------------------------

def _compositions(n):
    """Every way to cut n elements into non-empty consecutive segments."""
    for mask in range(1 << max(0, n - 1)):
        lens, run = [], 1
        for b in range(n - 1):
            if mask >> b & 1:
                lens.append(run)
                run = 1
            else:
                run += 1
        lens.append(run if n else 0)
        yield lens


def _view_exact(op, a, b, alpha):
    if op == O.IDENTITY:
        return a
    if op == O.SQUARE:
        return a * a
    if op == O.MUL:
        return a * b
    return a + alpha * b


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_brute_force_all_segmentations(n):
    rng = np.random.default_rng(100 + n)
    xi = rng.integers(-50, 51, size=n).astype(np.int32)
    yi = rng.integers(-50, 51, size=n).astype(np.int32)
    xf = rng.standard_normal(n).astype(np.float32)
    yf = rng.standard_normal(n).astype(np.float32)
    alpha = 3.0
    for lens in _compositions(n):
        for with_empty in (False, True):
            L = list(lens)
            if with_empty:
                L = [0] + [v for l in L for v in (l, 0)]
            for op in (O.IDENTITY, O.SQUARE, O.MUL, O.AXPY):
                b_i = I.split(yi, L) if O.ARITY[op] == 2 else None
                b_f = I.split(yf, L) if O.ARITY[op] == 2 else None
                # exact per-element values
                vi = [_view_exact(op, int(a), int(b), 3) for a, b in zip(xi, yi)]
                vf = [_view_exact(op, Fraction(float(a)), Fraction(float(b)), Fraction(alpha))
                      for a, b in zip(xf, yf)]
                for mode in (O.CONCAT, O.BATCH):
                    # direct loops over the flat range / per range
                    groups = [list(range(o, o + l)) for o, l in
                              zip(itertools.accumulate([0] + L[:-1]), L)]
                    if mode == O.CONCAT:
                        want_r = [sum(vi)]
                        want_rf = [sum(vf, Fraction(0))]
                    else:
                        want_r = [sum(vi[i] for i in g) for g in groups]
                        want_rf = [sum((vf[i] for i in g), Fraction(0)) for g in groups]
                    r, _ = O.reduce(I.split(xi, L), b_i, O.I32, op, mode=mode, alpha=alpha)
                    assert r.tolist() == want_r
                    rf, _ = O.reduce(I.split(xf, L), b_f, O.F32, op, mode=mode, alpha=alpha)
                    for got, want in zip(rf.tolist(), want_rf):
                        assert abs(Fraction(got) - want) <= Fraction(2 * U64) * abs(want)
                    for rev in (False, True):
                        want_s = []
                        order_groups = groups if mode == O.BATCH else [list(range(n))]
                        flat = [0] * n
                        flat_f = [Fraction(0)] * n
                        for g in order_groups:
                            idx = g[::-1] if rev else g
                            acc, accf = 0, Fraction(0)
                            for i in idx:
                                acc += vi[i]
                                accf += vf[i]
                                flat[i] = acc
                                flat_f[i] = accf
                        s = O.scan(I.split(xi, L), b_i, O.I32, op, mode=mode, reverse=rev,
                                   alpha=alpha)
                        assert np.concatenate(s).tolist() == flat
                        sf = O.scan(I.split(xf, L), b_f, O.F32, op, mode=mode, reverse=rev,
                                    alpha=alpha)
                        for got, want in zip(np.concatenate(sf).tolist(), flat_f):
                            assert abs(Fraction(got) - want) <= Fraction(2 * U64) * abs(want) + \
                                Fraction(1, 2 ** 200)
                        del want_s


# ---------------------------------------------------------------------------
# Invariants of the segmented model
# ---------------------------------------------------------------------------

def test_integer_segmentation_invariance():
    rng = np.random.default_rng(11)
    n = 200_000
    x = I.ints_0_100(n, 3)
    y = I.ints_0_100(n, 4)
    ref_scan = None
    ref_red = None
    for _ in range(6):
        L = _rand_segmentation(n, rng, max_segments=40)
        s = np.concatenate(O.scan(I.split(x, L), None, O.I32, O.IDENTITY))
        r, _ = O.reduce(I.split(x, L), I.split(y, L), O.I32, O.MUL)
        if ref_scan is None:
            ref_scan, ref_red = s, int(r[0])
        assert np.array_equal(s, ref_scan)
        assert int(r[0]) == ref_red


def test_batch_equals_per_range_concat():
    rng = np.random.default_rng(12)
    n = 30_000
    x = I.normal_f32(n, 5)
    y = I.normal_f32(n, 6)
    L = _rand_segmentation(n, rng, max_segments=20)
    rb, _ = O.reduce(I.split(x, L), I.split(y, L), O.F32, O.MUL, mode=O.BATCH)
    sb = O.scan(I.split(x, L), None, O.F32, O.IDENTITY, mode=O.BATCH)
    for k, (a, b) in enumerate(zip(I.split(x, L), I.split(y, L))):
        rc, _ = O.reduce([a], [b], O.F32, O.MUL)
        assert rb[k] == rc[0]
        sc = O.scan([a], None, O.F32, O.IDENTITY)[0]
        assert np.array_equal(sb[k], sc)


def test_scan_and_reduce_agree():
    n = 77_777
    x = I.ints_0_100(n, 9)
    L = I.lengths_dirichlet(n, 16, 1.0, 9)
    s = np.concatenate(O.scan(I.split(x, L), None, O.I32, O.IDENTITY))
    r, _ = O.reduce(I.split(x, L), None, O.I32, O.IDENTITY)
    assert s[-1] == r[0]
    assert np.array_equal(np.diff(s), x[1:].astype(np.int64))
    assert s[0] == x[0]
    assert np.all(np.diff(s) >= 0)


# ---------------------------------------------------------------------------
# Binary64 references against correctly rounded sums (math.fsum)
# ---------------------------------------------------------------------------

def test_fp_reduce_matches_fsum_on_ill_conditioned_data():
    n = 1 << 17
    x = I.mixture_f32(n, 21)
    y = I.mixture_f32(n, 22)
    L = I.lengths_block(n, 8)
    r, mag = O.reduce(I.split(x, L), I.split(y, L), O.F32, O.MUL)
    prods = [float(a) * float(b) for a, b in zip(x.tolist(), y.tolist())]   # exact in binary64
    want = math.fsum(prods)
    assert abs(r[0] - want) <= 4 * U64 * abs(want)
    assert abs(mag[0] - math.fsum(abs(p) for p in prods)) <= 4 * U64 * mag[0]
    # BF16 storage: decode exact, products exact
    xb, yb = I.bf16_bits(x), I.bf16_bits(y)
    rb, _ = O.reduce(I.split(xb, L), I.split(yb, L), O.BF16, O.MUL)
    xd, yd = I.bf16_to_f32(xb).tolist(), I.bf16_to_f32(yb).tolist()
    wantb = math.fsum(float(a) * float(b) for a, b in zip(xd, yd))
    assert abs(rb[0] - wantb) <= 4 * U64 * abs(wantb)


def test_fp_scan_matches_fsum_prefixes():
    n = 1 << 15
    x = I.normal_f32(n, 23)
    L = I.lengths_dirichlet(n, 16, 1.0, 23)
    out, absp = O.scan(I.split(x, L), None, O.F32, O.IDENTITY, want_abs=True)
    s = np.concatenate(out)
    a = np.concatenate(absp)
    xs = x.tolist()
    for i in list(range(0, n, 997)) + [n - 1]:
        want = math.fsum(xs[:i + 1])
        assert abs(s[i] - want) <= 2 * U64 * abs(want) + 4 * U64 * U64 * a[i] * (i + 1)
        assert abs(a[i] - math.fsum(abs(v) for v in xs[:i + 1])) <= 2 * U64 * a[i]


def test_sum_of_squares_precision_data():
    n = 1 << 16
    x = I.mixture_f32(n, 31)
    r, mag = O.reduce([x], None, O.F32, O.SQUARE)
    want = math.fsum(float(v) * float(v) for v in x.tolist())
    assert abs(r[0] - want) <= 2 * U64 * want
    assert r[0] == mag[0]


# ---------------------------------------------------------------------------
# for_each: triad rounding, bf16 decode, integer wrap
# ---------------------------------------------------------------------------

def test_triad_is_two_roundings_like_numpy_float32():
    n = 1 << 16
    t = I.triad(n=n, segments=8)
    L = t["lengths"]
    out = np.concatenate(O.for_each(I.split(t["b"], L), I.split(t["c"], L), O.F32, O.AXPY, O.F32,
                                    alpha=t["s"]))
    want = t["b"] + np.float32(t["s"]) * t["c"]     # numpy float32: one rounding per op
    assert want.dtype == np.float32
    assert np.array_equal(out.view(np.uint32), want.view(np.uint32))
    # and it is not the single-rounding (fused) result everywhere
    fused = (t["b"].astype(np.float64) + 3.0 * t["c"].astype(np.float64)).astype(np.float32)
    assert np.any(fused.view(np.uint32) != out.view(np.uint32))


def test_binary64_for_each_is_numpy_float64_arithmetic():
    """The binary64 branch: every op is numpy's float64 arithmetic with one
    rounding per operation (axpy = fl(x + fl(alpha * y)), never fused),
    bit for bit, over several segmentations and special values."""
    rng = np.random.default_rng(61)
    n = 4099
    x = rng.standard_normal(n) * np.exp(rng.uniform(-30, 30, n))
    y = rng.standard_normal(n) * np.exp(rng.uniform(-30, 30, n))
    x[:6] = [0.0, -0.0, np.inf, -np.inf, np.nan, 5e-324]
    y[:6] = [1.0, np.inf, -2.0, 0.0, 1.0, 3.0]
    alpha = 0.1   # not a power of two: alpha * y rounds
    with np.errstate(invalid="ignore", over="ignore"):
        want = {O.IDENTITY: x.copy(), O.SQUARE: x * x, O.MUL: x * y, O.AXPY: x + alpha * y}
    for L in ([n], [1, 0, 2048, 2050], I.lengths_dirichlet(n, 7, 1.0, 62)):
        for op, w in want.items():
            b = I.split(y, L) if O.ARITY[op] == 2 else None
            got = np.concatenate(O.for_each(I.split(x, L), b, O.F64, op, O.F64, alpha=alpha))
            assert got.dtype == np.float64
            assert np.array_equal(got.view(np.uint64), w.view(np.uint64)), (op, L)
    # and axpy is not the singly rounded (fused) result everywhere
    fused = [float(Fraction(a) + Fraction(alpha) * Fraction(b)) for a, b in zip(x[6:400], y[6:400])]
    assert np.any(np.array(fused) != want[O.AXPY][6:400])


def test_bf16_decode_known_patterns():
    bits = np.array([0x3F80, 0xC000, 0x4049, 0x7F80, 0xFF80, 0x0001, 0x8000], dtype=np.uint16)
    out = O.for_each([bits], None, O.BF16, O.IDENTITY, O.F32)[0]
    want = [1.0, -2.0, 3.140625, math.inf, -math.inf, 2.0 ** -133, -0.0]
    assert out.tolist() == want
    assert math.copysign(1.0, out[-1]) == -1.0


def test_bf16_rne_rounding_of_inputs():
    # ties to even: 1 + 2^-8 (exactly half an ulp of bf16 at 1) rounds to 1;
    # 1 + 3*2^-8 rounds up to 1 + 2^-6... (1 + 2^-7 + 2^-8 -> 1 + 2^-6)
    vals = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -1.5], dtype=np.float32)
    got = I.bf16_to_f32(I.bf16_bits(vals)).tolist()
    assert got == [1.0, 1 + 2 ** -6, 1 + 2 ** -7, -1.5]


def test_integer_for_each_wraps():
    x = np.array([70000, -3, 46341], dtype=np.int32)
    out32 = O.for_each([x], None, O.I32, O.SQUARE, O.I32)[0]
    out64 = O.for_each([x], None, O.I32, O.SQUARE, O.I64)[0]
    assert out64.tolist() == [70000 ** 2, 9, 46341 ** 2]
    assert out32.tolist() == [(v + 2 ** 31) % 2 ** 32 - 2 ** 31 for v in out64.tolist()]


# ---------------------------------------------------------------------------
# Adjoints
# ---------------------------------------------------------------------------

def test_dot_gradient_with_unit_upstream_is_the_other_operand():
    n = 1000
    x = I.normal_f32(n, 41)
    y = I.normal_f32(n, 42)
    L = [300, 0, 700]
    gx = np.concatenate(O.reduce_grad(I.split(x, L), I.split(y, L), O.F32, O.MUL, [1.0], 0))
    gy = np.concatenate(O.reduce_grad(I.split(x, L), I.split(y, L), O.F32, O.MUL, [1.0], 1))
    assert np.array_equal(gx, y.astype(np.float64))
    assert np.array_equal(gy, x.astype(np.float64))


def test_gradients_match_central_differences():
    rng = np.random.default_rng(43)
    L = [1, 7, 56]
    n = sum(L)
    x = rng.standard_normal(n)
    y = rng.standard_normal(n)
    g = rng.standard_normal(len(L))
    h = 1e-6
    for op, which in ((O.MUL, 0), (O.MUL, 1), (O.SQUARE, 0), (O.AXPY, 1)):
        b = I.split(y, L) if O.ARITY[op] == 2 else None
        grad = np.concatenate(O.reduce_grad(I.split(x, L), b, O.F64, op, g, which, mode=O.BATCH,
                                            alpha=2.5))
        for i in range(0, n, 5):
            xp, xm = x.copy(), x.copy()
            yp, ym = y.copy(), y.copy()
            if which == 0:
                xp[i] += h
                xm[i] -= h
            else:
                yp[i] += h
                ym[i] -= h
            rp, _ = O.reduce(I.split(xp, L), I.split(yp, L) if b else None, O.F64, op,
                             mode=O.BATCH, alpha=2.5)
            rm, _ = O.reduce(I.split(xm, L), I.split(ym, L) if b else None, O.F64, op,
                             mode=O.BATCH, alpha=2.5)
            fd = float(np.dot(g, (rp - rm) / (2 * h)))
            assert abs(fd - grad[i]) <= 1e-6 * (1 + abs(grad[i]))


def test_constant_derivatives_are_exact_and_match_central_differences():
    """d/dx of the identity view is 1 and d/dx0 of axpy is 1, so their
    gradients are the upstream gradient of the element's range, exactly;
    d/dx1 of axpy is alpha. Central differences of the binary64 reduce
    agree (the maps are linear, so only rounding separates them)."""
    rng = np.random.default_rng(44)
    L = [1, 7, 0, 56]
    n = sum(L)
    x = rng.standard_normal(n)
    y = rng.standard_normal(n)
    g = rng.standard_normal(len(L))
    per_elem = np.repeat(g, L)
    for op, which, b, scale in ((O.IDENTITY, 0, None, 1.0), (O.AXPY, 0, I.split(y, L), 1.0),
                                (O.AXPY, 1, I.split(y, L), 2.5)):
        for mode in (O.BATCH, O.CONCAT):
            gg = g if mode == O.BATCH else g[:1]
            grad = np.concatenate(O.reduce_grad(I.split(x, L), b, O.F64, op, gg, which, mode=mode, alpha=2.5))
            want = (per_elem if mode == O.BATCH else np.full(n, g[0])) * scale
            assert np.array_equal(grad, want), (op, which, mode)
    h = 1e-3
    for op, which in ((O.IDENTITY, 0), (O.AXPY, 0)):
        b = I.split(y, L) if O.ARITY[op] == 2 else None
        grad = np.concatenate(O.reduce_grad(I.split(x, L), b, O.F64, op, g, which, mode=O.BATCH, alpha=2.5))
        for i in range(n):
            xp, xm = x.copy(), x.copy()
            xp[i] += h
            xm[i] -= h
            rp, _ = O.reduce(I.split(xp, L), b, O.F64, op, mode=O.BATCH, alpha=2.5)
            rm, _ = O.reduce(I.split(xm, L), b, O.F64, op, mode=O.BATCH, alpha=2.5)
            fd = float(np.dot(g, (rp - rm) / (2 * h)))
            assert abs(fd - grad[i]) <= 1e-9 * (1 + abs(grad[i]))


def test_reverse_scan_is_the_adjoint_of_the_scan():
    # <gy, scan(x)> == <revscan(gy), x> exactly, per range (BATCH) and across ranges (CONCAT)
    n = 5000
    x = I.ints_0_100(n, 51) - 50
    gy = I.ints_0_100(n, 52) - 50
    L = I.lengths_dirichlet(n, 9, 1.0, 53)
    for mode in (O.CONCAT, O.BATCH):
        s = np.concatenate(O.scan(I.split(x, L), None, O.I32, O.IDENTITY, mode=mode))
        r = np.concatenate(O.scan(I.split(gy, L), None, O.I32, O.IDENTITY, mode=mode,
                                  reverse=True))
        assert int(np.dot(gy.astype(np.int64), s)) == int(np.dot(r, x.astype(np.int64)))


# ---------------------------------------------------------------------------
# Input generator shapes
# ---------------------------------------------------------------------------

def test_segment_length_recipes():
    assert I.lengths_fractions(1 << 20, I.TINY_FRACS) == [419430, 262144, 209715, 157287]
    assert I.lengths_block(10, 4) == [3, 3, 3, 1]
    assert I.lengths_block(8, 3) == [3, 3, 2]
    d = I.lengths_dirichlet(1 << 30, 16, 1.0, I.SEED_SCAN)
    assert sum(d) == 1 << 30 and len(d) == 16 and min(d) >= 0
    b = I.lengths_loguniform(10_000, 1 << 20, 1 << 28, I.SEED_BATCH)
    assert sum(b) == 1 << 28 and len(b) == 10_000 and min(b) >= 1


def test_oracle_rejects_bad_arguments():
    with pytest.raises(ValueError):
        O.reduce([np.ones(3, np.float32)], None, O.F32, O.MUL)   # arity 2 without a second input
    with pytest.raises(TypeError):
        O.scan([np.ones(3, np.float64)], None, O.F32, O.IDENTITY)


# --- generic operators, init and exclusive scans (section 4.3) -------------------

def test_exclusive_sum_scan_of_ones_with_init_is_shifted_iota():
    rng = np.random.default_rng(11)
    for trial in range(20):
        lens = _rand_segmentation(int(rng.integers(0, 60)), rng)
        n = sum(lens)
        ones = I.split(np.ones(n, dtype=np.int32), lens)
        c = int(rng.integers(-1000, 1000))
        ex = np.concatenate(O.scan_ex(ones, None, O.I32, O.IDENTITY, O.SUM, exclusive=True, init=c)) if n else []
        inc = np.concatenate(O.scan_ex(ones, None, O.I32, O.IDENTITY, O.SUM, init=c)) if n else []
        assert list(ex) == [c + i for i in range(n)]
        assert list(inc) == [c + i + 1 for i in range(n)]
        # BATCH: every range restarts from init
        outs = O.scan_ex(ones, None, O.I32, O.IDENTITY, O.SUM, mode=O.BATCH, exclusive=True, init=c)
        for o, L in zip(outs, lens):
            assert list(o) == [c + j for j in range(L)]
        # floating: the same closed form, exactly
        fo = I.split(np.ones(n, dtype=np.float32), lens)
        fex = np.concatenate(O.scan_ex(fo, None, O.F32, O.IDENTITY, O.SUM, exclusive=True, init=c + 0.5)) if n else []
        assert list(fex) == [c + 0.5 + i for i in range(n)]


def test_exclusive_is_inclusive_shifted_for_every_operator_and_direction():
    rng = np.random.default_rng(12)
    for trial in range(30):
        lens = _rand_segmentation(int(rng.integers(1, 50)), rng)
        n = sum(lens)
        k = (rng.integers(-100, 101, size=n)).astype(np.int32)
        segs = I.split(k, lens)
        for comb, mode, rev in itertools.product((O.SUM, O.MAX, O.MIN), (O.CONCAT, O.BATCH), (False, True)):
            init = int(rng.integers(-50, 50)) if trial % 2 else None
            inc = O.scan_ex(segs, None, O.I32, O.IDENTITY, comb, mode=mode, reverse=rev, init=init)
            exc = O.scan_ex(segs, None, O.I32, O.IDENTITY, comb, mode=mode, reverse=rev, exclusive=True, init=init)
            ident = {O.SUM: 0, O.MAX: np.iinfo(np.int64).min, O.MIN: np.iinfo(np.int64).max}[comb]
            start = ident if init is None else init
            # flatten in processing order (reverse: last element first)
            if mode == O.BATCH:
                groups = [(i, e) for i, e in zip(inc, exc)]
            else:
                groups = [(np.concatenate(inc), np.concatenate(exc))]
            for gi, ge in groups:
                if rev:
                    gi, ge = gi[::-1], ge[::-1]
                if len(gi):
                    assert ge[0] == start
                    assert np.array_equal(ge[1:], gi[:-1])


def test_max_min_scans_and_reduces_are_numpy_accumulates():
    """max / min of the values for_each would store: numpy's fmax / fmin
    accumulate over the float32 view values (NaN ignored), in both
    directions, per range in BATCH mode."""
    rng = np.random.default_rng(13)
    for trial in range(25):
        lens = _rand_segmentation(int(rng.integers(1, 80)), rng)
        n = sum(lens)
        x = rng.standard_normal(n).astype(np.float32)
        y = rng.standard_normal(n).astype(np.float32)
        if n > 3 and trial % 3 == 0:
            x[int(rng.integers(0, n))] = np.nan
        for name, op in OPS.items():
            a = np.float32(0.375)
            v = {"identity": x, "square": x * x, "mul": x * y, "axpy": x + a * y}[name].astype(np.float32)
            for comb, acc in ((O.MAX, np.fmax), (O.MIN, np.fmin)):
                got = np.concatenate(O.scan_ex(I.split(x, lens), I.split(y, lens), O.F32, op, comb, alpha=0.375))
                assert np.array_equal(got, acc.accumulate(v.astype(np.float64)), equal_nan=True)
                rgot = np.concatenate(O.scan_ex(I.split(x, lens), I.split(y, lens), O.F32, op, comb, reverse=True,
                                                alpha=0.375))
                assert np.array_equal(rgot, acc.accumulate(v[::-1].astype(np.float64))[::-1], equal_nan=True)
                red = O.reduce_ex(I.split(x, lens), I.split(y, lens), O.F32, op, comb, alpha=0.375)
                assert np.array_equal(red, [acc.reduce(v.astype(np.float64))], equal_nan=True)
                bred = O.reduce_ex(I.split(x, lens), I.split(y, lens), O.F32, op, comb, mode=O.BATCH, alpha=0.375)
                want = [acc.reduce(p.astype(np.float64)) if len(p) else (-np.inf if comb == O.MAX else np.inf)
                        for p in I.split(v, lens)]
                assert np.array_equal(bred, want, equal_nan=True)


def test_max_min_closed_forms_and_init():
    n = 1000
    iota = np.arange(n, dtype=np.int32)
    lens = [100, 0, 400, 500]
    assert list(np.concatenate(O.scan_ex(I.split(iota, lens), None, O.I32, O.IDENTITY, O.MAX))) == list(range(n))
    assert set(np.concatenate(O.scan_ex(I.split(iota[::-1].copy(), lens), None, O.I32, O.IDENTITY, O.MAX))) == {n - 1}
    assert O.reduce_ex(I.split(iota, lens), None, O.I32, O.SQUARE, O.MAX)[0] == (n - 1) ** 2
    assert O.reduce_ex(I.split(iota, lens), None, O.I32, O.IDENTITY, O.MIN, init=-7)[0] == -7
    assert O.reduce_ex(I.split(iota, lens), None, O.I32, O.IDENTITY, O.MAX, init=5000)[0] == 5000
    # empty ranges give init, or the identity without one
    e = [np.zeros(0, dtype=np.float32)]
    assert O.reduce_ex(e, None, O.F32, O.IDENTITY, O.MAX)[0] == -np.inf
    assert O.reduce_ex(e, None, O.F32, O.IDENTITY, O.MIN, init=2.5)[0] == 2.5
    # int32 output of a max scan wraps like the sum scan's
    big = [np.array([5], dtype=np.int32)]
    assert O.scan_ex(big, None, O.I32, O.IDENTITY, O.MAX, init=2 ** 33 + 9, out_dtype=O.I32)[0][0] == 9


def test_sum_with_init_matches_fsum():
    rng = np.random.default_rng(14)
    x = (rng.standard_normal(5000) * np.exp(rng.uniform(-20, 20, 5000))).astype(np.float32)
    lens = [1000, 2500, 1500]
    init = 1.2345e7
    r = O.reduce_ex(I.split(x, lens), None, O.F32, O.IDENTITY, O.SUM, init=init)[0]
    assert r == math.fsum([init] + [float(v) for v in x])
    ex = np.concatenate(O.scan_ex(I.split(x, lens), None, O.F32, O.IDENTITY, O.SUM, exclusive=True, init=init))
    for i in (0, 1, 17, 2499, 4999):
        want = math.fsum([init] + [float(v) for v in x[:i]])
        assert abs(ex[i] - want) <= 2 * U64 * (abs(init) + float(np.abs(x[:i].astype(np.float64)).sum()))


# --- Black-Scholes (section 5, "Black Scholes") -----------------------------------

def _bs(S, K, T, V, r):
    f = lambda a: [np.asarray(a, dtype=np.float32)]
    c, p = O.black_scholes(f(S), f(K), f(T), f(V), r)
    return c[0], p[0]


def test_black_scholes_textbook_example():
    """The standard textbook example (S = 42, K = 40, r = 0.1, sigma = 0.2,
    T = 0.5) prices the call at 4.76 and the put at 0.81."""
    c, p = _bs([42.0], [40.0], [0.5], [0.2], 0.1)
    assert round(float(c[0]), 2) == 4.76 and round(float(p[0]), 2) == 0.81


def test_black_scholes_put_call_parity_and_bounds():
    t = I.options(n=20000, segments=4, seed=7)
    c, p = _bs(t["S"], t["K"], t["T"], t["V"], t["r"])
    S, K, T = (t[n].astype(np.float64) for n in ("S", "K", "T"))
    fwd = S - K * np.exp(-t["r"] * T)
    assert np.all(np.abs((c - p) - fwd) <= 1e-12 * (S + K))
    # no-arbitrage bounds: max(S - K e^{-rT}, 0) <= call <= S; max(-fwd, 0) <= put <= K e^{-rT}
    assert np.all(c >= np.maximum(fwd, 0) - 1e-12 * S) and np.all(c <= S)
    assert np.all(p >= np.maximum(-fwd, 0) - 1e-12 * K) and np.all(p <= K * np.exp(-t["r"] * T) + 1e-12 * K)


def test_black_scholes_at_the_money_closed_form():
    """With r = 0 and S = K the call is S erf(sigma sqrt(T) / (2 sqrt 2))."""
    for S, T, V in ((10.0, 1.0, 0.2), (37.5, 0.25, 0.45), (12.0, 2.0, 0.1)):
        c, p = _bs([S], [S], [T], [V], 0.0)
        want = S * math.erf(float(np.float32(V)) * math.sqrt(float(np.float32(T))) / (2 * math.sqrt(2)))
        assert abs(c[0] - want) <= 1e-13 * S and abs(p[0] - want) <= 1e-13 * S


def test_black_scholes_matches_scipy_normal_cdf():
    from scipy.stats import norm
    t = I.options(n=5000, segments=1, seed=8)
    c, p = _bs(t["S"], t["K"], t["T"], t["V"], t["r"])
    S, K, T, V = (t[n].astype(np.float64) for n in ("S", "K", "T", "V"))
    r = t["r"]
    d1 = (np.log(S / K) + (r + V * V / 2) * T) / (V * np.sqrt(T))
    d2 = d1 - V * np.sqrt(T)
    wc = S * norm.cdf(d1) - K * np.exp(-r * T) * norm.cdf(d2)
    wp = K * np.exp(-r * T) * norm.cdf(-d2) - S * norm.cdf(-d1)
    assert np.all(np.abs(c - wc) <= 1e-12 * (S + K)) and np.all(np.abs(p - wp) <= 1e-12 * (S + K))


def test_black_scholes_deterministic_limit():
    """As sigma sqrt(T) -> 0 the call tends to max(S - K e^{-rT}, 0)."""
    c, p = _bs([50.0, 10.0], [10.0, 50.0], [0.01, 0.01], [0.001, 0.001], 0.05)
    disc = math.exp(-0.05 * float(np.float32(0.01)))      # T as stored (binary32), widened first
    assert abs(c[0] - (50 - 10 * disc)) < 1e-12 and c[1] < 1e-12
    assert p[0] < 1e-12 and abs(p[1] - (50 * disc - 10)) < 1e-12
