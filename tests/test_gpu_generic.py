"""GPU parity of the generic algorithms (section 4.3: any commutative
operator, an initial value, exclusive_scan): dr_scan with sum / max / min,
init and the exclusive form, and dr_reduce with max / min, against the
oracle's generic reduce and scan on the same seeded inputs. Max / min
results are exact (they are one of the values, or init), so they are
compared exactly; integer sums bit-exactly; binary32 sums within the derived
bound."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2406_00158_amd import binding as B
from paper_2406_00158_amd import inputs as I

from gpu_util import U64, announce, dev, empty_like_segments, gather, place, scan_fp32_bound

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

OR_DT = {B.DR_I32: O.I32, B.DR_F32: O.F32, B.DR_BF16: O.BF16, B.DR_F64: O.F64, B.DR_I64: O.I64}
OR_OP = {B.DR_OP_IDENTITY: O.IDENTITY, B.DR_OP_SQUARE: O.SQUARE, B.DR_OP_MUL: O.MUL, B.DR_OP_AXPY: O.AXPY}
OR_CMB = {B.DR_COMBINE_SUM: O.SUM, B.DR_COMBINE_MAX: O.MAX, B.DR_COMBINE_MIN: O.MIN}

SEGMENTATIONS = [
    ("tile_edges", [4095, 4096, 4097, 1, 0, 8191]),
    ("with_empties", [0, 3, 0, 0, 20000, 1, 0, 33333, 2]),
    ("many_rows", [(k * 37) % 1500 for k in range(130)]),      # > 64 rows: planned by dr_plan
]
SCAN_PAIRS = [(B.DR_I32, B.DR_I64), (B.DR_I32, B.DR_I32), (B.DR_F32, B.DR_F32), (B.DR_BF16, B.DR_F32),
              (B.DR_F64, B.DR_F64)]


def _values(dtype, n, seed, nan=False):
    if dtype == B.DR_I32:
        return I.ints_0_100(n, seed) - 50
    x = I.normal_f32(n, seed)
    if nan and n > 10:
        x[n // 3] = np.nan
    if dtype == B.DR_BF16:
        return I.bf16_bits(x)
    if dtype == B.DR_F64:
        return x.astype(np.float64) * (1 + 1e-9 * I.uniform_f32(n, seed + 1).astype(np.float64))
    return x


def _init(in_dt, which):
    if which is None:
        return None
    return {B.DR_I32: 1234, B.DR_F32: -0.75, B.DR_BF16: 2.5, B.DR_F64: 0.125}[in_dt] * (1 if which else -1)


@pytest.mark.parametrize("seg_name,lengths", SEGMENTATIONS)
@pytest.mark.parametrize("in_dt,out_dt", SCAN_PAIRS)
@pytest.mark.parametrize("mode", ["concat", "batch"])
@pytest.mark.parametrize("reverse", [False, True])
@pytest.mark.parametrize("form", ["two_pass", "chained", "look_back", "specialized"])
def test_sum_scan_exclusive_with_init(seg_name, lengths, in_dt, out_dt, mode, reverse, form):
    if form == "specialized" and out_dt == B.DR_I64:
        pytest.skip("int32 -> int64 scans keep the two passes")
    announce("sum scan excl+init", seg_name, in_dt, out_dt, mode, reverse, form)
    n = sum(lengths)
    x = _values(in_dt, n, 71)
    init = _init(in_dt, True)
    outs = empty_like_segments(lengths, B.TORCH_DTYPE[out_dt])
    tab = B.segments([place(x, lengths, "separate")], [outs], mode=mode)
    items = B.WS_ITEMS[in_dt] if form == "specialized" else 16
    tu = B.make_tuning(items, {"two_pass": B.DR_TUNE_TWO_PASS, "chained": B.DR_TUNE_CHAINED,
                               "look_back": B.DR_TUNE_TILE_PER_BLOCK, "specialized": B.DR_TUNE_SPECIALIZED}[form])
    flags = B.DR_SCAN_EXCLUSIVE | (B.DR_SCAN_REVERSE if reverse else 0)
    call = lambda: B.dr_scan(tab, B.make_view("identity", in_dt), out_dt, B.DR_COMBINE_SUM, flags, init, tuning=tu)
    if form == "chained" and (mode == "batch" or in_dt not in (B.DR_F32, B.DR_I32)):
        with pytest.raises(B.DrError) as e:   # built for one range of binary32 / int32
            call()
        assert e.value.status == B.DR_ERR_UNSUPPORTED
        return
    call()
    omode = O.BATCH if mode == "batch" else O.CONCAT
    got = gather(outs)
    if in_dt == B.DR_I32:
        want = np.concatenate(O.scan_ex(I.split(x, lengths), None, O.I32, O.IDENTITY, O.SUM, mode=omode,
                                        reverse=reverse, exclusive=True, init=init, out_dtype=OR_DT[out_dt]))
        assert np.array_equal(got, want)
        return
    ref, absp = O.scan_ex(I.split(x, lengths), None, OR_DT[in_dt], O.IDENTITY, O.SUM, mode=omode, reverse=reverse,
                          exclusive=True, init=init, want_abs=True)
    ref, absp = np.concatenate(ref), np.concatenate(absp)
    if in_dt == B.DR_F64:
        bound = 40 * U64 * absp + U64 * np.abs(ref)
    else:
        bound = scan_fp32_bound(ref, absp, items=items, tiles=n // 4096 + len(lengths))
    assert np.all(np.abs(got.astype(np.float64) - ref) <= bound)


@pytest.mark.parametrize("seg_name,lengths", SEGMENTATIONS)
@pytest.mark.parametrize("in_dt,out_dt", SCAN_PAIRS)
@pytest.mark.parametrize("combine", [B.DR_COMBINE_MAX, B.DR_COMBINE_MIN])
@pytest.mark.parametrize("mode", ["concat", "batch"])
@pytest.mark.parametrize("reverse", [False, True])
def test_max_min_scan_exact(seg_name, lengths, in_dt, out_dt, combine, mode, reverse):
    announce("minmax scan", seg_name, in_dt, out_dt, combine, mode, reverse)
    n = sum(lengths)
    x = _values(in_dt, n, 72, nan=(in_dt == B.DR_F32))
    if in_dt == B.DR_I32 and out_dt == B.DR_I32:
        x = x * 10_000_000
    omode = O.BATCH if mode == "batch" else O.CONCAT
    for exclusive, which in ((False, None), (True, None), (False, True), (True, False)):
        init = _init(in_dt, which)
        outs = empty_like_segments(lengths, B.TORCH_DTYPE[out_dt])
        tab = B.segments([place(x, lengths, "carved")], [outs], mode=mode)
        flags = (B.DR_SCAN_EXCLUSIVE if exclusive else 0) | (B.DR_SCAN_REVERSE if reverse else 0)
        B.dr_scan(tab, B.make_view("identity", in_dt), out_dt, combine, flags, init)
        want = np.concatenate(O.scan_ex(I.split(x, lengths), None, OR_DT[in_dt], O.IDENTITY, OR_CMB[combine],
                                        mode=omode, reverse=reverse, exclusive=exclusive, init=init,
                                        out_dtype=OR_DT[out_dt] if in_dt == B.DR_I32 else None))
        got = gather(outs)
        if in_dt in (B.DR_F32, B.DR_BF16):
            want = want.astype(np.float32)     # the values are binary32 (or init, chosen binary32)
        assert np.array_equal(got, want, equal_nan=True), (exclusive, init)


@pytest.mark.parametrize("seg_name,lengths", SEGMENTATIONS)
@pytest.mark.parametrize("in_dt", [B.DR_F32, B.DR_BF16, B.DR_F64, B.DR_I32])
@pytest.mark.parametrize("op", [B.DR_OP_IDENTITY, B.DR_OP_SQUARE, B.DR_OP_MUL, B.DR_OP_AXPY])
@pytest.mark.parametrize("combine", [B.DR_COMBINE_MAX, B.DR_COMBINE_MIN])
@pytest.mark.parametrize("mode", ["concat", "batch"])
def test_max_min_reduce_exact(seg_name, lengths, in_dt, op, combine, mode):
    announce("minmax reduce", seg_name, in_dt, op, combine, mode)
    n = sum(lengths)
    x, y = _values(in_dt, n, 73), _values(in_dt, n, 74)
    arity = B.OP_ARITY[op]
    alpha = 3.0 if in_dt == B.DR_I32 else 0.375
    tab = B.segments([place(a, lengths, "separate") for a in (x, y)[:arity]], mode=mode)
    nres = len(lengths) if mode == "batch" else 1
    omode = O.BATCH if mode == "batch" else O.CONCAT
    rdt = torch.int64 if in_dt == B.DR_I32 else torch.float64
    for which, tuning in ((None, None), (True, None), (False, B.make_tuning(16, B.DR_TUNE_TILE_PER_BLOCK))):
        init = _init(in_dt, which)
        res = torch.zeros(nres, dtype=rdt, device=dev())
        B.dr_reduce(tab, B.make_view(op, in_dt, alpha), combine, 0, init, res, tuning=tuning)
        want = O.reduce_ex(I.split(x, lengths), I.split(y, lengths) if arity == 2 else None, OR_DT[in_dt],
                           OR_OP[op], OR_CMB[combine], mode=omode, init=init, alpha=alpha)
        assert np.array_equal(res.cpu().numpy(), want), (init, tuning)


def test_reduce_sum_without_init_is_transform_reduce():
    announce("dr_reduce sum")
    lengths = [5000, 0, 12345]
    x = _values(B.DR_I32, sum(lengths), 75)
    tab = B.segments([place(x, lengths, "separate")])
    r = torch.zeros(1, dtype=torch.int64, device=dev())
    B.dr_reduce(tab, B.make_view("identity", B.DR_I32), B.DR_COMBINE_SUM, 0, None, r)
    assert r.item() == int(x.astype(np.int64).sum())
    B.dr_reduce(tab, B.make_view("identity", B.DR_I32), B.DR_COMBINE_SUM, 0, -7, r)
    assert r.item() == int(x.astype(np.int64).sum()) - 7


def test_empty_ranges_give_init_or_identity():
    announce("minmax empty")
    e = torch.empty(0, device=dev())
    tab = B.segments([[e, e]], mode="batch")
    r = torch.zeros(2, dtype=torch.float64, device=dev())
    B.dr_reduce(tab, B.make_view("identity", B.DR_F32), B.DR_COMBINE_MAX, 0, None, r)
    assert list(r.cpu().numpy()) == [-np.inf, -np.inf]
    B.dr_reduce(tab, B.make_view("identity", B.DR_F32), B.DR_COMBINE_MIN, 0, 2.5, r)
    assert list(r.cpu().numpy()) == [2.5, 2.5]
