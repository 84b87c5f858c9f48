"""Scan parity at 2^25 + a ragged tail, in the default form, with the
reduce-then-scan form named explicitly (its first pass gives every
workgroup a chunk of several tiles, with segment heads inside chunks) and
with the chained single pass (one range only), as at the benchmark's
sizes. Reverse scans (the scan adjoint), exclusive sums with an initial
value and max / min scans, over one distributed range (CONCAT, 16 Dirichlet
segments) and over 300 ragged independent ranges (BATCH, a planned table),
against the oracle: integers and max / min exactly, binary32 sums within
the derived per-element bound."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2406_00158_amd import binding as B
from paper_2406_00158_amd import inputs as I

from gpu_util import announce, dev, dev_to_np, scan_fp32_bound

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

N = (1 << 25) + 12345
OR_DT = {B.DR_I32: O.I32, B.DR_F32: O.F32, B.DR_I64: O.I64}
OR_CMB = {B.DR_COMBINE_SUM: O.SUM, B.DR_COMBINE_MAX: O.MAX, B.DR_COMBINE_MIN: O.MIN}
_CACHE: dict = {}


def _lengths(mode):
    if mode == "concat":
        return I.lengths_dirichlet(N, 16, 1.0, 91)
    return I.lengths_loguniform(300, 1 << 20, N, 92)


def _data(in_dt):
    if in_dt not in _CACHE:
        _CACHE[in_dt] = I.ints_0_100(N, 93) - 50 if in_dt == B.DR_I32 else I.normal_f32(N, 94)
    return _CACHE[in_dt]


def _pieces(t, lengths):
    out, o = [], 0
    for n in lengths:
        out.append(t[o:o + n])
        o += n
    return out


FORMS = {"default": None, "two_pass": B.make_tuning(None, B.DR_TUNE_TWO_PASS),
         "chained": B.make_tuning(16, B.DR_TUNE_CHAINED)}


def _run(in_dt, out_dt, mode, combine, flags, init, form="default"):
    if form == "chained" and mode == "batch":
        pytest.skip("the chained single pass scans one range (CONCAT); batches are refused on the host")
    lengths = _lengths(mode)
    x = _data(in_dt)
    xd = torch.from_numpy(x).to(dev())
    out = torch.empty(N, dtype=B.TORCH_DTYPE[out_dt], device=dev())
    tab = B.segments([_pieces(xd, lengths)], [_pieces(out, lengths)], mode=mode)
    ws = B.Workspace(dev())
    B.dr_scan(tab, B.make_view("identity", in_dt), out_dt, combine, flags, init, workspace=ws, host_check=False,
              tuning=FORMS[form])
    assert ws.device_status() == 0
    return lengths, x, dev_to_np(out)


def _check_sum(in_dt, out_dt, mode, lengths, x, got, reverse, exclusive, init):
    omode = O.BATCH if mode == "batch" else O.CONCAT
    if in_dt == B.DR_I32:
        want = np.concatenate(O.scan_ex(I.split(x, lengths), None, O.I32, O.IDENTITY, O.SUM, mode=omode,
                                        reverse=reverse, exclusive=exclusive, init=init, out_dtype=OR_DT[out_dt]))
        assert np.array_equal(got, want)
        return
    ref, absp = O.scan_ex(I.split(x, lengths), None, O.F32, O.IDENTITY, O.SUM, mode=omode, reverse=reverse,
                          exclusive=exclusive, init=init, want_abs=True)
    ref, absp = np.concatenate(ref), np.concatenate(absp)
    err = np.abs(got.astype(np.float64) - ref)
    bound = scan_fp32_bound(ref, absp, tiles=N // 4096 + len(lengths))
    print(f"max err / A_i {np.max(err / np.maximum(absp, 1e-300)):.3e}")
    assert np.all(err <= bound)


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("mode", ["concat", "batch"])
@pytest.mark.parametrize("in_dt,out_dt", [(B.DR_I32, B.DR_I64), (B.DR_F32, B.DR_F32)])
def test_reverse_scan_2_25(form, mode, in_dt, out_dt):
    announce("reverse scan 2^25", form, mode, in_dt, out_dt)
    lengths, x, got = _run(in_dt, out_dt, mode, B.DR_COMBINE_SUM, B.DR_SCAN_REVERSE, None, form)
    _check_sum(in_dt, out_dt, mode, lengths, x, got, True, False, None)


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("mode", ["concat", "batch"])
@pytest.mark.parametrize("reverse", [False, True])
@pytest.mark.parametrize("in_dt,out_dt", [(B.DR_I32, B.DR_I64), (B.DR_F32, B.DR_F32)])
def test_exclusive_sum_with_init_2_25(form, mode, reverse, in_dt, out_dt):
    announce("exclusive+init scan 2^25", form, mode, reverse, in_dt, out_dt)
    init = -987654 if in_dt == B.DR_I32 else 1.5
    flags = B.DR_SCAN_EXCLUSIVE | (B.DR_SCAN_REVERSE if reverse else 0)
    lengths, x, got = _run(in_dt, out_dt, mode, B.DR_COMBINE_SUM, flags, init, form)
    _check_sum(in_dt, out_dt, mode, lengths, x, got, reverse, True, init)


@pytest.mark.parametrize("combine", [B.DR_COMBINE_MAX, B.DR_COMBINE_MIN])
@pytest.mark.parametrize("mode", ["concat", "batch"])
@pytest.mark.parametrize("reverse", [False, True])
@pytest.mark.parametrize("in_dt,out_dt", [(B.DR_I32, B.DR_I32), (B.DR_F32, B.DR_F32)])
def test_max_min_scan_2_25(combine, mode, reverse, in_dt, out_dt):
    announce("max/min scan 2^25", combine, mode, reverse, in_dt, out_dt)
    omode = O.BATCH if mode == "batch" else O.CONCAT
    for exclusive, init in ((False, None), (True, 7 if in_dt == B.DR_I32 else 0.25)):
        flags = (B.DR_SCAN_EXCLUSIVE if exclusive else 0) | (B.DR_SCAN_REVERSE if reverse else 0)
        lengths, x, got = _run(in_dt, out_dt, mode, combine, flags, init)
        want = np.concatenate(O.scan_ex(I.split(x, lengths), None, OR_DT[in_dt], O.IDENTITY, OR_CMB[combine],
                                        mode=omode, reverse=reverse, exclusive=exclusive, init=init,
                                        out_dtype=OR_DT[out_dt] if in_dt == B.DR_I32 else None))
        if in_dt == B.DR_F32:
            want = want.astype(np.float32)   # the values are binary32 (and so is init)
        assert np.array_equal(got, want), (exclusive, init)
