"""Run-to-run reproducibility of the default forms, of the reduce-then-scan
passes named explicitly and of the single pass with specialised waves. The
reduce-then-scan carries are combined in a fixed order (tile records
relative to their chunk, then one fixed-shape scan of the chunk records);
the specialised form's agent scans the published tile totals with a fixed
shape; reductions combine tile partials in member order over a fixed tree. So repeated calls give the same bits for floating-point inputs,
not just results within the error bound. The workspace is shared between the
calls, as a caller's would be."""
import numpy as np
import pytest
import torch

from paper_2406_00158_amd import binding as B
from paper_2406_00158_amd import inputs as I

from gpu_util import announce, dev, empty_like_segments, place

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

LENGTHS = [1 << 22, 12345, 0, 777_777, 1 << 20, 3]
REPEATS = 3


def _bits(segs) -> torch.Tensor:
    flat = torch.cat([s.reshape(-1) for s in segs])
    return flat.view(torch.int64) if flat.dtype == torch.float64 else flat.view(torch.int32)


def _input(in_dt, n, seed):
    x = I.normal_f32(n, seed)
    if in_dt == B.DR_BF16:
        return I.bf16_bits(x)
    if in_dt == B.DR_F64:
        return x.astype(np.float64) * (1 + 1e-9 * I.uniform_f32(n, seed + 1).astype(np.float64))
    return x


@pytest.mark.parametrize("mode", ["concat", "batch"])
@pytest.mark.parametrize("reverse", [False, True])
@pytest.mark.parametrize("in_dt,out_dt,flags", [(B.DR_F32, B.DR_F32, 0), (B.DR_F32, B.DR_F32, B.DR_SCAN_CARRY_F32),
                                                (B.DR_BF16, B.DR_F32, 0), (B.DR_F64, B.DR_F64, 0)])
@pytest.mark.parametrize("form", ["default", "two_pass", "specialized"])
def test_float_scans_repeat_bit_for_bit(mode, reverse, in_dt, out_dt, flags, form):
    if form == "specialized" and flags & B.DR_SCAN_CARRY_F32:
        pytest.skip("the specialised-wave form keeps binary64 carries")
    tuning = {"default": None, "two_pass": B.make_tuning(None, B.DR_TUNE_TWO_PASS),
              "specialized": B.make_tuning(B.WS_ITEMS[in_dt], B.DR_TUNE_SPECIALIZED)}[form]
    announce("scan repeat", mode, reverse, in_dt, flags, form)
    x = _input(in_dt, sum(LENGTHS), 901)
    ins = place(x, LENGTHS, "separate")
    ws = B.Workspace(dev())
    first = None
    for rep in range(REPEATS):
        outs = empty_like_segments(LENGTHS, B.TORCH_DTYPE[out_dt])
        for o in outs:
            o.fill_(float(rep) + 0.5)          # stale contents differ between the calls
        tab = B.segments([ins], [outs], mode=mode)
        B.dr_inclusive_scan(tab, B.make_view("identity", in_dt), out_dt,
                            flags | (B.DR_SCAN_REVERSE if reverse else 0), workspace=ws, tuning=tuning)
        got = _bits(outs)
        if first is None:
            first = got
        else:
            assert torch.equal(got, first), f"call {rep} differs from call 0"
    assert ws.device_status() == 0


@pytest.mark.parametrize("mode", ["concat", "batch"])
@pytest.mark.parametrize("acc", [B.DR_ACC_PLAIN, B.DR_ACC_COMPENSATED])
def test_dot_repeats_bit_for_bit(mode, acc):
    announce("dot repeat", mode, acc)
    n = sum(LENGTHS)
    x, y = I.normal_f32(n, 902), I.normal_f32(n, 903)
    tab = B.segments([place(x, LENGTHS, "separate"), place(y, LENGTHS, "separate")], mode=mode)
    ws = B.Workspace(dev())
    nres = len(LENGTHS) if mode == "batch" else 1
    first = None
    for rep in range(REPEATS):
        res = torch.full((nres,), float(rep), dtype=torch.float64, device=dev())
        B.dr_transform_reduce(tab, B.make_view("mul", B.DR_F32), acc, 0.0, res, workspace=ws)
        got = res.view(torch.int64).clone()
        if first is None:
            first = got
        else:
            assert torch.equal(got, first), f"call {rep} differs from call 0"
    assert ws.device_status() == 0


@pytest.mark.parametrize("form", ["default", "two_pass", "specialized"])
def test_fused_scan_reduce_repeats_bit_for_bit(form):
    announce("fused repeat", form)
    tuning = {"default": None, "two_pass": B.make_tuning(None, B.DR_TUNE_TWO_PASS),
              "specialized": B.make_tuning(B.WS_ITEMS_FUSED, B.DR_TUNE_SPECIALIZED)}[form]
    lengths = I.lengths_loguniform(3000, 1 << 18, 1 << 22, 904)
    n = sum(lengths)
    x, y = I.normal_f32(n, 905), I.normal_f32(n, 906)
    ins = [place(x, lengths, "separate"), place(y, lengths, "separate")]
    ws = B.Workspace(dev())
    first = None
    for rep in range(REPEATS):
        outs = empty_like_segments(lengths, torch.float32)
        res = torch.full((len(lengths),), float(rep), dtype=torch.float64, device=dev())
        tab = B.segments(ins, [outs], mode="batch")
        B.dr_scan_reduce(tab, B.make_view("identity", B.DR_F32), B.make_view("mul", B.DR_F32),
                         B.DR_ACC_COMPENSATED, 0.0, res, workspace=ws, tuning=tuning)
        got = (_bits(outs), res.view(torch.int64).clone())
        if first is None:
            first = got
        else:
            assert torch.equal(got[0], first[0]) and torch.equal(got[1], first[1]), f"call {rep} differs"
    assert ws.device_status() == 0
