"""The chained single pass (DR_TUNE_CHAINED) on one range large enough for
many superblocks of chunks (a chunk is 4 tiles of 4096 elements, a
superblock 128 chunks): binary32 with binary64 and with binary32 carries,
int32 -> int64 and -> int32, forward and reverse, over 16 Dirichlet
segments carved from one buffer at a misaligned offset plus empty
segments; the exclusive form with an initial value; repeatability (the
carries are sums in a fixed shape). Against the oracle: integers exactly,
binary32 within the derived bound."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2406_00158_amd import binding as B
from paper_2406_00158_amd import inputs as I

from gpu_util import announce, carve, dev, empty_like_segments, gather, scan_fp32_bound

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

CHAIN = B.make_tuning(16, B.DR_TUNE_CHAINED)
SIZES = [(1 << 22) + 777, (1 << 25) + 12345]
OR_DT = {B.DR_I32: O.I32, B.DR_F32: O.F32, B.DR_I64: O.I64}


def _lengths(n, seed):
    L = I.lengths_dirichlet(n, 16, 1.0, seed)
    return L[:5] + [0] + L[5:11] + [0, 0] + L[11:]


def _data(in_dt, n, seed):
    if in_dt == B.DR_I32:
        return I.ints_0_100(n, seed) - 50
    return I.normal_f32(n, seed)


def _run(in_dt, out_dt, n, reverse, carry32=False, exclusive_init=None, seed=5):
    L = _lengths(n, seed)
    x = _data(in_dt, n, seed + 1)
    if in_dt == B.DR_I32 and out_dt == B.DR_I32:
        x = x * 10_000_000                                   # the int32 output wraps
    segs, buf = carve(x, L, offset=3)
    outs = empty_like_segments(L, B.TORCH_DTYPE[out_dt], "carved", offset=1)
    tab = B.segments([segs], [outs])
    ws = B.Workspace(dev())
    flags = (B.DR_SCAN_REVERSE if reverse else 0) | (B.DR_SCAN_CARRY_F32 if carry32 else 0)
    if exclusive_init is None:
        B.dr_inclusive_scan(tab, B.make_view("identity", in_dt), out_dt, flags, workspace=ws, tuning=CHAIN)
    else:
        B.dr_scan(tab, B.make_view("identity", in_dt), out_dt, B.DR_COMBINE_SUM, flags | B.DR_SCAN_EXCLUSIVE,
                  exclusive_init, workspace=ws, tuning=CHAIN)
    assert ws.device_status() == 0
    return L, x, gather(outs)


def _check(in_dt, out_dt, L, x, got, reverse, exclusive_init=None):
    kw = dict(reverse=reverse)
    if exclusive_init is not None:
        kw.update(exclusive=True, init=exclusive_init)
    if in_dt == B.DR_I32:
        want = np.concatenate(O.scan_ex(I.split(x, L), None, O.I32, O.IDENTITY, O.SUM,
                                        out_dtype=OR_DT[out_dt], **kw))
        assert np.array_equal(got, want)
        return
    ref, absp = O.scan_ex(I.split(x, L), None, O.F32, O.IDENTITY, O.SUM, want_abs=True, **kw)
    ref, absp = np.concatenate(ref), np.concatenate(absp)
    err = np.abs(got.astype(np.float64) - ref)
    bound = scan_fp32_bound(ref, absp, 16, tiles=sum(L) // 4096 + len(L))
    print(f"max err / A_i {np.max(err / np.maximum(absp, 1e-300)):.3e}")
    assert np.all(err <= bound), (float(err.max()), int(np.argmax(err - bound)))


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("in_dt,out_dt,carry32", [(B.DR_F32, B.DR_F32, False), (B.DR_F32, B.DR_F32, True),
                                                  (B.DR_I32, B.DR_I64, False), (B.DR_I32, B.DR_I32, False)])
def test_chained_forward(n, in_dt, out_dt, carry32):
    announce("chained forward", n, in_dt, out_dt, carry32)
    L, x, got = _run(in_dt, out_dt, n, False, carry32)
    if carry32:
        # binary32 carries: the carry chain rounds in binary32 (bound with u32 per tile)
        ref, absp = O.scan(I.split(x, L), None, O.F32, O.IDENTITY, want_abs=True)
        ref, absp = np.concatenate(ref), np.concatenate(absp)
        tiles = n // 4096 + len(L)
        bound = scan_fp32_bound(ref, absp, 16, tiles=1) + (tiles + 2) * 2.0 ** -24 * absp
        assert np.all(np.abs(got.astype(np.float64) - ref) <= bound)
        return
    _check(in_dt, out_dt, L, x, got, False)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("in_dt,out_dt", [(B.DR_F32, B.DR_F32), (B.DR_I32, B.DR_I64), (B.DR_I32, B.DR_I32)])
def test_chained_reverse(n, in_dt, out_dt):
    announce("chained reverse", n, in_dt, out_dt)
    L, x, got = _run(in_dt, out_dt, n, True)
    _check(in_dt, out_dt, L, x, got, True)


@pytest.mark.parametrize("reverse", [False, True])
@pytest.mark.parametrize("in_dt,out_dt,init", [(B.DR_F32, B.DR_F32, 1.5), (B.DR_I32, B.DR_I64, -987654)])
def test_chained_exclusive_with_init(in_dt, out_dt, init, reverse):
    n = SIZES[0]
    announce("chained exclusive+init", in_dt, out_dt, reverse)
    L, x, got = _run(in_dt, out_dt, n, reverse, exclusive_init=init)
    _check(in_dt, out_dt, L, x, got, reverse, exclusive_init=init)


def test_chained_repeats_bit_for_bit():
    n = SIZES[1]
    announce("chained repeatability", n)
    runs = [_run(B.DR_F32, B.DR_F32, n, False, seed=9)[2] for _ in range(3)]
    assert all(np.array_equal(r.view(np.uint32), runs[0].view(np.uint32)) for r in runs[1:])


def test_chained_is_the_default_for_one_long_range_and_runs_in_place():
    """Without a tuning, a binary32 sum of one range past 2^22 elements runs
    the chained pass (bit-identical to asking for it), also in place."""
    n = SIZES[0]
    announce("chained default, in place", n)
    L = _lengths(n, 13)
    x = _data(B.DR_F32, n, 14)
    segs, buf = carve(x, L, offset=0)
    outs = empty_like_segments(L, torch.float32, "carved")
    view = B.make_view("identity", B.DR_F32)
    B.dr_inclusive_scan(B.segments([segs], [outs]), view, B.DR_F32, tuning=CHAIN)
    asked = gather(outs)
    B.dr_inclusive_scan(B.segments([segs], [segs]), view, B.DR_F32)    # default, in place
    got = gather(segs)
    assert np.array_equal(got.view(np.uint32), asked.view(np.uint32))
    _check(B.DR_F32, B.DR_F32, L, x, got, False)


def test_chained_under_graph_replay():
    """The chained pass captured into a graph (its counters are zeroed by a
    kernel, not a memset node): every replay, with eager work between them,
    equals the eager call bit for bit."""
    n = SIZES[0]
    announce("chained graph replay", n)
    L = _lengths(n, 21)
    x = _data(B.DR_F32, n, 22)
    segs, buf = carve(x, L, offset=1)
    outs = empty_like_segments(L, torch.float32, "carved")
    tab = B.segments([segs], [outs])
    view = B.make_view("identity", B.DR_F32)
    ws = B.Workspace(dev())
    call = lambda: B.dr_inclusive_scan(tab, view, B.DR_F32, workspace=ws, host_check=False, tuning=CHAIN)
    call()
    torch.cuda.synchronize()
    eager = gather(outs)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        call()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    for k in range(3):
        for o in outs:
            o.fill_(float(k))                   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(gather(outs).view(np.uint32), eager.view(np.uint32)), k
    assert ws.device_status() == 0
