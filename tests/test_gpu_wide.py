"""Parity of the look-back scan at every launch shape built beside the
256 x {16, 32, 64} tiles: 512- and 1024-thread workgroups, and 4 / 8 items
at 256 threads (the shapes the autotuner adds for the batched scans).
Ragged ranges include empty ones, one element, exactly one tile and one
tile plus one, starts at every 16-byte alignment, and ranges several tiles
long (their look-backs chain tiles of one range and stop at its first).
Checked against the oracle: the fused scan + compensated dot per range
(BATCH), the reverse scan per range (BATCH), and forward / reverse scans of
one distributed range (CONCAT), binary32 within the derived bounds."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2406_00158_amd import binding as B
from paper_2406_00158_amd import inputs as I

from gpu_util import announce, carve, dev, dev_to_np, empty_like_segments, gather, reduce_bound, scan_fp32_bound

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

SHAPES = [(256, 4), (256, 8), (512, 8), (512, 16), (512, 32), (1024, 4), (1024, 8), (1024, 16)]


def _lengths(block, items, seed):
    tile = block * items
    special = [0, 1, tile, tile + 1, 3 * tile - 5, 5 * tile + 7, 2, 0]
    rest = I.lengths_loguniform(240, 4 * tile, (1 << 21) - sum(special), seed)
    out = special + rest
    return [out[i] for i in np.random.default_rng(seed).permutation(len(out))]


def _tuning(block, items):
    return B.make_tuning(items, B.DR_TUNE_TILE_PER_BLOCK, block)


@pytest.mark.parametrize("block,items", SHAPES)
def test_fused_scan_dot_batch(block, items):
    announce("wide look-back fused scan + dot, batch", block, items)
    L = _lengths(block, items, 700 + block + items)
    n = sum(L)
    xs, ys = I.normal_f32(n, 31), I.normal_f32(n, 32)
    x, bx = carve(xs, L, offset=1)
    y, by = carve(ys, L, offset=1)
    s = empty_like_segments(L, torch.float32, "carved", offset=1)
    r = torch.zeros(len(L), dtype=torch.float64, device=dev())
    tab = B.segments([x, y], [s], mode="batch")
    ws = B.Workspace(dev())
    B.dr_scan_reduce(tab, B.make_view("identity", B.DR_F32), B.make_view("mul", B.DR_F32), B.DR_ACC_COMPENSATED,
                     0.0, r, workspace=ws, tuning=_tuning(block, items))
    assert ws.device_status() == 0
    xl, yl = I.split(xs, L), I.split(ys, L)
    ref, absp = O.scan(xl, None, O.F32, O.IDENTITY, mode=O.BATCH, want_abs=True)
    ref, absp = np.concatenate(ref), np.concatenate(absp)
    got = gather(s)
    tiles = max(-(-k // (block * items)) for k in L)
    assert np.all(np.abs(got.astype(np.float64) - ref) <= scan_fp32_bound(ref, absp, items, tiles=tiles,
                                                                          block=block))
    want, mag = O.reduce(xl, yl, O.F32, O.MUL, mode=O.BATCH)
    rg = dev_to_np(r)
    for k, nk in enumerate(L):
        t_k = max(1, -(-nk // (block * items)))
        assert abs(rg[k] - want[k]) <= reduce_bound(mag[k], "compensated", items, tiles=t_k, block=block), k
    assert np.all(rg[np.asarray(L) == 0] == 0.0)


@pytest.mark.parametrize("block,items", SHAPES)
def test_reverse_scan_batch(block, items):
    announce("wide look-back reverse scan, batch", block, items)
    L = _lengths(block, items, 800 + block + items)
    n = sum(L)
    xs = I.normal_f32(n, 33)
    x, bx = carve(xs, L, offset=3)
    s = empty_like_segments(L, torch.float32, "carved", offset=3)
    tab = B.segments([x], [s], mode="batch")
    ws = B.Workspace(dev())
    B.dr_inclusive_scan(tab, B.make_view("identity", B.DR_F32), B.DR_F32, B.DR_SCAN_REVERSE, workspace=ws,
                        tuning=_tuning(block, items))
    assert ws.device_status() == 0
    ref, absp = O.scan(I.split(xs, L), None, O.F32, O.IDENTITY, mode=O.BATCH, reverse=True, want_abs=True)
    ref, absp = np.concatenate(ref), np.concatenate(absp)
    tiles = max(-(-k // (block * items)) for k in L)
    got = gather(s)
    assert np.all(np.abs(got.astype(np.float64) - ref) <= scan_fp32_bound(ref, absp, items, tiles=tiles,
                                                                          block=block))


@pytest.mark.parametrize("reverse", [False, True])
@pytest.mark.parametrize("block,items", SHAPES)
def test_scan_concat(block, items, reverse):
    announce("wide look-back scan, concat", block, items, reverse)
    L = [(1 << 19) + 3, 0, 77, 5 * block * items + 1, (1 << 18) - 9]
    n = sum(L)
    xs = I.normal_f32(n, 34)
    x, bx = carve(xs, L, offset=2)
    s = empty_like_segments(L, torch.float32, "carved", offset=2)
    tab = B.segments([x], [s])
    ws = B.Workspace(dev())
    B.dr_inclusive_scan(tab, B.make_view("identity", B.DR_F32), B.DR_F32, B.DR_SCAN_REVERSE if reverse else 0,
                        workspace=ws, tuning=_tuning(block, items))
    assert ws.device_status() == 0
    ref, absp = O.scan(I.split(xs, L), None, O.F32, O.IDENTITY, reverse=reverse, want_abs=True)
    ref, absp = np.concatenate(ref), np.concatenate(absp)
    tiles = sum(-(-k // (block * items)) + 1 for k in L)
    got = gather(s)
    assert np.all(np.abs(got.astype(np.float64) - ref) <= scan_fp32_bound(ref, absp, items, tiles=tiles,
                                                                          block=block))
