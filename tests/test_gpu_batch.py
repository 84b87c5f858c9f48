"""Batched ragged ranges: the fused scan + dot launch over thousands of
ranges against the oracle, its capture into a hipGraph (every replay checked
against the eager result, with eager work between replays), and the tile
autotuner."""
import os

import numpy as np
import pytest
import torch

import oracle as O
from paper_2406_00158_amd import autotune as AT
from paper_2406_00158_amd import binding as B
from paper_2406_00158_amd import inputs as I

from gpu_util import announce, dev, dev_to_np, reduce_bound, scan_fp32_bound

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _carve(t, lengths):
    out, o = [], 0
    for n in lengths:
        out.append(t[o:o + n])
        o += n
    return out


def _batch_case(count, total, seed):
    lengths = I.lengths_loguniform(count, 1 << 20, total, seed)
    n = sum(lengths)
    xs, ys = I.normal_f32(n, seed + 1), I.normal_f32(n, seed + 2)
    x, y = torch.from_numpy(xs).to(dev()), torch.from_numpy(ys).to(dev())
    s = torch.empty_like(x)
    res = torch.zeros(len(lengths), dtype=torch.float64, device=dev())
    tab = B.segments([_carve(x, lengths), _carve(y, lengths)], [_carve(s, lengths)], mode="batch")
    return lengths, xs, ys, x, y, s, res, tab


def _run(tab, res, ws, tuning=None):
    B.dr_scan_reduce(tab, B.make_view("identity", B.DR_F32), B.make_view("mul", B.DR_F32), B.DR_ACC_COMPENSATED,
                     0.0, res, workspace=ws, tuning=tuning, host_check=False)


@pytest.mark.parametrize("items", [16, 32, 64])
def test_batched_scan_dot_10000_ranges(items):
    announce("batched 10000", items)
    lengths, xs, ys, x, y, s, res, tab = _batch_case(10_000, 1 << 24, 5)
    ws = B.Workspace(dev())
    _run(tab, res, ws, B.make_tuning(items))
    assert ws.device_status() == 0
    ref, absp = O.scan(I.split(xs, lengths), None, O.F32, O.IDENTITY, mode=O.BATCH, want_abs=True)
    ref, absp = np.concatenate(ref), np.concatenate(absp)
    err = np.abs(dev_to_np(s).astype(np.float64) - ref)
    assert np.all(err <= scan_fp32_bound(ref, absp, items=items, tiles=(1 << 24) // 1024 + 10_000))
    want, mag = O.reduce(I.split(xs, lengths), I.split(ys, lengths), O.F32, O.MUL, mode=O.BATCH)
    got = dev_to_np(res)
    assert np.all(np.abs(got - want) <= reduce_bound(mag, "compensated", items=items, tiles=64) + 0)


def test_graph_capture_and_replay():
    announce("graph capture")
    lengths, xs, ys, x, y, s, res, tab = _batch_case(2000, 1 << 22, 9)
    ws = B.Workspace(dev())
    _run(tab, res, ws)                       # eager: plans and sizes the workspace
    torch.cuda.synchronize()
    ref_s, ref_r = s.clone(), res.clone()
    # the eager result (and with it every replay, compared bit for bit below)
    # against the oracle
    want_s, absp = O.scan(I.split(xs, lengths), None, O.F32, O.IDENTITY, mode=O.BATCH, want_abs=True)
    want_s, absp = np.concatenate(want_s), np.concatenate(absp)
    assert np.all(np.abs(dev_to_np(ref_s).astype(np.float64) - want_s) <=
                  scan_fp32_bound(want_s, absp, tiles=(1 << 22) // 4096 + 2000))
    want_r, mag = O.reduce(I.split(xs, lengths), I.split(ys, lengths), O.F32, O.MUL, mode=O.BATCH)
    assert np.all(np.abs(dev_to_np(ref_r) - want_r) <= reduce_bound(mag, "compensated", tiles=64))
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        _run(tab, res, ws)
    torch.cuda.current_stream().wait_stream(side)
    with torch.cuda.graph(g):
        _run(tab, res, ws)
    for rep in range(5):
        s.zero_()
        res.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(res, ref_r), f"replay {rep}: dot differs from eager"
        # the carries are sums in a fixed order: the replay repeats the eager bits
        assert torch.equal(s, ref_s), f"replay {rep}: scan differs from eager"
        # eager work between replays, through the same workspace
        _run(tab, res, ws)
        torch.cuda.synchronize()
        assert torch.equal(res, ref_r)
    # the graph reads the current inputs: doubling x doubles every result exactly
    x.mul_(2.0)
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(res, 2 * ref_r)
    x.mul_(0.5)
    assert ws.device_status() == 0


def test_autotuner_picks_and_caches(tmp_path, monkeypatch):
    monkeypatch.setenv("DR_TUNE_CACHE", str(tmp_path / "tune.json"))
    AT._cache = None
    announce("autotune")
    lengths, xs, ys, x, y, s, res, tab = _batch_case(500, 1 << 21, 13)
    ws = B.Workspace(dev())
    view = B.make_view("identity", B.DR_F32)
    tu = AT.tune(B.DR_ALGO_SCAN_REDUCE, view, B.DR_F32, tab, lambda t: _run(tab, res, ws, t))
    assert tu is not None and tu.items_per_thread in AT.ITEMS and tu.block_threads in AT.BLOCKS
    assert tu.flags in [f for _, f in AT.SCAN_FORMS]
    e = AT.entry(B.DR_ALGO_SCAN_REDUCE, view, B.DR_F32, tab)
    assert e["label"] == AT.label(tu) and len(e["all"]) == len(AT.candidates(B.DR_ALGO_SCAN_REDUCE, view, B.DR_F32))
    assert {AT.form_name(f) for _, f in AT.SCAN_FORMS} <= {k.split("/")[1] for k in e["all"]}
    assert os.path.exists(tmp_path / "tune.json")
    AT._cache = None
    tu2 = AT.tune(B.DR_ALGO_SCAN_REDUCE, view, B.DR_F32, tab, lambda t: pytest.fail("re-timed a cached shape"))
    assert (tu2.block_threads, tu2.items_per_thread, tu2.flags) == (tu.block_threads, tu.items_per_thread, tu.flags)
    _run(tab, res, ws, tu)
    want, mag = O.reduce(I.split(xs, lengths), I.split(ys, lengths), O.F32, O.MUL, mode=O.BATCH)
    assert np.all(np.abs(dev_to_np(res) - want) <= reduce_bound(mag, "compensated", items=64, tiles=64))


def test_specialized_scan_under_graph_capture_runs_two_passes():
    """A cooperative launch cannot be captured: a scan asking for the
    specialised-wave form inside a capture runs the two passes instead. Every
    replay is checked against the oracle, with eager work between replays,
    and the replays repeat each other bit for bit."""
    announce("specialised form under capture")
    lengths = [200_000, 0, 123_457, 77]
    n = sum(lengths)
    xs = I.normal_f32(n, 31)
    x = torch.from_numpy(xs).to(dev())
    s = torch.empty_like(x)
    tab = B.segments([_carve(x, lengths)], [_carve(s, lengths)])
    view = B.make_view("identity", B.DR_F32)
    tu = B.make_tuning(B.WS_ITEMS[B.DR_F32], B.DR_TUNE_SPECIALIZED)
    ws = B.Workspace(dev())
    ref, absp = O.scan(I.split(xs, lengths), None, O.F32, O.IDENTITY, want_abs=True)
    ref, absp = np.concatenate(ref), np.concatenate(absp)
    bound = scan_fp32_bound(ref, absp, items=B.WS_ITEMS[B.DR_F32], tiles=n // 8192 + len(lengths))
    B.dr_inclusive_scan(tab, view, B.DR_F32, workspace=ws, tuning=tu)      # eager: the specialised form
    torch.cuda.synchronize()
    assert np.all(np.abs(dev_to_np(s).astype(np.float64) - ref) <= bound)
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        B.dr_inclusive_scan(tab, view, B.DR_F32, workspace=ws, tuning=tu)
    torch.cuda.current_stream().wait_stream(side)
    with torch.cuda.graph(g):
        B.dr_inclusive_scan(tab, view, B.DR_F32, workspace=ws, tuning=tu)
    first = None
    for rep in range(3):
        s.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = dev_to_np(s)
        assert np.all(np.abs(got.astype(np.float64) - ref) <= bound), f"replay {rep}"
        if first is None:
            first = got.copy()
        else:
            assert np.array_equal(got.view(np.uint32), first.view(np.uint32)), f"replay {rep} differs"
        B.dr_inclusive_scan(tab, view, B.DR_F32, workspace=ws, tuning=tu)   # eager work between replays
        torch.cuda.synchronize()
    assert ws.device_status() == 0
