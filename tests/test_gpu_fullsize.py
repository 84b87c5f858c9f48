"""Parity at the full sizes of the five workloads, in the default launch
configuration (the one bench.py times), compared in full against the CPU
oracle: bit-exact for integers and for_each, within 2e-6 relative of binary64
for compensated binary32 reductions, within the derived per-element bound for
binary32 scans. Each test prints its error figures."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2406_00158_amd import binding as B
from paper_2406_00158_amd import inputs as I

from gpu_util import U32, announce, dev, dev_to_np, reduce_bound, scan_fp32_bound

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

REL_COMPENSATED = 2e-6
_INPUTS: dict = {}


def _workload(name):
    """Generate each workload once per test session (the large ones take tens
    of seconds)."""
    if name not in _INPUTS:
        _INPUTS.clear()
        _INPUTS[name] = getattr(I, name)()
    return _INPUTS[name]


def _pieces(t, lengths):
    out, o = [], 0
    for n in lengths:
        out.append(t[o:o + n])
        o += n
    return out


def _to_dev(a):
    if a.dtype == np.uint16:
        return torch.from_numpy(a.view(np.int16)).to(dev()).view(torch.bfloat16)
    return torch.from_numpy(a).to(dev())


def _rel(got, want):
    return abs(got - want) / abs(want) if want != 0 else abs(got)


@pytest.mark.parametrize("layout", ["separate", "carved"])
def test_tiny_dot_scan_sum(layout):
    t = _workload("tiny")
    L = t["lengths"]
    announce("tiny", layout)
    if layout == "separate":
        x = [_to_dev(p.copy()) for p in I.split(t["x"], L)]
        y = [_to_dev(p.copy()) for p in I.split(t["y"], L)]
        k = [_to_dev(p.copy()) for p in I.split(t["k"], L)]
    else:   # one buffer: segment starts at byte offsets 0, 8, 8, 4 (mod 16)
        x, y, k = (_pieces(_to_dev(t[n]), L) for n in ("x", "y", "k"))
    res = torch.zeros(1, dtype=torch.float64, device=dev())
    B.dr_transform_reduce(B.segments([x, y]), B.make_view("mul", B.DR_F32), B.DR_ACC_COMPENSATED, 0.0, res)
    want, mag = O.reduce(I.split(t["x"], L), I.split(t["y"], L), O.F32, O.MUL)
    rel = _rel(res.item(), want[0])
    print(f"tiny dot rel err {rel:.3e} cond {mag[0] / abs(want[0]):.3e}")
    assert rel <= REL_COMPENSATED
    out = [torch.empty(p.numel(), dtype=torch.int32, device=dev()) for p in k]
    B.dr_inclusive_scan(B.segments([k], [out]), B.make_view("identity", B.DR_I32), B.DR_I32)
    want_s = np.concatenate(O.scan(I.split(t["k"], L), None, O.I32, O.IDENTITY, out_dtype=O.I32))
    assert np.array_equal(np.concatenate([dev_to_np(p) for p in out]), want_s)
    ri = torch.zeros(1, dtype=torch.int64, device=dev())
    B.dr_transform_reduce(B.segments([k]), B.make_view("identity", B.DR_I32), 0, 0, ri)
    assert ri.item() == int(O.reduce(I.split(t["k"], L), None, O.I32, O.IDENTITY)[0][0])


def test_triad_and_dot_2_28():
    t = _workload("triad")
    L = t["lengths"]
    announce("triad 2^28")
    b, c = _to_dev(t["b"]), _to_dev(t["c"])
    a = torch.empty_like(b)
    B.dr_for_each(B.segments([_pieces(b, L), _pieces(c, L)], [_pieces(a, L)]),
                  B.make_view("axpy", B.DR_F32, t["s"]), B.DR_F32)
    want = np.concatenate(O.for_each(I.split(t["b"], L), I.split(t["c"], L), O.F32, O.AXPY, O.F32, alpha=t["s"]))
    assert np.array_equal(dev_to_np(a).view(np.uint32), want.view(np.uint32))
    del a, want
    res = torch.zeros(1, dtype=torch.float64, device=dev())
    B.dr_transform_reduce(B.segments([_pieces(b, L), _pieces(c, L)]), B.make_view("mul", B.DR_F32),
                          B.DR_ACC_COMPENSATED, 0.0, res)
    w, mag = O.reduce(I.split(t["b"], L), I.split(t["c"], L), O.F32, O.MUL)
    rel = _rel(res.item(), w[0])
    print(f"triad dot rel err {rel:.3e} cond {mag[0] / abs(w[0]):.3e}")
    assert rel <= REL_COMPENSATED


@pytest.mark.parametrize("form", ["default", "chained"])
@pytest.mark.parametrize("out_dt", [B.DR_I64, B.DR_I32])
def test_int_scan_2_30(out_dt, form):
    t = _workload("scan_int")
    L = t["lengths"]
    announce("int scan 2^30", out_dt, form)
    k = _to_dev(t["k"])
    out = torch.empty(k.numel(), dtype=B.TORCH_DTYPE[out_dt], device=dev())
    B.dr_inclusive_scan(B.segments([_pieces(k, L)], [_pieces(out, L)]), B.make_view("identity", B.DR_I32), out_dt,
                        tuning=B.make_tuning(16, B.DR_TUNE_CHAINED) if form == "chained" else None)
    del k
    got = dev_to_np(out)
    del out
    want = np.concatenate(O.scan(I.split(t["k"], L), None, O.I32, O.IDENTITY,
                                 out_dtype=O.I64 if out_dt == B.DR_I64 else O.I32))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("form", ["default", "two_pass", "chained", "specialized"])
def test_fp32_scan_2_28_f64_carry(form):
    t = _workload("scan_fp")
    L = t["lengths"]
    announce("fp scan 2^28", form)
    x = _to_dev(t["x"])
    out = torch.empty_like(x)
    tuning = {"default": None, "two_pass": B.make_tuning(None, B.DR_TUNE_TWO_PASS),
              "chained": B.make_tuning(16, B.DR_TUNE_CHAINED),
              "specialized": B.make_tuning(B.WS_ITEMS[B.DR_F32], B.DR_TUNE_SPECIALIZED)}[form]
    B.dr_inclusive_scan(B.segments([_pieces(x, L)], [_pieces(out, L)]), B.make_view("identity", B.DR_F32),
                        B.DR_F32, tuning=tuning)
    got = dev_to_np(out).astype(np.float64)
    ref, absp = O.scan(I.split(t["x"], L), None, O.F32, O.IDENTITY, want_abs=True)
    ref, absp = np.concatenate(ref), np.concatenate(absp)
    err = np.abs(got - ref)
    scaled = err / absp
    exact = np.mean(got.astype(np.float32) == ref.astype(np.float32))
    print(f"fp scan: max abs err {err.max():.3e}, max err/A_i {scaled.max():.3e} (u32 = {U32:.3e}), "
          f"fraction equal to fl32(ref) {exact:.6f}")
    items = B.WS_ITEMS[B.DR_F32] if form == "specialized" else 16
    assert np.all(err <= scan_fp32_bound(ref, absp, items=items, tiles=(1 << 28) // 4096 + 16))


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_precision_2_29(dtype):
    t = _workload("precision")
    L = t["lengths"]
    announce("precision 2^29", dtype)
    xs = t["x"] if dtype == "f32" else t["x_bf16"]
    ys = t["y"] if dtype == "f32" else t["y_bf16"]
    odt = O.F32 if dtype == "f32" else O.BF16
    bdt = B.DR_F32 if dtype == "f32" else B.DR_BF16
    x, y = _to_dev(xs), _to_dev(ys)
    tab1 = B.segments([_pieces(x, L)])
    tab2 = B.segments([_pieces(x, L), _pieces(y, L)])
    w_sq, m_sq = O.reduce(I.split(xs, L), None, odt, O.SQUARE)
    w_dot, m_dot = O.reduce(I.split(xs, L), I.split(ys, L), odt, O.MUL)
    for acc in ("compensated", "plain"):
        r = torch.zeros(1, dtype=torch.float64, device=dev())
        B.dr_transform_reduce(tab1, B.make_view("square", bdt), B.ACCS[acc], 0.0, r)
        rel_sq = _rel(r.item(), w_sq[0])
        B.dr_transform_reduce(tab2, B.make_view("mul", bdt), B.ACCS[acc], 0.0, r)
        rel_dot = _rel(r.item(), w_dot[0])
        print(f"{dtype} {acc}: sumsq rel err {rel_sq:.3e}; dot rel err {rel_dot:.3e} "
              f"(cond {m_dot[0] / abs(w_dot[0]):.3e})")
        if acc == "compensated":
            assert rel_sq <= REL_COMPENSATED and rel_dot <= REL_COMPENSATED
        else:
            items = 16 if dtype == "f32" else 32     # the default tile of the call
            assert abs(rel_sq * w_sq[0]) <= reduce_bound(m_sq[0], "plain", items=items, tiles=1 << 17)
            assert abs(rel_dot * w_dot[0]) <= reduce_bound(m_dot[0], "plain", items=items, tiles=1 << 17)


def test_batch_10000_ranges_forward_backward():
    t = _workload("batch")
    L = t["lengths"]
    announce("batch 10000 x 2^28")
    x, y = _to_dev(t["x"]), _to_dev(t["y"])
    s = torch.empty_like(x)
    res = torch.zeros(len(L), dtype=torch.float64, device=dev())
    tab = B.segments([_pieces(x, L), _pieces(y, L)], [_pieces(s, L)], mode="batch")
    B.dr_scan_reduce(tab, B.make_view("identity", B.DR_F32), B.make_view("mul", B.DR_F32), B.DR_ACC_COMPENSATED,
                     0.0, res)
    got_s = dev_to_np(s).astype(np.float64)
    ref, absp = O.scan(I.split(t["x"], L), None, O.F32, O.IDENTITY, mode=O.BATCH, want_abs=True)
    ref, absp = np.concatenate(ref), np.concatenate(absp)
    assert np.all(np.abs(got_s - ref) <= scan_fp32_bound(ref, absp, tiles=(1 << 28) // 4096 + len(L)))
    del got_s, ref, absp
    want, mag = O.reduce(I.split(t["x"], L), I.split(t["y"], L), O.F32, O.MUL, mode=O.BATCH)
    got = dev_to_np(res)
    rel = np.abs(got - want) / np.maximum(np.abs(want), 1e-300)
    print(f"batched dot: max rel err {rel.max():.3e}, median {np.median(rel):.3e}; "
          f"lengths min/median/max {min(L)}/{int(np.median(L))}/{max(L)}")
    assert np.all(np.abs(got - want) <= reduce_bound(mag, "compensated", tiles=128))
    # backward at full size: gx = g_d * y, gy = g_d * x against the binary64 oracle
    g = torch.from_numpy(I.normal_f32(len(L), 77).astype(np.float64)).to(dev())
    gx, gy = torch.empty_like(x), torch.empty_like(y)
    B.dr_broadcast_mul(B.segments([_pieces(x, L), _pieces(y, L)], [_pieces(gx, L), _pieces(gy, L)],
                                  mode="batch"), B.make_view("mul", B.DR_F32), g, 2)
    wx = np.concatenate(O.reduce_grad(I.split(t["x"], L), I.split(t["y"], L), O.F32, O.MUL, dev_to_np(g), 0,
                                      mode=O.BATCH))
    assert np.array_equal(dev_to_np(gx), wx.astype(np.float32))
    del wx
    wy = np.concatenate(O.reduce_grad(I.split(t["x"], L), I.split(t["y"], L), O.F32, O.MUL, dev_to_np(g), 1,
                                      mode=O.BATCH))
    assert np.array_equal(dev_to_np(gy), wy.astype(np.float32))
    del wy, gy
    # the scan's adjoint at full size: a reverse (suffix) scan of an upstream
    # gradient per range, against the binary64 oracle
    up_np = I.normal_f32(sum(L), 78)
    up = torch.from_numpy(up_np).to(dev())
    B.dr_inclusive_scan(B.segments([_pieces(up, L)], [_pieces(gx, L)], mode="batch"),
                        B.make_view("identity", B.DR_F32), B.DR_F32, B.DR_SCAN_REVERSE)
    ref, absp = O.scan(I.split(up_np, L), None, O.F32, O.IDENTITY, mode=O.BATCH, reverse=True, want_abs=True)
    ref, absp = np.concatenate(ref), np.concatenate(absp)
    err = np.abs(dev_to_np(gx).astype(np.float64) - ref)
    print(f"batched reverse scan: max err / A_i {np.max(err / np.maximum(absp, 1e-300)):.3e}")
    assert np.all(err <= scan_fp32_bound(ref, absp, tiles=(1 << 28) // 4096 + len(L)))


def test_black_scholes_2_28_options_sampled():
    """All 2^28 options priced in the default launch; a seeded sample of one
    million is checked against the oracle (elementwise, so sampled
    options are checked exactly as the whole would be)."""
    t = I.options()
    L = t["lengths"]
    announce("black-scholes 2^28")
    ins = [_to_dev(t[n]) for n in ("S", "K", "T", "V")]
    call, put = torch.empty_like(ins[0]), torch.empty_like(ins[0])
    B.dr_for_each(B.segments([_pieces(a, L) for a in ins], [_pieces(call, L), _pieces(put, L)]),
                  B.make_view("black_scholes", B.DR_F32, t["r"]), B.DR_F32)
    idx = np.sort(np.random.default_rng(5).choice(sum(L), size=1 << 20, replace=False))
    wc, wp = O.black_scholes(*([t[n][idx]] for n in ("S", "K", "T", "V")), t["r"])
    gc, gp = dev_to_np(call)[idx].astype(np.float64), dev_to_np(put)[idx].astype(np.float64)
    scale = t["S"][idx].astype(np.float64) + t["K"][idx].astype(np.float64)
    ec, ep = np.abs(gc - wc[0]) / scale, np.abs(gp - wp[0]) / scale
    print(f"black-scholes 2^28: max |err| / (S + K) call {ec.max() / U32:.2f} u32, put {ep.max() / U32:.2f} u32")
    assert np.all(ec <= 32 * U32) and np.all(ep <= 32 * U32)
    assert np.all(np.isfinite(dev_to_np(call))) and np.all(np.isfinite(dev_to_np(put)))
