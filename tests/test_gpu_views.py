"""The kernels over segment tables built by the segment algebra of section
4.4: zips of ranges whose segments are not aligned (refined by
dr_zip_segments), and take / drop / trim (dr_trim_segments), against the
oracle on the flat (concatenated) arrays. Bit-exact for integers and the
triad; the derived bounds for binary32 sums."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2406_00158_amd import binding as B
from paper_2406_00158_amd import inputs as I

from gpu_util import announce, dev, dev_to_np, reduce_bound

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _segments(flat: np.ndarray, lengths, pad: int = 0):
    """Separate device allocations holding consecutive pieces of `flat`
    (each allocation `pad` elements longer, so pieces are not contiguous
    with each other)."""
    out, o = [], 0
    for n in lengths:
        t = torch.from_numpy(np.ascontiguousarray(flat[o:o + n])).to(dev())
        if pad:
            buf = torch.empty(n + pad, dtype=t.dtype, device=dev())
            buf[pad:] = t
            t = buf[pad:]
        out.append(t)
        o += n
    return out


def _empty_segments(lengths, dtype):
    return [torch.empty(n, dtype=dtype, device=dev()) for n in lengths]


def _flat(segs) -> np.ndarray:
    return np.concatenate([dev_to_np(t) for t in segs]) if segs else np.zeros(0)


N = 40_000
X_SPLIT = [5000, 0, 13000, 1, 21999]
Y_SPLIT = [9000, 9000, 0, 22000]
OUT_SPLIT = [12345, 7, 27648]


def test_zip_non_aligned_dot_and_int_sum():
    announce("zip dot")
    x, y = I.normal_f32(N, 601), I.normal_f32(N, 602)
    tab = B.zip_segments([_segments(x, X_SPLIT, pad=1), _segments(y, Y_SPLIT, pad=3)])
    cuts = (set(np.cumsum(X_SPLIT)) | set(np.cumsum(Y_SPLIT))) - {0}
    assert tab.total_length == N and tab.n_segments == len(cuts)   # one row per piece between cuts
    res = torch.zeros(1, dtype=torch.float64, device=dev())
    B.dr_transform_reduce(tab, B.make_view("mul", B.DR_F32), B.DR_ACC_COMPENSATED, 0.0, res)
    want, mag = O.reduce([x], [y], O.F32, O.MUL)
    assert abs(res.item() - want[0]) <= reduce_bound(mag[0], "compensated", tiles=16)
    k1, k2 = I.ints_0_100(N, 603), I.ints_0_100(N, 604)
    tk = B.zip_segments([_segments(k1, X_SPLIT), _segments(k2, Y_SPLIT)])
    ri = torch.zeros(1, dtype=torch.int64, device=dev())
    B.dr_transform_reduce(tk, B.make_view("mul", B.DR_I32), 0, 0, ri)
    assert ri.item() == int(np.dot(k1.astype(np.int64), k2.astype(np.int64)))


def test_zip_non_aligned_triad_into_third_segmentation():
    announce("zip triad")
    b, c = I.uniform_f32(N, 611), I.uniform_f32(N, 612)
    out = _empty_segments(OUT_SPLIT, torch.float32)
    tab = B.zip_segments([_segments(b, X_SPLIT), _segments(c, Y_SPLIT)], [out])
    B.dr_for_each(tab, B.make_view("axpy", B.DR_F32, 3.0), B.DR_F32)
    want = O.for_each([b], [c], O.F32, O.AXPY, O.F32, alpha=3.0)[0]
    assert np.array_equal(_flat(out).view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("mode", ["concat", "batch"])
def test_scan_over_refined_table(mode):
    """CONCAT: the refinement does not change the scan. BATCH: every refined
    row is its own range, so the scan restarts at every cut of either
    range (what BATCH means for the refined table)."""
    announce("zip scan", mode)
    k = I.ints_0_100(N, 621) - 50
    out = _empty_segments(OUT_SPLIT, torch.int64)
    tab = B.zip_segments([_segments(k, X_SPLIT)], [out], mode=mode)
    B.dr_inclusive_scan(tab, B.make_view("identity", B.DR_I32), B.DR_I64)
    lens = [tab.host_rows[i].length for i in range(tab.n_segments)]
    omode = O.BATCH if mode == "batch" else O.CONCAT
    want = np.concatenate(O.scan(I.split(k, lens), None, O.I32, O.IDENTITY, mode=omode, out_dtype=O.I64))
    if mode == "concat":
        assert np.array_equal(want, np.cumsum(k.astype(np.int64)))
    assert np.array_equal(_flat(out), want)


def test_zip_stops_at_the_shortest_range():
    announce("zip shortest")
    k1, k2 = I.ints_0_100(N, 631), I.ints_0_100(N - 777, 632)
    tab = B.zip_segments([_segments(k1, X_SPLIT), _segments(k2, [N - 777])])
    assert tab.total_length == N - 777
    ri = torch.zeros(1, dtype=torch.int64, device=dev())
    B.dr_transform_reduce(tab, B.make_view("mul", B.DR_I32), 0, 0, ri)
    assert ri.item() == int(np.dot(k1[:N - 777].astype(np.int64), k2.astype(np.int64)))


@pytest.mark.parametrize("first,last", [(0, 17_000), (4_999, 40_000), (5_000, 18_001), (123, 124), (7, 7),
                                        (-5, 99_999)])
def test_trim_take_drop_then_reduce_and_scan(first, last):
    announce("trim", first, last)
    k = I.ints_0_100(N, 641) - 50
    segs = _segments(k, X_SPLIT, pad=2)
    trimmed = B.trim_segments(segs, first, last)
    f, l = min(max(first, 0), N), min(max(last, 0), N)
    assert sum(t.numel() for t in trimmed) == max(0, l - f)
    ri = torch.zeros(1, dtype=torch.int64, device=dev())
    B.dr_transform_reduce(B.segments([trimmed]) if trimmed else B.segments([[segs[0][:0]]]),
                          B.make_view("identity", B.DR_I32), 0, 0, ri)
    assert ri.item() == int(k[f:max(f, l)].astype(np.int64).sum())
    if trimmed:
        out = [torch.empty(t.numel(), dtype=torch.int64, device=dev()) for t in trimmed]
        B.dr_inclusive_scan(B.segments([trimmed], [out]), B.make_view("identity", B.DR_I32), B.DR_I64)
        assert np.array_equal(_flat(out), np.cumsum(k[f:l].astype(np.int64)))
    # take and drop are the two halves
    head, tail = B.take(segs, first), B.drop(segs, first)
    assert np.array_equal(np.concatenate([_flat(head), _flat(tail)]).astype(np.int64), k.astype(np.int64))
