"""dr_inclusive_scan_noalloc (the inclusive scan on the library's static
scratch, for callers that cannot allocate) against dr_inclusive_scan with a
workspace, through the C ABI: bit for bit (the same kernels; their carries
are sums in a fixed order), on two calls in a row with the second one
smaller, for a small table and a planned one (more than 64 rows); a call
that would not fit the scratch is rejected before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2406_00158_amd import binding as B
from paper_2406_00158_amd import inputs as I

from gpu_util import announce, dev, dev_to_np

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _cut(t, lengths):
    out, o = [], 0
    for n in lengths:
        out.append(t[o:o + n])
        o += n
    return out


def _pair(lengths, in_dt, out_dt, mode, seed):
    n = sum(lengths)
    x = I.ints_0_100(n, seed) - 50 if in_dt == B.DR_I32 else I.normal_f32(n, seed)
    xd = torch.from_numpy(x).to(dev())
    a = torch.full((n,), -1, dtype=B.TORCH_DTYPE[out_dt], device=dev())
    b = torch.full((n,), -2, dtype=B.TORCH_DTYPE[out_dt], device=dev())
    return (B.segments([_cut(xd, lengths)], [_cut(a, lengths)], mode=mode),
            B.segments([_cut(xd, lengths)], [_cut(b, lengths)], mode=mode), a, b)


CASES = [
    # (input, output, mode, flags, first lengths, second (smaller) lengths)
    (B.DR_F32, B.DR_F32, "concat", 0, [3_000_000, 0, 1_234_567, 77], [100_000, 5]),
    (B.DR_F32, B.DR_F32, "batch", B.DR_SCAN_REVERSE, [(k * 7919) % 40_000 + 1 for k in range(130)],
     [(k * 31) % 900 for k in range(70)]),
    (B.DR_I32, B.DR_I64, "batch", 0, [(k * 7919) % 40_000 for k in range(130)], [4097, 1, 8191]),
    (B.DR_I32, B.DR_I32, "concat", B.DR_SCAN_REVERSE, [1 << 22, 12345], [3, 4096, 2]),
]


@pytest.mark.parametrize("in_dt,out_dt,mode,flags,first,second", CASES)
def test_noalloc_scan_matches_the_workspace_scan(in_dt, out_dt, mode, flags, first, second):
    view = B.make_view("identity", in_dt)
    ws = B.Workspace(dev())
    B.dr_check_device_error()   # start from a clear device fault word (earlier tests plant faults)
    for call, lengths in enumerate((first, second)):
        announce("noalloc scan", in_dt, out_dt, mode, flags, "call", call, "rows", len(lengths), "n", sum(lengths))
        t_na, t_ws, a, b = _pair(lengths, in_dt, out_dt, mode, 300 + call)
        B.dr_inclusive_scan_noalloc(t_na, view, out_dt, flags)
        B.dr_inclusive_scan(t_ws, view, out_dt, flags, workspace=ws)
        got, want = dev_to_np(a), dev_to_np(b)
        assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), f"call {call}"
    assert ws.device_status() == 0
    assert B.dr_check_device_error() == 0


def test_noalloc_rejects_a_call_larger_than_its_scratch():
    announce("noalloc oversize")
    B.dr_check_device_error()
    x = torch.zeros(16, device=dev())
    y = torch.zeros(16, device=dev())
    tab = B.segments([[x]], [[y]])
    c = tab.c_table(host_check=False)
    c.total_length = 1 << 31              # 2^31 elements: more tiles than the scratch can track
    rows = (B.dr_segment * 1)()
    ctypes.memmove(rows, tab.host_rows, ctypes.sizeof(B.dr_segment))
    rows[0].length = 1 << 31
    dev_rows = torch.from_numpy(np.frombuffer(bytes(rows), dtype=np.uint8).copy()).to(dev())
    c.rows = dev_rows.data_ptr()
    view = B.make_view("identity", B.DR_F32)
    st = B.lib().dr_inclusive_scan_noalloc(ctypes.byref(c), ctypes.byref(view), B.DR_F32, 0, None,
                                           B._stream(dev()))
    assert st == B.DR_ERR_WORKSPACE
    assert b"static scratch" in B.lib().dr_last_error()
    torch.cuda.synchronize()
    assert np.all(dev_to_np(y) == 0)
    assert B.dr_check_device_error() == 0
