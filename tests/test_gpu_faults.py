"""Device-detected faults are reported for every call, with or without a
workspace: a malformed device table (no host mirror, so only the kernels
can see it) in for_each and broadcast_mul is flagged in the call's
workspace and in the device's fault word, the kernels exit normally
without touching the outputs, and the next well-formed call works. The
faults are planted in the table rows from the host; every pointer the
kernels could follow is valid or NULL, and the kernels check the rows
before any element access."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2406_00158_amd import binding as B

from gpu_util import announce, dev, dev_to_np

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

BAD_TABLE, TIMEOUT, PLAN = 1, 2, 4
SENTINEL = -7.0


def _upload(tab):
    raw = np.frombuffer(bytes(tab.host_rows), dtype=np.uint8)[: 64 * tab.n_segments]
    tab.dev_rows = torch.from_numpy(raw.copy()).to(dev())
    tab.__dict__.pop("_c_cache", None)


def _case(m, fault):
    """x, y -> out tables over m segments of 40 elements; the device copy of
    the rows carries `fault`: 'null_input' (row 1 has no in[0]) or 'length'
    (row 0 claims one more element than the table's total allows)."""
    n = 40 * m
    x = torch.arange(n, dtype=torch.float32, device=dev())
    y = torch.full((n,), 2.0, device=dev())
    out = torch.full((n,), SENTINEL, device=dev())
    out2 = torch.full((n,), SENTINEL, device=dev())
    cut = lambda t: [t[40 * k:40 * (k + 1)] for k in range(m)]
    tab_fe = B.segments([cut(x), cut(y)], [cut(out)])
    tab_bm = B.segments([cut(x), cut(y)], [cut(out), cut(out2)])
    for tab in (tab_fe, tab_bm):
        if fault == "null_input":
            tab.host_rows[1].in_[0] = None
        else:
            tab.host_rows[0].length = 41
        _upload(tab)
    return x, y, out, out2, tab_fe, tab_bm, cut


@pytest.mark.parametrize("m", [4, 130])
@pytest.mark.parametrize("fault", ["null_input", "length"])
def test_for_each_and_broadcast_mul_flag_malformed_device_tables(m, fault):
    announce("faults", m, fault)
    B.dr_check_device_error()   # start from a clear fault word (earlier tests plant faults too)
    x, y, out, out2, tab_fe, tab_bm, cut = _case(m, fault)
    want_bits = BAD_TABLE if m <= B.DR_SMALL_TABLE else (BAD_TABLE | PLAN)
    v = B.make_view("mul", B.DR_F32)
    for call in ("for_each", "broadcast_mul"):
        ws = B.Workspace(dev())
        if call == "for_each":
            B.dr_for_each(tab_fe, v, B.DR_F32, workspace=ws, host_check=False)
        else:
            g = torch.ones(1, dtype=torch.float64, device=dev())
            B.dr_broadcast_mul(tab_bm, v, g, 2, workspace=ws, host_check=False)
        torch.cuda.synchronize()
        got_ws, got_dev = ws.device_status(), B.dr_check_device_error()
        assert got_ws & BAD_TABLE and (got_ws & ~want_bits) == 0, (call, got_ws)
        assert got_dev & BAD_TABLE and (got_dev & ~want_bits) == 0, (call, got_dev)
        assert np.all(dev_to_np(out) == SENTINEL) and np.all(dev_to_np(out2) == SENTINEL), call
        assert ws.device_status() == 0 and B.dr_check_device_error() == 0   # both cleared by the reads
    # the same workspace and device then run a well-formed call normally
    good = B.segments([cut(x), cut(y)], [cut(out)])
    ws = B.Workspace(dev())
    B.dr_for_each(good, v, B.DR_F32, workspace=ws)
    assert np.array_equal(dev_to_np(out), 2.0 * np.arange(40 * m, dtype=np.float32))
    assert ws.device_status() == 0 and B.dr_check_device_error() == 0


def test_for_each_without_workspace_reports_to_the_device_fault_word():
    """Through the C ABI with no workspace at all (a small table): the fault
    can only reach the device's fault word."""
    announce("faults without workspace")
    B.dr_check_device_error()
    x, y, out, out2, tab_fe, tab_bm, cut = _case(4, "null_input")
    c = tab_fe.c_table(host_check=False)
    v = B.make_view("mul", B.DR_F32)
    st = B.lib().dr_for_each(ctypes.byref(c), ctypes.byref(v), B.DR_F32, None, 0, None,
                             B._stream(dev()))
    assert st == B.DR_OK
    g = torch.ones(1, dtype=torch.float64, device=dev())
    c2 = tab_bm.c_table(host_check=False)
    st = B.lib().dr_broadcast_mul(ctypes.byref(c2), ctypes.byref(v), g.data_ptr(), 2, None, 0, None,
                                  B._stream(dev()))
    assert st == B.DR_OK
    torch.cuda.synchronize()
    assert B.dr_check_device_error() == BAD_TABLE
    assert np.all(dev_to_np(out) == SENTINEL) and np.all(dev_to_np(out2) == SENTINEL)
    flags = ctypes.c_uint32(99)
    assert B.lib().dr_check_device_error(ctypes.byref(flags), B._stream(dev())) == B.DR_OK
    assert flags.value == 0


def test_wait_timeout_is_flagged_and_the_launch_completes(monkeypatch):
    """A bound of one tick on every wait between workgroups (set from the
    host): the single-pass look-back scan and a reduction's combine give up
    waiting, flag a timeout (bit 2) and return; with the normal bound the
    same calls are correct again."""
    announce("wait timeout")
    B.dr_check_device_error()
    n = 1 << 22
    x = torch.ones(n, device=dev())
    out = torch.empty(n, device=dev())
    tab = B.segments([[x]], [[out]])
    v = B.make_view("identity", B.DR_F32)
    lb = B.make_tuning(16, B.DR_TUNE_TILE_PER_BLOCK)
    res = torch.zeros(1, dtype=torch.float64, device=dev())
    ws = B.Workspace(dev())
    monkeypatch.setenv("DR_SPIN_TICKS", "1")
    B.dr_inclusive_scan(tab, v, B.DR_F32, workspace=ws, tuning=lb)
    B.dr_transform_reduce(B.segments([[x]]), v, B.DR_ACC_PLAIN, 0.0, res, workspace=ws, tuning=lb)
    torch.cuda.synchronize()
    flags = ws.device_status()
    assert flags & TIMEOUT and (flags & ~TIMEOUT) == 0, flags
    assert B.dr_check_device_error() & TIMEOUT
    monkeypatch.delenv("DR_SPIN_TICKS")
    B.dr_inclusive_scan(tab, v, B.DR_F32, workspace=ws, tuning=lb)
    B.dr_transform_reduce(B.segments([[x]]), v, B.DR_ACC_PLAIN, 0.0, res, workspace=ws, tuning=lb)
    assert np.array_equal(dev_to_np(out), np.arange(1, n + 1, dtype=np.float32))
    assert res.item() == n
    assert ws.device_status() == 0 and B.dr_check_device_error() == 0
