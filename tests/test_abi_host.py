"""The C ABI library loads, exports every entry point include/dr.h declares,
and rejects malformed arguments on the host before touching the GPU.
CPU only: every call here fails its host checks, so no kernel is launched."""
import ctypes
import os
import re

import pytest

from paper_2406_00158_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dr.h")

pytestmark = pytest.mark.skipif(not os.path.exists(B.LIB_PATH), reason="libdr.so not built")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dr_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = B.lib()
    names = _declared()
    assert "dr_for_each" in names and "dr_inclusive_scan" in names and "dr_transform_reduce" in names
    for n in names:
        assert hasattr(L, n), f"{n} declared in dr.h but not exported"
    assert set(names) == set(B.EXPORTS)


def test_chained_scan_form_scope():
    """The chained single pass scans one range (CONCAT) of binary32 or int32
    sums at 16 items per thread; anything else is refused on the host."""
    L = B.lib()
    v = B.make_view("identity", B.DR_F32)
    tu = B.make_tuning(16, B.DR_TUNE_CHAINED)
    sup = lambda algo, view, odt, t: L.dr_tuning_supported(algo, ctypes.byref(view), odt, ctypes.byref(t))
    assert sup(B.DR_ALGO_SCAN, v, B.DR_F32, tu) == 1
    assert sup(B.DR_ALGO_SCAN, B.make_view("identity", B.DR_I32), B.DR_I64, tu) == 1
    assert sup(B.DR_ALGO_SCAN, B.make_view("identity", B.DR_I32), B.DR_I32, tu) == 1
    assert sup(B.DR_ALGO_SCAN, B.make_view("identity", B.DR_F64), B.DR_F64, tu) == 0
    assert sup(B.DR_ALGO_SCAN, B.make_view("square", B.DR_F32), B.DR_F32, tu) == 0
    assert sup(B.DR_ALGO_SCAN, v, B.DR_F32, B.make_tuning(32, B.DR_TUNE_CHAINED)) == 0
    assert sup(B.DR_ALGO_SCAN_REDUCE, v, B.DR_F32, tu) == 0
    tb, keep_b = _host_table([((A,), (O,), 10)], 10)
    tb.mode = B.DR_MODE_BATCH
    assert L.dr_inclusive_scan(ctypes.byref(tb), ctypes.byref(v), B.DR_F32, 0, 0x40000000, 1 << 30,
                               ctypes.byref(tu), None) == B.DR_ERR_UNSUPPORTED
    assert b"CONCAT" in L.dr_last_error()
    init = ctypes.c_double(0.0)
    assert L.dr_scan(ctypes.byref(tb), ctypes.byref(v), B.DR_F32, B.DR_COMBINE_MAX, 0, ctypes.byref(init),
                     0x40000000, 1 << 30, ctypes.byref(tu), None) == B.DR_ERR_UNSUPPORTED
    del keep_b
    t, keep = _host_table([((A,), (O,), 10)], 10)
    tu2 = B.make_tuning(16, B.DR_TUNE_TILE_PER_BLOCK | B.DR_TUNE_TWO_PASS)
    assert L.dr_inclusive_scan(ctypes.byref(t), ctypes.byref(v), B.DR_F32, 0, 0x40000000, 1 << 30,
                               ctypes.byref(tu2), None) == B.DR_ERR_INVALID_ARG   # one form flag at most
    del keep


def test_check_device_error_rejects_null_flags():
    assert B.lib().dr_check_device_error(None, None) == B.DR_ERR_INVALID_ARG


def test_version_and_status_strings():
    L = B.lib()
    assert L.dr_abi_version() == 1
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert L.dr_status_string(code).decode()
    assert L.dr_status_string(12345).decode() == "unknown status"


def _host_table(rows, total, mode=B.DR_MODE_CONCAT):
    arr = (B.dr_segment * max(1, len(rows)))()
    for k, (ins, outs, n) in enumerate(rows):
        for i, p in enumerate(ins):
            arr[k].in_[i] = p
        for i, p in enumerate(outs):
            arr[k].out[i] = p
        arr[k].length = n
    # `rows` (device) gets a non-NULL dummy: the host checks fail before any use
    t = B.dr_table(0x1000, ctypes.addressof(arr), len(rows), total, mode, 0)
    return t, arr


A, Bp, O = 0x10000000, 0x20000000, 0x30000000


def _call_scan(t, view, out_dtype=B.DR_F32, flags=0, ws=0x40000000, ws_bytes=1 << 30):
    return B.lib().dr_inclusive_scan(ctypes.byref(t), ctypes.byref(view), out_dtype, flags, ws, ws_bytes,
                                     None, None)


def test_view_and_table_errors():
    L = B.lib()
    t, keep = _host_table([((A,), (O,), 10)], 10)
    bad_arity = B.dr_view(2, B.DR_F32, B.DR_OP_IDENTITY, 0, 0.0)
    assert _call_scan(t, bad_arity) == -1
    assert b"arity" in L.dr_last_error()
    bad_op = B.dr_view(1, B.DR_F32, 99, 0, 0.0)
    assert _call_scan(t, bad_op) == -1
    bad_dtype = B.dr_view(1, 77, B.DR_OP_IDENTITY, 0, 0.0)
    assert _call_scan(t, bad_dtype) == -2
    v = B.make_view("identity", B.DR_F32)
    assert _call_scan(t, v, out_dtype=B.DR_I64) == -2        # f32 -> i64 not a scan pair
    assert _call_scan(t, v, flags=0x80) == -1                # unknown flag
    vi = B.make_view("identity", B.DR_I32)
    assert _call_scan(t, vi, out_dtype=B.DR_I64, flags=B.DR_SCAN_CARRY_F32) == -1
    assert L.dr_inclusive_scan(None, ctypes.byref(v), B.DR_F32, 0, 0, 0, None, None) == -1
    t2 = B.dr_table(0x1000, None, 1, 10, 7, 0)               # unknown mode
    assert _call_scan(t2, v) == -1
    t3 = B.dr_table(0x1000, None, -1, 10, 0, 0)
    assert _call_scan(t3, v) == -1
    vi_axpy = B.dr_view(2, B.DR_I32, B.DR_OP_AXPY, 0, 0.5)   # int axpy needs integer alpha
    assert _call_scan(t, vi_axpy, out_dtype=B.DR_I64) == -1
    del keep


def test_host_row_errors():
    v = B.make_view("identity", B.DR_F32)
    t, keep = _host_table([((A,), (O,), -1)], -1 + 0)
    assert _call_scan(t, v) == -1                             # negative total_length
    t, keep = _host_table([((A,), (O,), -5), ((A,), (O,), 10)], 5)
    assert _call_scan(t, v) == -1 and b"negative length" in B.lib().dr_last_error()
    t, keep = _host_table([((A,), (O,), 10), ((A + 40,), (O + 40,), 10)], 21)
    assert _call_scan(t, v) == -1 and b"sum of lengths" in B.lib().dr_last_error()
    t, keep = _host_table([((0,), (O,), 10)], 10)
    assert _call_scan(t, v) == -1 and b"NULL" in B.lib().dr_last_error()
    t, keep = _host_table([((A,), (0,), 10)], 10)
    assert _call_scan(t, v) == -1 and b"NULL" in B.lib().dr_last_error()
    t, keep = _host_table([((A + 2,), (O,), 10)], 10)         # float pointer not 4-byte aligned
    assert _call_scan(t, v) == -1 and b"aligned" in B.lib().dr_last_error()
    # output overlapping another row's input
    t, keep = _host_table([((A,), (O,), 10), ((O + 8,), (O + 400,), 10)], 20)
    assert _call_scan(t, v) == -1 and b"overlaps" in B.lib().dr_last_error()
    # two outputs overlapping
    t, keep = _host_table([((A,), (O,), 10), ((A + 40,), (O + 20,), 10)], 20)
    assert _call_scan(t, v) == -1 and b"overlaps" in B.lib().dr_last_error()
    # in-place of a non-identity view is rejected; in-place identity scan passes
    # the host checks (it then needs a GPU, so only the failing case is run)
    sq = B.make_view("square", B.DR_F32)
    t, keep = _host_table([((A,), (A,), 10)], 10)
    assert _call_scan(t, sq) == -1
    del keep


def test_workspace_errors_and_sizes():
    L = B.lib()
    v = B.make_view("mul", B.DR_F32)
    size = ctypes.c_size_t(0)
    assert L.dr_workspace_bytes(B.DR_ALGO_REDUCE, 8, 1 << 28, ctypes.byref(v), None, ctypes.byref(size)) == 0
    small = size.value
    assert small >= 256 and small % 256 == 0
    assert L.dr_workspace_bytes(B.DR_ALGO_REDUCE, 10_000, 1 << 28, ctypes.byref(v), None,
                                ctypes.byref(size)) == 0
    assert size.value > small                                  # large tables hold a plan
    assert L.dr_workspace_bytes(B.DR_ALGO_FOR_EACH, 8, 1 << 28, ctypes.byref(v), None,
                                ctypes.byref(size)) == 0
    assert size.value == 256                                   # header only
    bad_tune = B.dr_tuning(128, 16, 0, 0)
    assert L.dr_workspace_bytes(B.DR_ALGO_REDUCE, 8, 100, ctypes.byref(v), ctypes.byref(bad_tune),
                                ctypes.byref(size)) == -2
    t, keep = _host_table([((A, Bp), (), 10)], 10)
    init = ctypes.c_double(0.0)
    # workspace missing, misaligned, too small
    assert L.dr_transform_reduce(ctypes.byref(t), ctypes.byref(v), 1, ctypes.byref(init), O, None, 0, None,
                                 None) == -3
    assert L.dr_transform_reduce(ctypes.byref(t), ctypes.byref(v), 1, ctypes.byref(init), O, 0x40000010,
                                 1 << 20, None, None) == -3
    assert L.dr_transform_reduce(ctypes.byref(t), ctypes.byref(v), 1, ctypes.byref(init), O, 0x40000000,
                                 256, None, None) == -3
    assert L.dr_transform_reduce(ctypes.byref(t), ctypes.byref(v), 5, ctypes.byref(init), O, 0x40000000,
                                 1 << 20, None, None) == -1    # unknown acc
    assert L.dr_transform_reduce(ctypes.byref(t), ctypes.byref(v), 1, None, O, 0x40000000, 1 << 20, None,
                                 None) == -1                   # NULL init
    assert L.dr_workspace_init(None, 1024, None) == -3
    assert L.dr_workspace_init(0x40000010, 1024, None) == -3
    flags = ctypes.c_uint32(0)
    assert L.dr_device_status(None, ctypes.byref(flags), None) == -3
    del keep


def test_fused_and_adjoint_argument_checks():
    L = B.lib()
    t, keep = _host_table([((A, Bp), (O,), 10)], 10)
    sv = B.make_view("identity", B.DR_F32)
    rv = B.make_view("mul", B.DR_F32)
    init = ctypes.c_double(0.0)
    assert L.dr_scan_reduce(ctypes.byref(t), ctypes.byref(rv), ctypes.byref(rv), 1, ctypes.byref(init), O,
                            0, 0x40000000, 1 << 20, None, None) == -2
    assert L.dr_scan_reduce(ctypes.byref(t), ctypes.byref(sv), ctypes.byref(sv), 1, ctypes.byref(init), O,
                            0, 0x40000000, 1 << 20, None, None) == -2
    assert L.dr_scan_reduce(ctypes.byref(t), ctypes.byref(sv), ctypes.byref(rv), 1, ctypes.byref(init), O,
                            2, 0x40000000, 1 << 20, None, None) == -1
    assert L.dr_broadcast_mul(ctypes.byref(t), ctypes.byref(rv), None, 2, None, 0, None, None) == -1
    assert L.dr_broadcast_mul(ctypes.byref(t), ctypes.byref(rv), 0x50000000, 3, None, 0, None, None) == -1
    vi = B.make_view("mul", B.DR_I32)
    assert L.dr_broadcast_mul(ctypes.byref(t), ctypes.byref(vi), 0x50000000, 1, None, 0, None, None) == -2
    del keep


def test_tuning_supported_table():
    L = B.lib()
    v = B.make_view("mul", B.DR_F32)
    assert L.dr_tuning_supported(B.DR_ALGO_REDUCE, ctypes.byref(v), B.DR_ACC_COMPENSATED, None) == 1
    t32 = B.dr_tuning(256, 32, 0, 0)
    assert L.dr_tuning_supported(B.DR_ALGO_REDUCE, ctypes.byref(v), B.DR_ACC_COMPENSATED, ctypes.byref(t32)) == 1
    t7 = B.dr_tuning(256, 7, 0, 0)
    assert L.dr_tuning_supported(B.DR_ALGO_REDUCE, ctypes.byref(v), B.DR_ACC_COMPENSATED, ctypes.byref(t7)) == 0
    vs = B.make_view("identity", B.DR_I32)
    assert L.dr_tuning_supported(B.DR_ALGO_SCAN, ctypes.byref(vs), B.DR_I64, None) == 1
    assert L.dr_tuning_supported(B.DR_ALGO_SCAN, ctypes.byref(vs), B.DR_F32, None) == 0


def test_generic_operator_argument_errors():
    """dr_scan / dr_reduce reject what they do not support before anything
    is enqueued (every call here fails a host check)."""
    L = B.lib()
    t, keep = _host_table([((A,), (O,), 10)], 10)
    v = B.make_view("identity", B.DR_F32)
    sq = B.make_view("square", B.DR_F32)
    init = ctypes.c_double(1.5)

    def scan(view, combine, flags=0, tuning=None, out=B.DR_F32):
        return L.dr_scan(ctypes.byref(t), ctypes.byref(view), out, combine, flags, ctypes.byref(init),
                         0x40000000, 1 << 30, ctypes.byref(tuning) if tuning else None, None)

    assert scan(v, 7) == -1 and b"combine" in L.dr_last_error()
    assert scan(v, B.DR_COMBINE_SUM, flags=0x40) == -1                       # unknown flag
    assert scan(sq, B.DR_COMBINE_MAX) == -2 and b"identity" in L.dr_last_error()
    assert scan(v, B.DR_COMBINE_MIN, flags=B.DR_SCAN_CARRY_F32) == -2
    assert scan(v, B.DR_COMBINE_MAX, tuning=B.make_tuning(16, B.DR_TUNE_TILE_PER_BLOCK)) == -2
    assert scan(v, B.DR_COMBINE_MAX, tuning=B.make_tuning(64)) == -2
    # the specialised-wave form: sums of the identity view at its own tile size
    ws_tu = B.make_tuning(B.WS_ITEMS[B.DR_F32], B.DR_TUNE_SPECIALIZED)
    assert scan(v, B.DR_COMBINE_MAX, tuning=ws_tu) == -2
    assert scan(sq, B.DR_COMBINE_SUM, tuning=ws_tu) == -2                  # square view: not built
    assert scan(v, B.DR_COMBINE_SUM, tuning=B.make_tuning(16, B.DR_TUNE_SPECIALIZED)) == -2
    assert b"items per thread" in L.dr_last_error()
    assert scan(v, B.DR_COMBINE_SUM, tuning=B.make_tuning(32, B.DR_TUNE_SPECIALIZED | B.DR_TUNE_TILE_PER_BLOCK)) == -1
    assert scan(v, B.DR_COMBINE_MAX, out=B.DR_I64) == -2                     # f32 -> i64 not a scan pair
    # the exclusive flag belongs to dr_scan, not dr_inclusive_scan
    assert _call_scan(t, v, flags=B.DR_SCAN_EXCLUSIVE) == -1
    tr, keep2 = _host_table([((A,), (), 10)], 10)
    assert L.dr_reduce(ctypes.byref(tr), ctypes.byref(v), 9, 0, None, O, 0x40000000, 1 << 30, None, None) == -1
    assert L.dr_reduce(ctypes.byref(tr), ctypes.byref(v), B.DR_COMBINE_MAX, 0, None, None, 0x40000000, 1 << 30,
                       None, None) == -1                                     # result NULL
    assert L.dr_reduce(ctypes.byref(tr), ctypes.byref(v), B.DR_COMBINE_MIN, 0, None, O, 0x40000000, 1 << 30,
                       ctypes.byref(B.make_tuning(32)), None) == -2
    del keep, keep2


def test_wide_look_back_shapes():
    """512- and 1024-thread workgroups (and 4 / 8 items at 256) exist for the
    look-back scan only: binary32 sums with binary64 carries, plain or fused
    with the compensated dot. Everything else with them is refused on the
    host, and workspace sizes follow the tile of block_threads x items."""
    L = B.lib()
    vid, vmul = B.make_view("identity", B.DR_F32), B.make_view("mul", B.DR_F32)
    sup = lambda algo, v, odt, tu: L.dr_tuning_supported(algo, ctypes.byref(v), odt, ctypes.byref(tu))
    lb = B.DR_TUNE_TILE_PER_BLOCK
    for block, items in ((512, 8), (512, 16), (512, 32), (1024, 4), (1024, 8), (1024, 16), (256, 4), (256, 8)):
        tu = B.make_tuning(items, lb, block)
        assert sup(B.DR_ALGO_SCAN, vid, B.DR_F32, tu) == 1, (block, items)
        assert sup(B.DR_ALGO_SCAN_REDUCE, vid, B.DR_F32, tu) == 1, (block, items)
        # the same shape in the two-pass form, for other dtypes or algorithms: not built
        assert sup(B.DR_ALGO_SCAN, vid, B.DR_F32, B.make_tuning(items, B.DR_TUNE_TWO_PASS, block)) == 0
        assert sup(B.DR_ALGO_SCAN, B.make_view("identity", B.DR_I32), B.DR_I64, tu) == 0
    assert sup(B.DR_ALGO_SCAN, vid, B.DR_F32, B.make_tuning(32, lb, 1024)) == 0   # 128 registers per thread
    assert sup(B.DR_ALGO_REDUCE, vmul, B.DR_ACC_COMPENSATED, B.make_tuning(16, 0, 512)) == 0
    assert sup(B.DR_ALGO_FOR_EACH, vid, B.DR_F32, B.make_tuning(16, 0, 512)) == 0
    assert sup(B.DR_ALGO_SCAN, vid, B.DR_F32, B.make_tuning(16, lb, 384)) == 0
    # tile = block x items: 2^28 elements at 512 x 16 need the tile words of 256 x 32
    size = ctypes.c_size_t(0)
    sizes = []
    for block, items in ((512, 16), (256, 32), (256, 16)):
        tu = B.make_tuning(items, lb, block)
        assert L.dr_workspace_bytes(B.DR_ALGO_SCAN, 16, 1 << 28, ctypes.byref(vid), ctypes.byref(tu),
                                    ctypes.byref(size)) == 0
        sizes.append(size.value)
    assert sizes[0] == sizes[1] < sizes[2]
    # calls: the wide shape in the two-pass form, and a reduction at 512 threads, fail before any launch
    t, keep = _host_table([((A,), (O,), 10)], 10)
    tu = B.make_tuning(16, B.DR_TUNE_TWO_PASS, 512)
    assert L.dr_inclusive_scan(ctypes.byref(t), ctypes.byref(vid), B.DR_F32, 0, 0x40000000, 1 << 30,
                               ctypes.byref(tu), None) == B.DR_ERR_UNSUPPORTED
    assert b"look-back" in L.dr_last_error()
    tr, keep2 = _host_table([((A, Bp), (), 10)], 10)
    init = ctypes.c_double(0.0)
    tu = B.make_tuning(16, 0, 1024)
    assert L.dr_transform_reduce(ctypes.byref(tr), ctypes.byref(vmul), 1, ctypes.byref(init), O, 0x40000000,
                                 1 << 20, ctypes.byref(tu), None) == B.DR_ERR_UNSUPPORTED
    del keep, keep2
