"""Thin ctypes binding of libdr.so (include/dr.h), with the same names.

Argument marshalling only: tensors become device pointers and lengths,
segment lists become dr_table rows, and every step of the computation runs
in the HIP kernels behind the C ABI. PyTorch supplies device memory and the
current stream. If the library is not built this module raises on import
of the library (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdr.so")

# --- constants mirrored from include/dr.h ------------------------------------
DR_OK = 0
DR_ERR_INVALID_ARG, DR_ERR_UNSUPPORTED, DR_ERR_WORKSPACE, DR_ERR_HIP, DR_ERR_NOT_ALIGNED, DR_ERR_DEVICE = \
    -1, -2, -3, -4, -5, -6
DR_I32, DR_F32, DR_BF16, DR_F64, DR_I64 = 0, 1, 2, 3, 4
DR_OP_IDENTITY, DR_OP_SQUARE, DR_OP_MUL, DR_OP_AXPY = 0, 1, 2, 3
DR_ACC_PLAIN, DR_ACC_COMPENSATED = 0, 1
DR_MODE_CONCAT, DR_MODE_BATCH = 0, 1
DR_SCAN_REVERSE, DR_SCAN_CARRY_F32, DR_SCAN_EXCLUSIVE = 1, 2, 4
DR_COMBINE_SUM, DR_COMBINE_MAX, DR_COMBINE_MIN = 0, 1, 2
COMBINES = {"sum": DR_COMBINE_SUM, "max": DR_COMBINE_MAX, "min": DR_COMBINE_MIN}
DR_ALGO_FOR_EACH, DR_ALGO_REDUCE, DR_ALGO_SCAN, DR_ALGO_SCAN_REDUCE, DR_ALGO_BROADCAST_MUL = 0, 1, 2, 3, 4
DR_SMALL_TABLE = 64
DR_MAX_ARITY = 4
DR_MAX_OUTPUTS = 2
DR_OP_BLACK_SCHOLES = 4
OP_ARITY = {DR_OP_IDENTITY: 1, DR_OP_SQUARE: 1, DR_OP_MUL: 2, DR_OP_AXPY: 2, DR_OP_BLACK_SCHOLES: 4}

TORCH_DTYPE = {DR_I32: torch.int32, DR_F32: torch.float32, DR_BF16: torch.bfloat16,
               DR_F64: torch.float64, DR_I64: torch.int64}
DR_DTYPE = {v: k for k, v in TORCH_DTYPE.items()}

OPS = {"identity": DR_OP_IDENTITY, "square": DR_OP_SQUARE, "mul": DR_OP_MUL, "axpy": DR_OP_AXPY,
       "black_scholes": DR_OP_BLACK_SCHOLES}
ACCS = {"plain": DR_ACC_PLAIN, "compensated": DR_ACC_COMPENSATED}
MODES = {"concat": DR_MODE_CONCAT, "batch": DR_MODE_BATCH}


class dr_view(ctypes.Structure):
    _fields_ = [("arity", ctypes.c_int32), ("in_dtype", ctypes.c_int32), ("op", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("alpha", ctypes.c_double)]


class dr_segment(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p * DR_MAX_ARITY), ("out", ctypes.c_void_p * DR_MAX_OUTPUTS),
                ("length", ctypes.c_int64), ("reserved", ctypes.c_int64)]


class dr_table(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_void_p), ("host_rows", ctypes.c_void_p),
                ("n_segments", ctypes.c_int64), ("total_length", ctypes.c_int64),
                ("mode", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class dr_span(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("length", ctypes.c_int64)]


class dr_range(ctypes.Structure):
    _fields_ = [("spans", ctypes.POINTER(dr_span)), ("n_spans", ctypes.c_int64),
                ("elem_size", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class dr_tuning(ctypes.Structure):
    _fields_ = [("block_threads", ctypes.c_int32), ("items_per_thread", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32)]


assert ctypes.sizeof(dr_segment) == 64
assert ctypes.sizeof(dr_view) == 24

EXPORTS = ["dr_abi_version", "dr_status_string", "dr_last_error", "dr_tuning_supported",
           "dr_workspace_bytes", "dr_workspace_init", "dr_plan", "dr_for_each",
           "dr_transform_reduce", "dr_inclusive_scan", "dr_scan_reduce", "dr_broadcast_mul",
           "dr_device_status", "dr_trim_segments", "dr_zip_segments", "dr_reduce", "dr_scan",
           "dr_check_device_error", "dr_inclusive_scan_noalloc"]

_lib = None


class DrError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{detail} (status {status})")
        self.status = status


def lib() -> ctypes.CDLL:
    """The loaded libdr.so. Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2406_00158_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, S = ctypes.c_void_p, ctypes.c_size_t
    i32, u32, i64 = ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64
    VP, TP, UP = ctypes.POINTER(dr_view), ctypes.POINTER(dr_table), ctypes.POINTER(dr_tuning)
    L.dr_abi_version.restype = ctypes.c_int
    L.dr_status_string.argtypes = [ctypes.c_int]
    L.dr_status_string.restype = ctypes.c_char_p
    L.dr_last_error.restype = ctypes.c_char_p
    L.dr_tuning_supported.argtypes = [i32, VP, i32, UP]
    L.dr_workspace_bytes.argtypes = [i32, i64, i64, VP, UP, ctypes.POINTER(S)]
    L.dr_workspace_init.argtypes = [P, S, P]
    L.dr_plan.argtypes = [TP, i32, VP, UP, P, S, P]
    L.dr_for_each.argtypes = [TP, VP, i32, P, S, UP, P]
    L.dr_transform_reduce.argtypes = [TP, VP, i32, P, P, P, S, UP, P]
    L.dr_inclusive_scan.argtypes = [TP, VP, i32, u32, P, S, UP, P]
    L.dr_scan_reduce.argtypes = [TP, VP, VP, i32, P, P, u32, P, S, UP, P]
    L.dr_broadcast_mul.argtypes = [TP, VP, P, i32, P, S, UP, P]
    L.dr_device_status.argtypes = [P, ctypes.POINTER(u32), P]
    L.dr_check_device_error.argtypes = [ctypes.POINTER(u32), P]
    L.dr_inclusive_scan_noalloc.argtypes = [TP, VP, i32, u32, UP, P]
    L.dr_reduce.argtypes = [TP, VP, i32, i32, P, P, P, S, UP, P]
    L.dr_scan.argtypes = [TP, VP, i32, i32, u32, P, P, S, UP, P]
    RP, I64P = ctypes.POINTER(dr_range), ctypes.POINTER(i64)
    L.dr_trim_segments.argtypes = [RP, i64, i64, ctypes.POINTER(dr_span), i64, I64P]
    L.dr_zip_segments.argtypes = [RP, i32, RP, i32, ctypes.POINTER(dr_segment), i64, I64P, I64P]
    for name in EXPORTS[3:]:
        if name not in ("dr_status_string", "dr_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(status: int) -> None:
    if status != DR_OK:
        raise DrError(status, lib().dr_last_error().decode())


def _stream(device: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def make_view(op: int | str, in_dtype: int | torch.dtype, alpha: float = 0.0) -> dr_view:
    op = OPS[op] if isinstance(op, str) else op
    dt = DR_DTYPE[in_dtype] if isinstance(in_dtype, torch.dtype) else in_dtype
    return dr_view(OP_ARITY[op], dt, op, 0, float(alpha))


DR_TUNE_TILE_PER_BLOCK = 1
DR_TUNE_SPECIALIZED = 2
DR_TUNE_TWO_PASS = 4
DR_TUNE_CHAINED = 8
# items per thread of the specialised-wave scan form, by input dtype (fused: 16)
WS_ITEMS = {DR_F32: 32, DR_BF16: 32, DR_I32: 32, DR_F64: 16}
WS_ITEMS_FUSED = 16


def make_tuning(items_per_thread: int | None, flags: int = 0, block_threads: int = 256) -> dr_tuning | None:
    """A launch shape; None (the library's defaults) when nothing is set."""
    if items_per_thread is None and not flags and block_threads == 256:
        return None
    return dr_tuning(int(block_threads), int(items_per_thread or 0), int(flags), 0)


# --- segment tables -----------------------------------------------------------

@dataclass
class Table:
    """A segment table: row k holds segment k of every zipped input and of
    every output stream, and its length. `keep` holds the tensors alive when
    the table was built with keep_alive=True."""
    n_segments: int
    mode: int
    device: torch.device
    host_rows: ctypes.Array = field(repr=False, default=None)
    dev_rows: torch.Tensor = field(repr=False, default=None)
    total_length: int = 0
    keep: list = field(repr=False, default_factory=list)

    def c_table(self, host_check: bool = True) -> dr_table:
        # the struct is rebuilt only when a field it mirrors has changed
        rows = self.dev_rows.data_ptr() if self.n_segments else None
        key = (host_check, rows, self.n_segments, self.total_length, self.mode)
        cached = self.__dict__.get("_c_cache")
        if cached is not None and cached[0] == key:
            return cached[1]
        host = ctypes.addressof(self.host_rows) if (host_check and self.n_segments) else None
        c = dr_table(rows, host, self.n_segments, self.total_length, self.mode, 0)
        self.__dict__["_c_cache"] = (key, c)
        return c


def segments(inputs, outputs=None, mode: int | str = DR_MODE_CONCAT, device=None,
             keep_alive: bool = True) -> Table:
    """Build a table from per-segment tensors.

    inputs:  list over zipped inputs of lists over segments of 1-D tensors
             (all inputs must have the same number of segments and lengths).
    outputs: optional list (at most 2) of such lists for output streams.
    keep_alive: hold references to the tensors (otherwise the caller must
             keep them alive while the table is used).
    """
    mode = MODES[mode] if isinstance(mode, str) else mode
    outputs = outputs or []
    if not inputs or len(inputs) > DR_MAX_ARITY or len(outputs) > DR_MAX_OUTPUTS:
        raise ValueError("between 1 and 4 inputs and at most 2 outputs")
    m = len(inputs[0])
    for lst in list(inputs) + list(outputs):
        if len(lst) != m:
            raise ValueError("every input/output needs the same number of segments")
    if device is None:
        first = next((t for t in inputs[0]), None)
        device = first.device if first is not None else torch.device("cuda")
    host = (dr_segment * max(1, m))()
    total = 0
    for k in range(m):
        n = inputs[0][k].numel()
        for lst in list(inputs) + list(outputs):
            t = lst[k]
            if t.dim() != 1 or t.numel() != n:
                raise ValueError(f"segment {k}: every zipped tensor must be 1-D with {n} elements")
            if not t.is_contiguous():
                raise ValueError(f"segment {k}: tensors must be contiguous")
            if t.device != device:
                raise ValueError(f"segment {k}: tensor on {t.device}, table on {device}")
        for i, lst in enumerate(inputs):
            host[k].in_[i] = lst[k].data_ptr() if n else None
        for i, lst in enumerate(outputs):
            host[k].out[i] = lst[k].data_ptr() if n else None
        host[k].length = n
        total += n
    raw = np.frombuffer(bytes(host), dtype=np.uint8)[: 64 * m]
    dev = torch.from_numpy(raw.copy()).to(device) if m else torch.empty(0, dtype=torch.uint8, device=device)
    keep = [list(inputs), list(outputs)] if keep_alive else []
    return Table(m, mode, device, host, dev, total, keep)


# --- workspace ----------------------------------------------------------------

class Workspace:
    """A caller-owned device workspace: grown on demand, zero-filled once by
    dr_workspace_init when (re)allocated, and tracking the plan it holds."""

    def __init__(self, device=None):
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        self.buf = None
        self.plan_key = None
        self._sizes = {}   # (algo, rows, length, view dtype/op/arity, tuning) -> bytes

    @property
    def ptr(self) -> int:
        return self.buf.data_ptr() if self.buf is not None else 0

    @property
    def nbytes(self) -> int:
        return self.buf.numel() if self.buf is not None else 0

    def ensure(self, nbytes: int) -> None:
        if self.buf is not None and self.buf.numel() >= nbytes:
            return
        nbytes = max(int(nbytes), 256)
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.buf.data_ptr()) % 256
        self.buf = self.buf[off: off + nbytes]
        check(lib().dr_workspace_init(self.ptr, nbytes, _stream(self.device)))
        self.plan_key = None

    def for_call(self, algo: int, table: Table, view: dr_view, tuning: dr_tuning | None) -> None:
        tptr = ctypes.byref(tuning) if tuning is not None else None
        tkey = (tuning.block_threads, tuning.items_per_thread, tuning.flags, tuning.reserved) if tuning else None
        skey = (algo, table.n_segments, table.total_length, view.in_dtype, view.op, view.arity, tkey)
        nbytes = self._sizes.get(skey)
        if nbytes is None:
            size = ctypes.c_size_t(0)
            check(lib().dr_workspace_bytes(algo, table.n_segments, table.total_length, ctypes.byref(view),
                                           tptr, ctypes.byref(size)))
            nbytes = self._sizes[skey] = size.value
        self.ensure(nbytes)
        if table.n_segments > DR_SMALL_TABLE:
            # a plan is built for one tile size: the algorithm and the tuning
            # fix it (the defaults differ between algorithms and dtypes)
            items = tuning.items_per_thread if tuning is not None else 0
            key = (table.dev_rows.data_ptr(), table.n_segments, table.total_length, view.in_dtype, algo, items)
            if key != self.plan_key:
                c = table.c_table(host_check=False)
                check(lib().dr_plan(ctypes.byref(c), algo, ctypes.byref(view), tptr, self.ptr,
                                    self.nbytes, _stream(self.device)))
                self.plan_key = key

    def device_status(self) -> int:
        flags = ctypes.c_uint32(0)
        st = lib().dr_device_status(self.ptr, ctypes.byref(flags), _stream(self.device))
        if st not in (DR_OK, -6):
            check(st)
        return int(flags.value)


_default_ws: dict = {}


def default_workspace(device) -> Workspace:
    device = torch.device(device)
    key = (device.type, device.index if device.index is not None else torch.cuda.current_device())
    ws = _default_ws.get(key)
    if ws is None:
        ws = _default_ws[key] = Workspace(torch.device("cuda", key[1]))
    return ws


# --- entry points (same names as the C ABI) -----------------------------------

def _tp(tuning):
    return ctypes.byref(tuning) if tuning is not None else None


def dr_for_each(table: Table, view: dr_view, out_dtype: int, workspace: Workspace | None = None,
                tuning: dr_tuning | None = None, host_check: bool = True) -> None:
    workspace = workspace or default_workspace(table.device)
    workspace.for_call(DR_ALGO_FOR_EACH, table, view, tuning)
    c = table.c_table(host_check)
    check(lib().dr_for_each(ctypes.byref(c), ctypes.byref(view), out_dtype, workspace.ptr, workspace.nbytes,
                            _tp(tuning), _stream(table.device)))


def dr_transform_reduce(table: Table, view: dr_view, acc: int, init, result: torch.Tensor,
                        workspace: Workspace | None = None, tuning: dr_tuning | None = None,
                        host_check: bool = True) -> None:
    workspace = workspace or default_workspace(table.device)
    workspace.for_call(DR_ALGO_REDUCE, table, view, tuning)
    c = table.c_table(host_check)
    init_c = ctypes.c_int64(int(init)) if view.in_dtype == DR_I32 else ctypes.c_double(float(init))
    check(lib().dr_transform_reduce(ctypes.byref(c), ctypes.byref(view), acc, ctypes.byref(init_c),
                                    result.data_ptr() if result.numel() else None, workspace.ptr,
                                    workspace.nbytes, _tp(tuning), _stream(table.device)))


def _init_ref(view: dr_view, init):
    """ctypes value for an initial value (None = the operator's identity)."""
    if init is None:
        return None, None
    v = ctypes.c_int64(int(init)) if view.in_dtype == DR_I32 else ctypes.c_double(float(init))
    return v, ctypes.byref(v)


def dr_reduce(table: Table, view: dr_view, combine: int, acc: int, init, result: torch.Tensor,
              workspace: Workspace | None = None, tuning: dr_tuning | None = None, host_check: bool = True) -> None:
    workspace = workspace or default_workspace(table.device)
    workspace.for_call(DR_ALGO_REDUCE, table, view, tuning)
    c = table.c_table(host_check)
    keep, ref = _init_ref(view, init)
    check(lib().dr_reduce(ctypes.byref(c), ctypes.byref(view), combine, acc, ref,
                          result.data_ptr() if result.numel() else None, workspace.ptr, workspace.nbytes,
                          _tp(tuning), _stream(table.device)))


def dr_scan(table: Table, view: dr_view, out_dtype: int, combine: int = DR_COMBINE_SUM, flags: int = 0, init=None,
            workspace: Workspace | None = None, tuning: dr_tuning | None = None, host_check: bool = True) -> None:
    workspace = workspace or default_workspace(table.device)
    workspace.for_call(DR_ALGO_SCAN, table, view, tuning)
    c = table.c_table(host_check)
    keep, ref = _init_ref(view, init)
    check(lib().dr_scan(ctypes.byref(c), ctypes.byref(view), out_dtype, combine, flags, ref, workspace.ptr,
                        workspace.nbytes, _tp(tuning), _stream(table.device)))


def dr_inclusive_scan(table: Table, view: dr_view, out_dtype: int, flags: int = 0,
                      workspace: Workspace | None = None, tuning: dr_tuning | None = None,
                      host_check: bool = True) -> None:
    workspace = workspace or default_workspace(table.device)
    workspace.for_call(DR_ALGO_SCAN, table, view, tuning)
    c = table.c_table(host_check)
    check(lib().dr_inclusive_scan(ctypes.byref(c), ctypes.byref(view), out_dtype, flags, workspace.ptr,
                                  workspace.nbytes, _tp(tuning), _stream(table.device)))


def dr_inclusive_scan_noalloc(table: Table, view: dr_view, out_dtype: int, flags: int = 0,
                              tuning: dr_tuning | None = None, host_check: bool = True) -> None:
    """dr_inclusive_scan on the library's static scratch (no workspace, no
    allocation)."""
    c = table.c_table(host_check)
    check(lib().dr_inclusive_scan_noalloc(ctypes.byref(c), ctypes.byref(view), out_dtype, flags, _tp(tuning),
                                          _stream(table.device)))


def dr_scan_reduce(table: Table, scan_view: dr_view, reduce_view: dr_view, acc: int, init: float,
                   result: torch.Tensor, flags: int = 0, workspace: Workspace | None = None,
                   tuning: dr_tuning | None = None, host_check: bool = True) -> None:
    workspace = workspace or default_workspace(table.device)
    workspace.for_call(DR_ALGO_SCAN_REDUCE, table, scan_view, tuning)
    c = table.c_table(host_check)
    init_c = ctypes.c_double(float(init))
    check(lib().dr_scan_reduce(ctypes.byref(c), ctypes.byref(scan_view), ctypes.byref(reduce_view), acc,
                               ctypes.byref(init_c), result.data_ptr() if result.numel() else None, flags,
                               workspace.ptr, workspace.nbytes, _tp(tuning), _stream(table.device)))


def dr_broadcast_mul(table: Table, view: dr_view, g: torch.Tensor, n_grads: int,
                     workspace: Workspace | None = None, tuning: dr_tuning | None = None,
                     host_check: bool = True) -> None:
    if g.dtype != torch.float64 or not g.is_contiguous():
        raise TypeError("g must be a contiguous float64 device tensor")
    workspace = workspace or default_workspace(table.device)
    workspace.for_call(DR_ALGO_BROADCAST_MUL, table, view, tuning)
    c = table.c_table(host_check)
    check(lib().dr_broadcast_mul(ctypes.byref(c), ctypes.byref(view), g.data_ptr(), n_grads,
                                 workspace.ptr, workspace.nbytes, _tp(tuning), _stream(table.device)))


def dr_device_status(workspace: Workspace) -> int:
    """Raw device fault flags of the workspace (0 = none); clears them."""
    return workspace.device_status()


def dr_check_device_error(device=None) -> int:
    """Raw bits of the device's library-wide fault word (0 = none), covering
    every call on the device, with or without a workspace; clears them."""
    device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    flags = ctypes.c_uint32(0)
    st = lib().dr_check_device_error(ctypes.byref(flags), _stream(device))
    if st not in (DR_OK, DR_ERR_DEVICE):
        check(st)
    return int(flags.value)


# --- segment algebra (section 4.4): take / drop and zip of non-aligned ranges ----

def _range_of(segs) -> tuple[dr_range, ctypes.Array]:
    """A dr_range over a list of 1-D contiguous tensors (one distributed
    range); returns the struct and the span array it points to."""
    if not segs:
        raise ValueError("a range needs at least one segment list entry (it may be empty)")
    es = segs[0].element_size()
    spans = (dr_span * len(segs))()
    for k, t in enumerate(segs):
        if t.dim() != 1 or not t.is_contiguous() or t.element_size() != es:
            raise ValueError(f"segment {k}: 1-D contiguous tensors of one element size")
        spans[k].ptr = t.data_ptr() if t.numel() else None
        spans[k].length = t.numel()
    return dr_range(spans, len(segs), es, 0), spans


def _view_at(segs, k0: int, ptr: int, length: int):
    """The tensor view of `length` elements at device address `ptr`, which
    lies in one of segs[k0:]; returns (view, index of that segment)."""
    for k in range(k0, len(segs)):
        t = segs[k]
        if t.numel() and t.data_ptr() <= ptr < t.data_ptr() + t.numel() * t.element_size():
            off = (ptr - t.data_ptr()) // t.element_size()
            return t[off:off + length], k
    raise RuntimeError("span outside the range's segments")


def trim_segments(segs, first: int, last: int) -> list:
    """The segments (tensor views) of the range restricted to its elements
    [first, last) (section 4.4, "Take and Drop"), computed by
    dr_trim_segments."""
    r, keep = _range_of(segs)
    out = (dr_span * max(1, len(segs)))()
    n = ctypes.c_int64(0)
    check(lib().dr_trim_segments(ctypes.byref(r), first, last, out, len(segs), ctypes.byref(n)))
    views, k = [], 0
    for i in range(n.value):
        v, k = _view_at(segs, k, out[i].ptr, out[i].length)
        views.append(v)
    return views


def take(segs, n: int) -> list:
    """The first n elements of a segmented range."""
    return trim_segments(segs, 0, n)


def drop(segs, n: int) -> list:
    """All but the first n elements of a segmented range."""
    return trim_segments(segs, n, sum(t.numel() for t in segs))


def zip_segments(inputs, outputs=None, mode: int | str = DR_MODE_CONCAT) -> Table:
    """Table of the zip of ranges whose segments need not be aligned
    (section 4.4, "Zip"): `inputs` / `outputs` are lists of ranges, each a
    list of 1-D tensors; dr_zip_segments refines their boundaries into
    aligned rows. The zip is as long as the shortest range."""
    outputs = outputs or []
    if not inputs or len(inputs) > DR_MAX_ARITY or len(outputs) > DR_MAX_OUTPUTS:
        raise ValueError("between 1 and 4 input ranges and at most 2 output ranges")
    rin = [_range_of(r) for r in inputs]
    rout = [_range_of(r) for r in outputs]
    ins = (dr_range * len(rin))(*[r for r, _ in rin])
    outs = (dr_range * max(1, len(rout)))(*[r for r, _ in rout])
    cap = sum(len(r) for r in inputs) + sum(len(r) for r in outputs)
    rows = (dr_segment * max(1, cap))()
    n, total = ctypes.c_int64(0), ctypes.c_int64(0)
    check(lib().dr_zip_segments(ins, len(rin), outs, len(rout), rows, cap, ctypes.byref(n), ctypes.byref(total)))
    m = n.value
    device = inputs[0][0].device
    host = (dr_segment * max(1, m))()
    ctypes.memmove(host, rows, ctypes.sizeof(dr_segment) * m)
    raw = np.frombuffer(bytes(host), dtype=np.uint8)[: 64 * m]
    dev = torch.from_numpy(raw.copy()).to(device) if m else torch.empty(0, dtype=torch.uint8, device=device)
    mode = MODES[mode] if isinstance(mode, str) else mode
    return Table(m, mode, device, host, dev, total.value, [list(inputs), list(outputs)])

