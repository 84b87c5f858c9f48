"""Differentiable segmented scan / dot / sum of squares.

A range here is one flat 1-D tensor cut into consecutive segments of the
given lengths: the one-GPU form of the paper's block-distributed vector
(section 4.2.1), where each segment is a contiguous block. `mode` is
"concat" (the segments are one range) or "batch" (each segment is its own
range: per-segment results, the scan restarts per segment).

Backward passes are written by hand and run in the library's kernels:
  * inclusive_scan: the adjoint is the reverse (suffix) inclusive scan of
    the upstream gradient, within the same ranges;
  * dot(x, y): dR/dx = g * y and dR/dy = g * x, one fused broadcast multiply
    over the zipped inputs that writes both gradients;
  * sum of squares: dR/dx = 2 g x;
  * fused scan + dot: gx = reverse_scan(g_scan) + g_dot * y, gy = g_dot * x.
"""
from __future__ import annotations

import torch

from . import binding as B

_TABLES: dict = {}


def _pieces(t: torch.Tensor, lengths):
    out, o = [], 0
    for n in lengths:
        out.append(t[o:o + n])
        o += n
    if o != t.numel():
        raise ValueError(f"lengths sum to {o}, tensor has {t.numel()} elements")
    return out


def table(inputs, outputs, lengths, mode) -> B.Table:
    """Segment table over flat tensors cut at `lengths` (cached by pointers)."""
    key = (tuple(t.data_ptr() for t in inputs), tuple(t.data_ptr() for t in outputs), tuple(lengths), mode,
           tuple(t.dtype for t in inputs))
    tab = _TABLES.get(key)
    if tab is None:
        if len(_TABLES) > 256:
            _TABLES.clear()
        tab = B.segments([_pieces(t, lengths) for t in inputs], [_pieces(t, lengths) for t in outputs],
                         mode=mode, keep_alive=False)
        _TABLES[key] = tab
    return tab


def _check(x: torch.Tensor) -> torch.Tensor:
    if x.dim() != 1:
        raise ValueError("expected a 1-D tensor")
    if x.device.type != "cuda":
        raise ValueError("the segmented kernels run on the GPU; move the tensor to cuda first")
    return x.contiguous()


def _nres(lengths, mode) -> int:
    return len(lengths) if mode == "batch" else 1


def _scan(x, lengths, mode, reverse):
    out = torch.empty_like(x)
    B.dr_inclusive_scan(table([x], [out], lengths, mode), B.make_view("identity", x.dtype), B.DR_DTYPE[x.dtype],
                        B.DR_SCAN_REVERSE if reverse else 0)
    return out


def _grad_mul(x, y, g, lengths, mode, n_grads):
    gx, gy = torch.empty_like(x), torch.empty_like(y)
    outs = [gx, gy][:n_grads]
    B.dr_broadcast_mul(table([x, y], outs, lengths, mode), B.make_view("mul", x.dtype), g.contiguous(), n_grads)
    return gx, gy


def _add(a, b):
    out = torch.empty_like(a)
    B.dr_for_each(table([a, b], [out], [a.numel()], "concat"), B.make_view("axpy", a.dtype, 1.0),
                  B.DR_DTYPE[a.dtype])
    return out


class ScanFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, lengths, mode):
        x = _check(x)
        ctx.lengths, ctx.mode = tuple(lengths), mode
        return _scan(x, ctx.lengths, mode, reverse=False)

    @staticmethod
    def backward(ctx, gy):
        return _scan(_check(gy), ctx.lengths, ctx.mode, reverse=True), None, None


class DotFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y, lengths, mode, acc):
        x, y = _check(x), _check(y)
        ctx.lengths, ctx.mode = tuple(lengths), mode
        res = torch.empty(_nres(lengths, mode), dtype=torch.float64, device=x.device)
        B.dr_transform_reduce(table([x, y], [], ctx.lengths, mode), B.make_view("mul", x.dtype), B.ACCS[acc], 0.0,
                              res)
        ctx.save_for_backward(x, y)
        return res

    @staticmethod
    def backward(ctx, g):
        x, y = ctx.saved_tensors
        gx, gy = _grad_mul(x, y, g.to(torch.float64), ctx.lengths, ctx.mode, 2)
        return gx, gy, None, None, None


class SumSqFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, lengths, mode, acc):
        x = _check(x)
        ctx.lengths, ctx.mode = tuple(lengths), mode
        res = torch.empty(_nres(lengths, mode), dtype=torch.float64, device=x.device)
        B.dr_transform_reduce(table([x], [], ctx.lengths, mode), B.make_view("square", x.dtype), B.ACCS[acc], 0.0,
                              res)
        ctx.save_for_backward(x)
        return res

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        gx = torch.empty_like(x)
        B.dr_broadcast_mul(table([x], [gx], ctx.lengths, ctx.mode), B.make_view("square", x.dtype),
                           g.to(torch.float64).contiguous(), 1)
        return gx, None, None, None


class ScanDotFn(torch.autograd.Function):
    """Fused forward: per range, inclusive_scan(x) and dot(x, y) in one launch."""

    @staticmethod
    def forward(ctx, x, y, lengths, mode, acc):
        x, y = _check(x), _check(y)
        ctx.lengths, ctx.mode = tuple(lengths), mode
        s = torch.empty_like(x)
        res = torch.empty(_nres(lengths, mode), dtype=torch.float64, device=x.device)
        B.dr_scan_reduce(table([x, y], [s], ctx.lengths, mode), B.make_view("identity", x.dtype),
                         B.make_view("mul", x.dtype), B.ACCS[acc], 0.0, res)
        ctx.save_for_backward(x, y)
        return s, res

    @staticmethod
    def backward(ctx, g_scan, g_dot):
        x, y = ctx.saved_tensors
        gx_scan = _scan(_check(g_scan), ctx.lengths, ctx.mode, reverse=True) if g_scan is not None else None
        if g_dot is None:
            return gx_scan, None, None, None, None
        gx_dot, gy = _grad_mul(x, y, g_dot.to(torch.float64), ctx.lengths, ctx.mode, 2)
        gx = gx_dot if gx_scan is None else _add(gx_scan, gx_dot)
        return gx, gy, None, None, None


def inclusive_scan(x, lengths, mode="concat"):
    return ScanFn.apply(x, tuple(lengths), mode)


def dot(x, y, lengths, mode="concat", acc="compensated"):
    return DotFn.apply(x, y, tuple(lengths), mode, acc)


def sum_of_squares(x, lengths, mode="concat", acc="compensated"):
    return SumSqFn.apply(x, tuple(lengths), mode, acc)


def scan_dot(x, y, lengths, mode="batch", acc="compensated"):
    return ScanDotFn.apply(x, y, tuple(lengths), mode, acc)
