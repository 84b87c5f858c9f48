"""Helpers of the GPU parity tests: device placement of the seeded inputs,
segment layouts, and the error bounds the tests assert (derived from the
arithmetic of each kernel)."""
from __future__ import annotations

import sys

import numpy as np
import torch

from paper_2406_00158_amd import binding as B

U32 = 2.0 ** -24
U64 = 2.0 ** -53
ITEMS = 16          # default elements per thread
BLOCK = 256


def gpu_available() -> bool:
    return torch.cuda.is_available()


def announce(*parts) -> None:
    """Name the case before it touches the GPU (flushed)."""
    print("[case]", *parts, file=sys.stderr, flush=True)


def dev() -> torch.device:
    return torch.device("cuda", 0)


def np_to_dev(a: np.ndarray) -> torch.Tensor:
    if a.dtype == np.uint16:   # bfloat16 bit patterns
        return torch.from_numpy(a.view(np.int16).copy()).to(dev()).view(torch.bfloat16)
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def dev_to_np(t: torch.Tensor) -> np.ndarray:
    if t.dtype == torch.bfloat16:
        return t.view(torch.int16).cpu().numpy().view(np.uint16)
    return t.cpu().numpy()


def carve(a: np.ndarray, lengths, offset: int = 0):
    """Segments as consecutive slices of one device buffer, starting
    `offset` elements into it (so segment starts have mixed alignment)."""
    buf = np_to_dev(np.concatenate([np.zeros(offset, dtype=a.dtype), a]))
    out, o = [], offset
    for n in lengths:
        out.append(buf[o:o + n])
        o += n
    return out, buf


def separate(a: np.ndarray, lengths):
    """One device allocation per segment."""
    out, o = [], 0
    for n in lengths:
        out.append(np_to_dev(a[o:o + n]))
        o += n
    return out


def empty_like_segments(lengths, dtype: torch.dtype, layout: str = "separate", offset: int = 0):
    if layout == "separate":
        return [torch.empty(n, dtype=dtype, device=dev()) for n in lengths]
    buf = torch.empty(sum(lengths) + offset, dtype=dtype, device=dev())
    out, o = [], offset
    for n in lengths:
        out.append(buf[o:o + n])
        o += n
    return out


def place(a: np.ndarray, lengths, layout: str, offset: int = 0):
    if layout == "separate":
        return separate(a, lengths)
    return carve(a, lengths, offset)[0]


def gather(segs) -> np.ndarray:
    if not segs:
        return np.zeros(0)
    return np.concatenate([dev_to_np(s) for s in segs]) if len(segs) else np.zeros(0)


# --- error bounds -------------------------------------------------------------

def scan_depth(items: int = ITEMS, elem_bytes: int = 4, block: int = BLOCK) -> int:
    """Most roundings an element's tile-local binary32 prefix goes through:
    the serial scan of one 16-byte vector, the six-step wave scan, the
    running offsets of the thread's earlier vectors and of the earlier
    waves (block / 64 of them), and two joins."""
    V = 16 // elem_bytes
    slots = items // V
    return (V - 1) + 6 + slots + block // 64 + 2


def scan_fp32_bound(ref: np.ndarray, absprefix: np.ndarray, items: int = ITEMS, elem_bytes: int = 4,
                    tiles: int = 1, block: int = BLOCK) -> np.ndarray:
    """|y - y_ref| bound of a binary32 scan with binary64 carries: one final
    rounding to binary32, the tile-local binary32 roundings, and the
    binary64 carry chain (a sum of at most `tiles` tile totals, in any
    order)."""
    d = scan_depth(items, elem_bytes, block)
    return U32 * np.abs(ref) + d * U32 * absprefix + (tiles + 2) * U64 * absprefix


def reduce_bound(absum: float, acc: str, items: int = ITEMS, in_bytes: int = 4, tiles: int = 1,
                 block: int = BLOCK) -> float:
    """|R - R_ref| bound of a reduction of `tiles` tiles of 256 * `items`
    elements. binary32 / bfloat16 inputs accumulate in binary32 through the
    workgroup: each thread runs serially over its elements (its tile's
    `items`, or in the streaming form those of every tile its workgroup
    takes: at most ceil(tiles / 256) tiles, the device running at least one
    workgroup per CU), then a 64-lane tree and the block / 64 waves in
    order; plain:
    recursive summation, (n + 10) u32 sum|v|; compensated: TwoSum/TwoProduct
    pairs leave only second-order terms, 4 ((n + 10) u32)^2 sum|v| (Ogita,
    Rump and Oishi's Sum2 / Dot2). The workgroup partials are widened and
    combined in binary64 over a tree of depth 2 log2(tiles) + a few."""
    per_thread = items * max(1, -(-tiles // 256))
    b64 = (2 * np.log2(max(tiles, 2)) + 8) * U64 * absum
    if in_bytes == 8:
        return (per_thread + 6 + block // 64) * U64 * absum + b64
    depth = per_thread + 6 + block // 64
    if acc == "plain":
        return depth * U32 * absum + b64
    return 4 * (depth * U32) ** 2 * absum + b64
