"""Segment algebra of section 4.4 (take / drop through trim_segments, and
the zip of ranges whose segments are not aligned), checked by brute force:
every composition of small ranges into segments, including empty segments,
against the element-by-element definition. The C functions only do
arithmetic on addresses, so the ranges here are synthetic addresses (one
distinct block per segment) and no memory is touched."""
import ctypes
import itertools
import os

import pytest

from paper_2406_00158_amd import binding as B

pytestmark = pytest.mark.skipif(not os.path.exists(B.LIB_PATH), reason="libdr.so not built")

ES = 4                      # element size of the synthetic ranges
BLOCK = 1 << 20             # address distance between segments


def _range(lengths, base):
    """A dr_range whose segment k starts at base + k*BLOCK; also returns a
    map address -> logical index for every element."""
    spans = (B.dr_span * max(1, len(lengths)))()
    where, o = {}, 0
    for k, n in enumerate(lengths):
        addr = base + k * BLOCK
        spans[k].ptr = addr
        spans[k].length = n
        for j in range(n):
            where[addr + j * ES] = o + j
        o += n
    return B.dr_range(spans, len(lengths), ES, 0), spans, where


def _seg_of(addr, base):
    return (addr - base) // BLOCK


def compositions(n, max_parts):
    """Segment length lists summing to n (each part >= 0 for inserted empty
    segments, at most max_parts parts)."""
    out = set()
    for parts in range(1, max_parts + 1):
        for cuts in itertools.combinations_with_replacement(range(n + 1), parts - 1):
            bounds = (0,) + cuts + (n,)
            out.add(tuple(bounds[i + 1] - bounds[i] for i in range(parts)))
    return sorted(out)


def _trim(r, first, last, cap):
    out = (B.dr_span * max(1, cap))()
    n = ctypes.c_int64(-1)
    st = B.lib().dr_trim_segments(ctypes.byref(r), first, last, out, cap, ctypes.byref(n))
    return st, [(out[i].ptr or 0, out[i].length) for i in range(max(n.value, 0))]


@pytest.mark.parametrize("n", range(0, 7))
def test_trim_every_composition_and_window(n):
    base = 0x10000000
    for lengths in compositions(n, 4):
        r, keep, where = _range(list(lengths), base)
        for first in range(-1, n + 2):
            for last in range(-1, n + 2):
                st, spans = _trim(r, first, last, len(lengths))
                assert st == 0, B.lib().dr_last_error()
                f, l = min(max(first, 0), n), min(max(last, 0), n)
                got = []
                for ptr, length in spans:
                    assert length > 0
                    # a span stays inside one segment
                    assert _seg_of(ptr, base) == _seg_of(ptr + (length - 1) * ES, base)
                    got += [where[ptr + j * ES] for j in range(length)]
                assert got == list(range(f, max(f, l))), (lengths, first, last, spans)
                # segments are kept in order, at most one span per segment
                segs = [_seg_of(p, base) for p, _ in spans]
                assert segs == sorted(set(segs))


def _zip(ranges_in, ranges_out, cap):
    ins = (B.dr_range * len(ranges_in))(*ranges_in)
    outs = (B.dr_range * max(1, len(ranges_out)))(*ranges_out)
    rows = (B.dr_segment * max(1, cap))()
    n, total = ctypes.c_int64(-1), ctypes.c_int64(-1)
    st = B.lib().dr_zip_segments(ins, len(ranges_in), outs, len(ranges_out), rows, cap, ctypes.byref(n),
                                 ctypes.byref(total))
    return st, rows, n.value, total.value


def _check_zip(lens_list, n_in):
    bases = [0x10000000 * (i + 1) for i in range(len(lens_list))]
    built = [_range(list(L), b) for L, b in zip(lens_list, bases)]
    cap = sum(len(L) for L in lens_list)
    st, rows, m, total = _zip([r for r, _, _ in built[:n_in]], [r for r, _, _ in built[n_in:]], cap)
    assert st == 0, B.lib().dr_last_error()
    shortest = min(sum(L) for L in lens_list)
    assert total == shortest
    pos = 0
    cuts = set()
    for L in lens_list:   # every segment boundary of every range, below the zip length
        o = 0
        for n in L:
            o += n
            cuts.add(o)
    for k in range(m):
        row = rows[k]
        length = row.length
        assert length > 0
        ptrs = [row.in_[i] for i in range(n_in)] + [row.out[j] for j in range(len(lens_list) - n_in)]
        for i, p in enumerate(ptrs):
            _, _, where = built[i]
            # the piece of range i is inside one of its segments and covers
            # the same logical positions as every other range's piece
            assert _seg_of(p, bases[i]) == _seg_of(p + (length - 1) * ES, bases[i])
            assert [where[p + j * ES] for j in range(length)] == list(range(pos, pos + length))
        for i in range(n_in, B.DR_MAX_ARITY):
            assert not row.in_[i]
        pos += length
        # coarsest refinement: a row ends only where some range's segment ends
        assert pos in cuts
    assert pos == shortest


@pytest.mark.parametrize("n", range(0, 6))
def test_zip_every_pair_of_compositions(n):
    comps = compositions(n, 3)
    for a in comps:
        for b in comps:
            _check_zip([a, b], 2)


def test_zip_three_ranges_with_outputs_and_unequal_lengths():
    for a, b, c in itertools.product(compositions(4, 3), compositions(5, 2), compositions(3, 3)):
        _check_zip([a, b, c], 2)     # two inputs, one output; the zip stops at the shortest
        _check_zip([a, b, c], 1)     # one input, two outputs


def test_zip_of_aligned_ranges_is_the_identity_refinement():
    lens = [7, 0, 3, 12]
    bases = (0x10000000, 0x20000000)
    r1, _, _ = _range(lens, bases[0])
    r2, _, _ = _range(lens, bases[1])
    st, rows, m, total = _zip([r1, r2], [], 8)
    assert st == 0 and m == 3 and total == 22
    assert [rows[k].length for k in range(m)] == [7, 3, 12]


def test_algebra_rejects_bad_arguments():
    L = B.lib()
    r, keep, _ = _range([3, 4], 0x10000000)
    st, _ = _trim(r, 0, 7, 1)                       # needs 2 spans
    assert st == B.DR_ERR_INVALID_ARG and b"capacity" in L.dr_last_error()
    bad, keep2, _ = _range([3, -1], 0x10000000)
    assert _trim(bad, 0, 2, 4)[0] == B.DR_ERR_INVALID_ARG
    zero = B.dr_range(keep, 2, 0, 0)
    assert _trim(zero, 0, 2, 4)[0] == B.DR_ERR_INVALID_ARG
    assert _zip([], [], 4)[0] == B.DR_ERR_INVALID_ARG
    assert _zip([r] * 5, [], 16)[0] == B.DR_ERR_INVALID_ARG
    assert _zip([r], [r, r, r], 16)[0] == B.DR_ERR_INVALID_ARG
    assert _zip([r, r], [], 1)[0] == B.DR_ERR_INVALID_ARG   # 2 rows needed
