"""The autotuner's search space, on the host: every launch shape the
library has a kernel for (block_threads x items_per_thread x scan form, as
dr_tuning_supported reports), and the labels it records."""
import os

import pytest

from paper_2406_00158_amd import autotune as AT
from paper_2406_00158_amd import binding as B

pytestmark = pytest.mark.skipif(not os.path.exists(B.LIB_PATH), reason="libdr.so not built")


def test_scan_reduce_candidates_span_blocks_items_and_forms():
    v = B.make_view("identity", B.DR_F32)
    c = AT.candidates(B.DR_ALGO_SCAN_REDUCE, v, B.DR_F32)
    shapes = {(t.block_threads, t.items_per_thread, AT.form_name(t.flags)) for t in c}
    for items in (16, 32, 64):
        assert (256, items, "two_pass") in shapes and (256, items, "look_back") in shapes
    for block, items in ((256, 4), (256, 8), (512, 8), (512, 16), (512, 32), (1024, 4), (1024, 8), (1024, 16)):
        assert (block, items, "look_back") in shapes and (block, items, "two_pass") not in shapes
    assert {b for b, _, _ in shapes} == set(AT.BLOCKS)
    assert len(shapes) == len(c) == 14


def test_other_algorithms_keep_256_threads():
    vm = B.make_view("mul", B.DR_F32)
    c = AT.candidates(B.DR_ALGO_REDUCE, vm, B.DR_ACC_COMPENSATED)
    assert c and all(t.block_threads == 256 and t.flags == 0 for t in c)
    assert {t.items_per_thread for t in c} <= {16, 32, 64} and 16 in {t.items_per_thread for t in c}
    vi = B.make_view("identity", B.DR_I32)
    c = AT.candidates(B.DR_ALGO_SCAN, vi, B.DR_I64)
    assert all(t.block_threads == 256 for t in c)
    assert {(t.items_per_thread, AT.form_name(t.flags)) for t in c} == {
        (i, f) for i in (16, 32, 64) for f in ("two_pass", "look_back")}


def test_labels():
    assert AT.label(B.dr_tuning(512, 16, B.DR_TUNE_TILE_PER_BLOCK, 0)) == "512x16/look_back"
    assert AT.label(B.dr_tuning(256, 32, B.DR_TUNE_TWO_PASS, 0)) == "256x32/two_pass"
    assert AT.label(B.dr_tuning(256, 16, 0, 0)) == "256x16/default"
    assert AT._from_entry({"items": 32}).block_threads == 256   # entries written before block sizes
