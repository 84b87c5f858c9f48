#!/usr/bin/env python3
"""Benchmark of the segmented for_each / transform_reduce / inclusive_scan
path on one MI355X.

One step is one pass of the whole hot path over the four full-size
workloads (seeded synthetic inputs, resident in HBM before timing):

  triad      2^28 binary32, 8 equal segments: for_each a = b + 3c, and the
             compensated dot(b, c)
  scan       2^30 int32 U{0..100} in 16 Dirichlet(1) segments -> int64, and
             -> int32 (wrapping); 2^28 binary32 N(0,1) in 16 Dirichlet(1)
             segments with binary64 carries, and with binary32 carries
  precision  2^29 values of the |N(0,1)| / lognormal(0,4) mixture, binary32
             and bfloat16: sum of squares and dot, compensated and plain
  batch      10,000 ragged binary32 ranges (2^28 in all): the fused per-range
             scan + dot replayed from a hipGraph; backward: the dot's
             adjoint (broadcast multiply) and the scan's (reverse scan)

`value` is the step's algorithmic HBM bytes (each input read once, each
output written once) divided by its time. `config.per_op` gives every
operation's time, GB/s, fraction of the 8 TB/s peak and (from the CPU leg)
its error against the binary64 oracle. `roofline` is for the longest-running
operation that is one kernel launch, timed with HIP events on its stream.
`cpu_baseline` times the oracle on the host: once serially (one thread) and
once on every core, beside plain binary32 loops; its outputs are the
references of the error figures.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
    python bench.py --configs     # every workload alone, median / p10 / p90
    python bench.py --copy-only   # the copy kernel that calibrates the counters
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2406_00158_amd.traffic import sources_hash  # noqa: E402 (no torch import)

METRIC = "effective HBM GB/s (% of peak) for fused reduce/scan; batched+compensated vs plain"
HBM_PEAK_GBS = 8000.0
U32 = 2.0 ** -24


def load_traffic(kernel: str):
    """Measured HBM bytes per launch for `kernel` from profiles/traffic.json,
    if it was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("sources") != sources_hash():
        return None   # counters taken on other kernel sources
    ent = rec.get("kernels", {}).get(kernel)
    return None if ent is None else ent.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_topology() -> dict:
    """What `lscpu` reports of the host (model, sockets, cores, threads,
    clock), with the CPUs this process may run on."""
    import subprocess
    info = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        want = ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core", "CPU(s)", "CPU max MHz",
                "L3 cache", "NUMA node(s)")
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in want:
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        info["usable_cpus"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        info["usable_cpus"] = os.cpu_count()
    return info


# ---------------------------------------------------------------------------
# The step
# ---------------------------------------------------------------------------

class Op:
    def __init__(self, name, nbytes, fn, kernel=None):
        self.name, self.nbytes, self.fn = name, nbytes, fn
        self.kernel = kernel   # the one kernel the call launches (besides a few-us prologue), or None


def setup(dev):
    """Inputs of the four workloads on the device, the tables, and the step's
    operations. Returns (ops, host, out): `host` keeps the seeded inputs for
    the oracle, `out` the device outputs the error figures compare."""
    import numpy as np
    import torch

    from paper_2406_00158_amd import autotune as AT
    from paper_2406_00158_amd import binding as B
    from paper_2406_00158_amd import inputs as I

    def to_dev(a):
        if a.dtype == np.uint16:
            return torch.from_numpy(a.view(np.int16)).to(dev).view(torch.bfloat16)
        return torch.from_numpy(a).to(dev)

    def pieces(t, lengths):
        out, o = [], 0
        for n in lengths:
            out.append(t[o:o + n])
            o += n
        return out

    host, out, ops = {}, {}, []
    f32, v_id = B.DR_F32, B.make_view("identity", B.DR_F32)
    tuning = out["tuning"] = {}

    def look_back_kernel(tu, fused):
        """The one kernel of a look-back scan call (binary32, binary64
        carries), by its template arguments <in, out, op, carry64, fused,
        reduce op, acc, items, reverse, block>; None for the other forms."""
        if tu is None or tu.flags != B.DR_TUNE_TILE_PER_BLOCK:
            return None
        if fused:
            return f"k_scan<1, 1, 0, true, true, 2, 1, {tu.items_per_thread}, false, {tu.block_threads}>"
        return f"k_scan<1, 1, 0, true, false, 0, 0, {tu.items_per_thread}, true, {tu.block_threads}>"

    def tuned(name, algo, view, odt, table, call, extra=""):
        """The autotuner's shape for `call` (timed now, outside the timed
        region), recorded with every candidate's time."""
        tu = AT.tune(algo, view, odt, table, call, extra=extra)
        e = AT.entry(algo, view, odt, table, extra) or {}
        tuning[name] = {"choice": AT.label(tu) if tu is not None else "default",
                        "candidates_ms": {k: round(v, 4) for k, v in (e.get("all") or {}).items()}}
        return tu

    # triad: 2^28 binary32, 8 equal segments
    t = I.triad()
    L2 = t["lengths"]
    host["triad"] = t
    b, c = to_dev(t["b"]), to_dev(t["c"])
    a = torch.empty_like(b)
    out["triad_a"] = a
    t_tr = B.segments([pieces(b, L2), pieces(c, L2)], [pieces(a, L2)])
    t_dot = B.segments([pieces(b, L2), pieces(c, L2)])
    ws2 = B.Workspace(dev)
    r_dot = torch.zeros(1, dtype=torch.float64, device=dev)
    out["triad_dot"] = r_dot
    n2 = sum(L2)
    v_axpy, v_mul = B.make_view("axpy", f32, t["s"]), B.make_view("mul", f32)
    ops.append(Op("triad: for_each a = b + 3c", 12 * n2,
                  lambda: B.dr_for_each(t_tr, v_axpy, f32, workspace=ws2, host_check=False), "k_for_each"))
    ops.append(Op("triad: dot(b, c) compensated", 8 * n2,
                  lambda: B.dr_transform_reduce(t_dot, v_mul, B.DR_ACC_COMPENSATED, 0.0, r_dot, workspace=ws2,
                                                host_check=False), "k_reduce_stream<1, 2, 1, 16>"))

    # scan: 2^30 int32 (16 Dirichlet segments) and 2^28 binary32 (its own 16)
    t = I.scan_int()
    L3 = t["lengths"]
    host["scan_int"] = t
    k = to_dev(t["k"])
    n3 = k.numel()
    k64 = torch.empty(n3, dtype=torch.int64, device=dev)
    k32 = torch.empty(n3, dtype=torch.int32, device=dev)
    out["scan_i64"], out["scan_i32"] = k64, k32
    t64 = B.segments([pieces(k, L3)], [pieces(k64, L3)])
    t32 = B.segments([pieces(k, L3)], [pieces(k32, L3)])
    ws3 = B.Workspace(dev)
    v_i = B.make_view("identity", B.DR_I32)
    # one range past 2^22 elements: the chained single pass (one kernel
    # after the counter prologue), k_scan_chain<in, out, carry64, reverse>
    ops.append(Op("scan: int32 2^30 -> int64", 12 * n3,
                  lambda: B.dr_inclusive_scan(t64, v_i, B.DR_I64, workspace=ws3, host_check=False),
                  "k_scan_chain<0, 4, true, false>"))
    ops.append(Op("scan: int32 2^30 -> int32 (wrap)", 8 * n3,
                  lambda: B.dr_inclusive_scan(t32, v_i, B.DR_I32, workspace=ws3, host_check=False),
                  "k_scan_chain<0, 0, true, false>"))
    t = I.scan_fp()
    L3f = t["lengths"]
    host["scan_fp"] = t
    xf = to_dev(t["x"])
    n3f = xf.numel()
    yf64, yf32 = torch.empty_like(xf), torch.empty_like(xf)
    out["scan_f_c64"], out["scan_f_c32"] = yf64, yf32
    tf64 = B.segments([pieces(xf, L3f)], [pieces(yf64, L3f)])
    tf32 = B.segments([pieces(xf, L3f)], [pieces(yf32, L3f)])
    ops.append(Op("scan: f32 2^28, binary64 carries", 8 * n3f,
                  lambda: B.dr_inclusive_scan(tf64, v_id, f32, 0, workspace=ws3, host_check=False),
                  "k_scan_chain<1, 1, true, false>"))
    ops.append(Op("scan: f32 2^28, binary32 carries", 8 * n3f,
                  lambda: B.dr_inclusive_scan(tf32, v_id, f32, B.DR_SCAN_CARRY_F32, workspace=ws3,
                                              host_check=False),
                  "k_scan_chain<1, 1, false, false>"))

    # precision: 2^29 mixture, binary32 and bfloat16, 8 equal segments
    t = I.precision()
    L4 = t["lengths"]
    host["precision"] = t
    n4 = sum(L4)
    ws4 = B.Workspace(dev)
    for dt, xs, ys, eb in (("f32", t["x"], t["y"], 4), ("bf16", t["x_bf16"], t["y_bf16"], 2)):
        xd, yd = to_dev(xs), to_dev(ys)
        bdt = B.DR_F32 if dt == "f32" else B.DR_BF16
        items = 16 if dt == "f32" else 32
        t1, tz = B.segments([pieces(xd, L4)]), B.segments([pieces(xd, L4), pieces(yd, L4)])
        for acc in ("compensated", "plain"):
            r1 = torch.zeros(1, dtype=torch.float64, device=dev)
            r2 = torch.zeros(1, dtype=torch.float64, device=dev)
            out[f"prec_{dt}_sumsq_{acc}"], out[f"prec_{dt}_dot_{acc}"] = r1, r2
            ac = B.ACCS[acc]
            kn = lambda arity: f"k_reduce_stream<{bdt}, {arity}, {ac}, {items}>"
            ops.append(Op(f"precision: {dt} sum of squares, {acc}", eb * n4,
                          (lambda t1=t1, v=B.make_view("square", bdt), ac=ac, r1=r1:
                           B.dr_transform_reduce(t1, v, ac, 0.0, r1, workspace=ws4, host_check=False)),
                          kn(1).replace(", 1, ", ", 1, ", 1)))
            ops.append(Op(f"precision: {dt} dot, {acc}", 2 * eb * n4,
                          (lambda tz=tz, v=B.make_view("mul", bdt), ac=ac, r2=r2:
                           B.dr_transform_reduce(tz, v, ac, 0.0, r2, workspace=ws4, host_check=False)),
                          kn(2)))
    # the reduce kernels' template arguments: <in dtype, op, acc, items>
    for o in ops:
        if o.kernel and o.kernel.startswith("k_reduce_stream<") and "sum of squares" in o.name:
            parts = o.kernel[len("k_reduce_stream<"):-1].split(", ")
            o.kernel = f"k_reduce_stream<{parts[0]}, {B.DR_OP_SQUARE}, {parts[2]}, {parts[3]}>"
        elif o.kernel and o.kernel.startswith("k_reduce_stream<") and "dot" in o.name and "precision" in o.name:
            parts = o.kernel[len("k_reduce_stream<"):-1].split(", ")
            o.kernel = f"k_reduce_stream<{parts[0]}, {B.DR_OP_MUL}, {parts[2]}, {parts[3]}>"

    # batch: 10,000 ragged ranges, fused scan + dot from a graph, backward
    t = I.batch()
    L5 = t["lengths"]
    host["batch"] = t
    n5 = sum(L5)
    x5, y5 = to_dev(t["x"]), to_dev(t["y"])
    s5 = torch.empty_like(x5)
    r5 = torch.zeros(len(L5), dtype=torch.float64, device=dev)
    out["batch_s"], out["batch_r"] = s5, r5
    out["batch_x"], out["batch_y"] = x5, y5
    ws5, ws5b, ws5r = B.Workspace(dev), B.Workspace(dev), B.Workspace(dev)
    t5 = B.segments([pieces(x5, L5), pieces(y5, L5)], [pieces(s5, L5)], mode="batch")
    # the launch shape (workgroup size x items per thread x scan form) of the
    # batch's two scans comes from the autotuner, timed here, before capture
    tu5 = tuned("batch: fused scan + dot per range (hipGraph replay)", B.DR_ALGO_SCAN_REDUCE, v_id, f32, t5,
                lambda tu: B.dr_scan_reduce(t5, v_id, v_mul, B.DR_ACC_COMPENSATED, 0.0, r5, workspace=ws5,
                                            host_check=False, tuning=tu))
    fused = lambda: B.dr_scan_reduce(t5, v_id, v_mul, B.DR_ACC_COMPENSATED, 0.0, r5, workspace=ws5,
                                     host_check=False, tuning=tu5)
    out["batch_tuning"] = tu5
    fused()                                 # eager: plans and sizes the workspace
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        fused()
    torch.cuda.current_stream(dev).wait_stream(side)
    with torch.cuda.graph(graph):
        fused()
    ops.append(Op("batch: fused scan + dot per range (hipGraph replay)", 12 * n5, graph.replay,
                  look_back_kernel(tu5, True)))
    g5_np = I.normal_f32(len(L5), 1105).astype(np.float64)
    up5_np = I.normal_f32(n5, 1106)
    host["batch_g"], host["batch_up"] = g5_np, up5_np
    g5, up5 = torch.from_numpy(g5_np).to(dev), to_dev(up5_np)
    gx5, gy5, gs5 = torch.empty_like(x5), torch.empty_like(y5), torch.empty_like(x5)
    out["batch_gx"], out["batch_gy"], out["batch_gs"] = gx5, gy5, gs5
    tbm = B.segments([pieces(x5, L5), pieces(y5, L5)], [pieces(gx5, L5), pieces(gy5, L5)], mode="batch")
    trs = B.segments([pieces(up5, L5)], [pieces(gs5, L5)], mode="batch")
    ops.append(Op("batch: backward, dot adjoint (broadcast multiply)", 16 * n5,
                  lambda: B.dr_broadcast_mul(tbm, v_mul, g5, 2, workspace=ws5b, host_check=False),
                  "k_broadcast_mul<1, 2, 16, 2>"))
    tu5r = tuned("batch: backward, scan adjoint (reverse scan)", B.DR_ALGO_SCAN, v_id, f32, trs,
                 lambda tu: B.dr_inclusive_scan(trs, v_id, f32, B.DR_SCAN_REVERSE, workspace=ws5r,
                                                host_check=False, tuning=tu), extra="reverse")
    ops.append(Op("batch: backward, scan adjoint (reverse scan)", 8 * n5,
                  lambda: B.dr_inclusive_scan(trs, v_id, f32, B.DR_SCAN_REVERSE, workspace=ws5r,
                                              host_check=False, tuning=tu5r),
                  look_back_kernel(tu5r, False)))
    out["workspaces"] = [ws2, ws3, ws4, ws5, ws5b, ws5r]
    out["graph"] = graph
    return ops, host, out


def per_range_leg(host, out, dev, sample: int = 64) -> dict:
    """The batch workload's fused scan + dot run again, outside the timed
    region, on one-row tables for `sample` seeded ranges (with the batched
    call's launch shape): the per-range results that the accuracy record
    compares with the batched ones."""
    import numpy as np
    import torch

    from paper_2406_00158_amd import binding as B

    L = host["batch"]["lengths"]
    offs = np.concatenate([[0], np.cumsum(L)]).astype(np.int64)
    idx = sorted(int(i) for i in np.random.default_rng(1107).choice(len(L), size=sample, replace=False))
    x5, y5 = out["batch_x"], out["batch_y"]
    vid, vmul = B.make_view("identity", B.DR_F32), B.make_view("mul", B.DR_F32)
    ws = B.Workspace(dev)
    s_list, r_list = [], []
    for i in idx:
        lo, hi = int(offs[i]), int(offs[i + 1])
        s = torch.empty(hi - lo, dtype=torch.float32, device=dev)
        r = torch.zeros(1, dtype=torch.float64, device=dev)
        B.dr_scan_reduce(B.segments([[x5[lo:hi]], [y5[lo:hi]]], [[s]]), vid, vmul, B.DR_ACC_COMPENSATED, 0.0, r,
                         workspace=ws, host_check=False, tuning=out.get("batch_tuning"))
        s_list.append(s)
        r_list.append(r)
    torch.cuda.synchronize()
    return {"idx": idx, "offs": offs, "s": [t.cpu().numpy() for t in s_list], "r": [t.item() for t in r_list],
            "status": ws.device_status()}


# ---------------------------------------------------------------------------
# CPU leg: the oracle (references of the error figures), its twin on every
# core, and plain binary32 loops
# ---------------------------------------------------------------------------

def cpu_leg(host, out, per_range=None) -> tuple[dict, dict]:
    """Returns (errors by op name, cpu_baseline). With `per_range` (from
    per_range_leg) the batch entry also compares the per-range results with
    the batched ones."""
    import numpy as np

    import oracle as O
    import oracle.parallel as OP
    import oracle.plain as PL
    from paper_2406_00158_amd import inputs as I

    def d2h(t, lo=None, hi=None):
        v = t if lo is None else t[lo:hi]
        return v.cpu().numpy()

    err, work = {}, 0
    t_serial = 0.0

    def timed(fn):
        nonlocal t_serial
        t0 = time.perf_counter()
        r = fn()
        t_serial += time.perf_counter() - t0
        return r

    def scan_metrics(got, ref, absp):
        e = np.abs(got.astype(np.float64) - ref)
        return {"max_abs_err": float(e.max()), "max_err_over_abs_prefix": float(np.max(e / np.maximum(absp, 1e-300))),
                "frac_equal_fl32_ref": float(np.mean(got == ref.astype(np.float32)))}

    def rel(gotv, want, mag):
        return {"rel_err": abs(gotv - want) / abs(want), "cond": mag / abs(want)}

    # triad
    t = host["triad"]
    L = t["lengths"]
    b, c = I.split(t["b"], L), I.split(t["c"], L)
    want = np.concatenate(timed(lambda: O.for_each(b, c, O.F32, O.AXPY, O.F32, alpha=t["s"])))
    got = d2h(out["triad_a"])
    err["triad: for_each a = b + 3c"] = {"bit_exact": bool(np.array_equal(got.view(np.uint32), want.view(np.uint32))),
                                         "mismatches": int(np.sum(got.view(np.uint32) != want.view(np.uint32)))}
    w, m = timed(lambda: O.reduce(b, c, O.F32, O.MUL))
    err["triad: dot(b, c) compensated"] = rel(out["triad_dot"].item(), w[0], m[0])
    work += 20 * sum(L)
    del want, got

    # scans
    t = host["scan_int"]
    L = t["lengths"]
    k = I.split(t["k"], L)
    for odt, key, name in ((O.I64, "scan_i64", "scan: int32 2^30 -> int64"),
                           (O.I32, "scan_i32", "scan: int32 2^30 -> int32 (wrap)")):
        want = np.concatenate(timed(lambda: O.scan(k, None, O.I32, O.IDENTITY, out_dtype=odt)))
        mism, step = 0, 1 << 26
        for lo in range(0, want.shape[0], step):
            hi = min(lo + step, want.shape[0])
            mism += int(np.sum(d2h(out[key], lo, hi) != want[lo:hi]))
        err[name] = {"bit_exact": mism == 0, "mismatches": mism}
        work += (12 if odt == O.I64 else 8) * want.shape[0]
        del want
    t = host["scan_fp"]
    L = t["lengths"]
    ref, absp = timed(lambda: O.scan(I.split(t["x"], L), None, O.F32, O.IDENTITY, want_abs=True))
    ref, absp = np.concatenate(ref), np.concatenate(absp)
    err["scan: f32 2^28, binary64 carries"] = scan_metrics(d2h(out["scan_f_c64"]), ref, absp)
    err["scan: f32 2^28, binary32 carries"] = scan_metrics(d2h(out["scan_f_c32"]), ref, absp)
    work += 8 * ref.shape[0]
    del ref, absp

    # precision
    t = host["precision"]
    L = t["lengths"]
    for dt, xs, ys, odt in (("f32", t["x"], t["y"], O.F32), ("bf16", t["x_bf16"], t["y_bf16"], O.BF16)):
        xl, yl = I.split(xs, L), I.split(ys, L)
        wsq, msq = timed(lambda: O.reduce(xl, None, odt, O.SQUARE))
        wd, md = timed(lambda: O.reduce(xl, yl, odt, O.MUL))
        for acc in ("compensated", "plain"):
            err[f"precision: {dt} sum of squares, {acc}"] = rel(out[f"prec_{dt}_sumsq_{acc}"].item(), wsq[0], msq[0])
            err[f"precision: {dt} dot, {acc}"] = rel(out[f"prec_{dt}_dot_{acc}"].item(), wd[0], md[0])
        work += 3 * xs.nbytes

    # batch
    t = host["batch"]
    L = t["lengths"]
    xl, yl = I.split(t["x"], L), I.split(t["y"], L)
    ref, absp = timed(lambda: O.scan(xl, None, O.F32, O.IDENTITY, mode=O.BATCH, want_abs=True))
    ref, absp = np.concatenate(ref), np.concatenate(absp)
    got_s = d2h(out["batch_s"])
    e_scan = scan_metrics(got_s, ref, absp)
    w, m = timed(lambda: O.reduce(xl, yl, O.F32, O.MUL, mode=O.BATCH))
    got = d2h(out["batch_r"])
    r_err = np.abs(got - w) / np.maximum(np.abs(w), 1e-300)
    e_scan.update({"dot_max_rel_err": float(r_err.max()), "dot_median_rel_err": float(np.median(r_err)),
                   "dot_max_cond": float(np.max(m / np.maximum(np.abs(w), 1e-300)))})
    if per_range is not None:
        # the sampled ranges alone (one-row tables) beside the batched call
        offs, eq, n_el, d_pref, e_one, e_bat, d_dot, re_one, re_bat = per_range["offs"], 0, 0, 0.0, 0.0, 0.0, \
            0.0, 0.0, 0.0
        for j, i in enumerate(per_range["idx"]):
            lo, hi = int(offs[i]), int(offs[i + 1])
            one, bat, a_i = per_range["s"][j], got_s[lo:hi], np.maximum(absp[lo:hi], 1e-300)
            eq += int(np.sum(one.view(np.uint32) == bat.view(np.uint32)))
            n_el += hi - lo
            d_pref = max(d_pref, float(np.max(np.abs(one.astype(np.float64) - bat) / a_i)))
            e_one = max(e_one, float(np.max(np.abs(one.astype(np.float64) - ref[lo:hi]) / a_i)))
            e_bat = max(e_bat, float(np.max(np.abs(bat.astype(np.float64) - ref[lo:hi]) / a_i)))
            r1, rb = per_range["r"][j], float(got[i])
            d_dot = max(d_dot, abs(r1 - rb) / max(abs(rb), 1e-300))
            re_one = max(re_one, abs(r1 - w[i]) / max(abs(w[i]), 1e-300))
            re_bat = max(re_bat, abs(rb - w[i]) / max(abs(w[i]), 1e-300))
        e_scan["per_range_vs_batched"] = {
            "ranges": len(per_range["idx"]), "elements": n_el, "scan_frac_bitwise_equal": eq / max(n_el, 1),
            "scan_max_diff_over_abs_prefix": d_pref, "scan_max_err_over_abs_prefix_per_range": e_one,
            "scan_max_err_over_abs_prefix_batched": e_bat, "dot_max_rel_diff": d_dot,
            "dot_max_rel_err_per_range": re_one, "dot_max_rel_err_batched": re_bat,
            "device_status": per_range["status"]}
    del ref, absp, got_s
    err["batch: fused scan + dot per range (hipGraph replay)"] = e_scan
    g = host["batch_g"]
    mism = 0
    for which, key in ((0, "batch_gx"), (1, "batch_gy")):
        wg = np.concatenate(timed(lambda: O.reduce_grad(xl, yl, O.F32, O.MUL, g, which, mode=O.BATCH)))
        mism += int(np.sum(d2h(out[key]).view(np.uint32) != wg.astype(np.float32).view(np.uint32)))
        del wg
    err["batch: backward, dot adjoint (broadcast multiply)"] = {"bit_exact": mism == 0, "mismatches": mism}
    up = host["batch_up"]
    ref, absp = timed(lambda: O.scan(I.split(up, L), None, O.F32, O.IDENTITY, mode=O.BATCH, reverse=True,
                                     want_abs=True))
    ref, absp = np.concatenate(ref), np.concatenate(absp)
    err["batch: backward, scan adjoint (reverse scan)"] = scan_metrics(d2h(out["batch_gs"]), ref, absp)
    del ref, absp
    work += 36 * sum(L)

    # the oracle on every core (the same operations), and plain loops
    nthreads = OP.threads()
    t0 = time.perf_counter()
    t = host["triad"]
    OP.for_each(t["b"], t["c"], O.F32, O.AXPY, O.F32, alpha=t["s"])
    OP.reduce(t["b"], t["c"], O.F32, O.MUL)
    OP.scan(host["scan_int"]["k"], O.I32, O.I64)
    OP.scan(host["scan_int"]["k"], O.I32, O.I32)
    OP.scan(host["scan_fp"]["x"], O.F32)
    t = host["precision"]
    for xs, ys, odt in ((t["x"], t["y"], O.F32), (t["x_bf16"], t["y_bf16"], O.BF16)):
        OP.reduce(xs, None, odt, O.SQUARE)
        OP.reduce(xs, ys, odt, O.MUL)
    t = host["batch"]
    L = t["lengths"]
    OP.scan_batch(t["x"], L)
    OP.reduce_batch(t["x"], t["y"], L)
    OP.reduce_grad_batch(t["x"], t["y"], L, host["batch_g"], 0)
    OP.reduce_grad_batch(t["x"], t["y"], L, host["batch_g"], 1)
    OP.scan_batch(host["batch_up"], L, reverse=True)
    t_par = time.perf_counter() - t0

    Pl = PL.lib()
    p = PL.ptr
    t0 = time.perf_counter()
    t = host["triad"]
    a = np.empty_like(t["b"])
    Pl.plain_triad(a.shape[0], p(t["b"]), p(t["c"]), p(a), t["s"])
    Pl.plain_dot_f32(a.shape[0], p(t["b"]), p(t["c"]))
    del a
    k = host["scan_int"]["k"]
    y64 = np.empty(k.shape[0], dtype=np.int64)
    Pl.plain_scan_i32_i64(k.shape[0], p(k), p(y64))
    del y64
    y32 = np.empty_like(k)
    Pl.plain_scan_i32_i32(k.shape[0], p(k), p(y32))
    del y32
    x = host["scan_fp"]["x"]
    yf = np.empty_like(x)
    Pl.plain_scan_f32(x.shape[0], p(x), p(yf))
    del yf
    t = host["precision"]
    n4 = t["x"].shape[0]
    Pl.plain_sumsq_f32(n4, p(t["x"]))
    Pl.plain_dot_f32(n4, p(t["x"]), p(t["y"]))
    Pl.plain_sumsq_bf16(n4, p(t["x_bf16"]))
    Pl.plain_dot_bf16(n4, p(t["x_bf16"]), p(t["y_bf16"]))
    t = host["batch"]
    lens = np.asarray(t["lengths"], dtype=np.int64)
    s5, r5 = np.empty_like(t["x"]), np.empty(lens.shape[0])
    Pl.plain_scan_f32_batch(lens.shape[0], p(lens), p(t["x"]), p(s5), 0)
    Pl.plain_dot_f32_batch(lens.shape[0], p(lens), p(t["x"]), p(t["y"]), p(r5))
    gx, gy = np.empty_like(t["x"]), np.empty_like(t["x"])
    Pl.plain_bcast_mul_batch(lens.shape[0], p(lens), p(t["x"]), p(t["y"]), p(host["batch_g"]), p(gx), p(gy))
    Pl.plain_scan_f32_batch(lens.shape[0], p(lens), p(host["batch_up"]), p(s5), 1)
    t_plain = time.perf_counter() - t0
    del s5, gx, gy

    gbs = lambda s: round(work / s / 1e9, 3)
    base = {"value": gbs(t_par), "unit": "GB/s", "cores": nthreads, "kind": "oracle",
            "sample": f"the whole step once (every operation of the four workloads at full size: {work / 1e9:.1f} GB "
                      f"of algorithmic bytes, with the C4 plain/compensated pairs sharing one reference each), "
                      f"the binary64 / int64 oracle (gcc -O2) on all {nthreads} host threads: {t_par:.2f} s",
            "cpu_model": cpu_model(), "lscpu": cpu_topology(),
            "serial": {"value": gbs(t_serial), "cores": 1, "seconds": round(t_serial, 2),
                       "what": "the same oracle calls on one thread (they produced the error references)"},
            "plain_f32_loop": {"value": gbs(t_plain), "cores": 1, "seconds": round(t_plain, 2),
                               "what": "plain serial binary32 / int64 loops over the same operations (no "
                                       "binary64, no compensation): the cost of the arithmetic alone"}}
    return err, base


def write_accuracy(path: str, line: dict, device_name: str) -> None:
    """The accuracy record of one bench run: every result of the step
    against the binary64 / int64 oracle, as a markdown file."""
    per_op = line["config"]["per_op"]
    u32 = 2.0 ** -24
    fmt = lambda v: f"{v:.2e}" if isinstance(v, float) else str(v)
    rows = ["# Accuracy of the bench step against the binary64 oracle", "",
            f"`python bench.py {' '.join(sys.argv[1:])}` on {device_name}; kernel sources `{sources_hash()}`.",
            "Every result of one step, compared on the host with the oracle's binary64 (integers: int64) result",
            "on the same seeded inputs. Condition number of a sum: sum of |terms| / |sum|. A_i: the exact sum of",
            "|x_j| over the prefix of element i (the scale of a prefix's rounding error).", "",
            "## Exact results", "", "| operation | bit-exact | mismatching elements |", "|---|---|---|"]
    for name, o in per_op.items():
        e = o.get("error_vs_fp64_oracle", {})
        if "bit_exact" in e:
            rows.append(f"| {name} | {e['bit_exact']} | {e['mismatches']} |")
    rows += ["", "## Reductions: plain vs compensated accumulation", "",
             "| operation | relative error | condition number | u32 x condition |", "|---|---|---|---|"]
    for name, o in per_op.items():
        e = o.get("error_vs_fp64_oracle", {})
        if "rel_err" in e:
            rows.append(f"| {name} | {fmt(e['rel_err'])} | {fmt(e['cond'])} | {fmt(u32 * e['cond'])} |")
    rows += ["", "## Scans: binary64 vs binary32 carries, batched", "",
             "| operation | max abs error | max error / A_i | elements equal to the rounded exact prefix |",
             "|---|---|---|---|"]
    for name, o in per_op.items():
        e = o.get("error_vs_fp64_oracle", {})
        if "max_err_over_abs_prefix" in e:
            rows.append(f"| {name} | {fmt(e['max_abs_err'])} | {fmt(e['max_err_over_abs_prefix'])} | "
                        f"{e['frac_equal_fl32_ref']:.3f} |")
    for name, o in per_op.items():
        e = o.get("error_vs_fp64_oracle", {})
        if "dot_max_rel_err" in e:
            rows += ["", f"Per-range dots of `{name}`: max relative error {fmt(e['dot_max_rel_err'])}, median "
                         f"{fmt(e['dot_median_rel_err'])}, largest condition number {fmt(e['dot_max_cond'])}."]
        pr = e.get("per_range_vs_batched")
        if pr:
            rows += ["", "## Batched vs per-range", "",
                     f"{pr['ranges']} seeded ranges ({pr['elements']} elements) of the batch workload, each run "
                     "alone as a one-row table, beside the same ranges of the batched call:", "",
                     "| quantity | per-range calls | batched call |", "|---|---|---|",
                     f"| scan: max error / A_i | {fmt(pr['scan_max_err_over_abs_prefix_per_range'])} | "
                     f"{fmt(pr['scan_max_err_over_abs_prefix_batched'])} |",
                     f"| dot: max relative error | {fmt(pr['dot_max_rel_err_per_range'])} | "
                     f"{fmt(pr['dot_max_rel_err_batched'])} |", "",
                     f"Scan outputs bitwise equal between the two: {pr['scan_frac_bitwise_equal']:.6f} of the "
                     f"elements (largest difference {fmt(pr['scan_max_diff_over_abs_prefix'])} A_i); dots: largest "
                     f"relative difference {fmt(pr['dot_max_rel_diff'])}."]
    with open(path, "w") as f:
        f.write("\n".join(rows) + "\n")


# ---------------------------------------------------------------------------

def configs_report(reps: int) -> int:
    """Every workload of the hot path at its full size, timed alone: the
    median, 10th and 90th percentile of `reps` launches (HIP events on the
    launch stream), as GB/s at algorithmic bytes, fraction of the 8 TB/s
    peak and of a plain copy measured here. One JSON line per case."""
    import numpy as np
    import torch

    from paper_2406_00158_amd import binding as B
    from paper_2406_00158_amd import inputs as I

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)

    def to_dev(a):
        if a.dtype == np.uint16:
            return torch.from_numpy(a.view(np.int16)).to(dev).view(torch.bfloat16)
        return torch.from_numpy(a).to(dev)

    def pieces(t, lengths):
        out, o = [], 0
        for n in lengths:
            out.append(t[o:o + n])
            o += n
        return out

    def timed(fn, n_reps, warm=3):
        for _ in range(warm):
            fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_reps)]
        for e0, e1 in ev:
            e0.record(stream)
            fn()
            e1.record(stream)
        torch.cuda.synchronize()
        ms = sorted(e0.elapsed_time(e1) for e0, e1 in ev)
        pick = lambda q: ms[min(len(ms) - 1, int(q * (len(ms) - 1) + 0.5))]
        return pick(0.5), pick(0.1), pick(0.9)

    copy_gbs = [None]
    ws = B.Workspace(dev)

    def report(cfg, case, nbytes, fn, n_reps=reps, latency=False, note=None):
        med, p10, p90 = timed(fn, n_reps)
        gbs = nbytes / (med * 1e-3) / 1e9
        line = {"config": cfg, "case": case, "median_us": round(med * 1e3, 1), "p10_us": round(p10 * 1e3, 1),
                "p90_us": round(p90 * 1e3, 1), "algorithmic_bytes": nbytes, "GB/s": round(gbs, 1),
                "frac_of_peak": None if latency else round(gbs / HBM_PEAK_GBS, 4),
                "frac_of_copy": None if (latency or copy_gbs[0] is None) else round(gbs / copy_gbs[0], 4),
                "reps": n_reps}
        if note:
            line["note"] = note
        print(json.dumps(line), flush=True)
        return gbs

    # copy reference: for_each identity, 2^28 binary32 (1 GiB each way)
    N = 1 << 28
    src = torch.rand(N, device=dev)
    dst = torch.empty_like(src)
    tcp = B.segments([[src]], [[dst]])
    copy_gbs[0] = report("copy", "for_each identity 2^28 f32", 8 * N,
                         lambda: B.dr_for_each(tcp, B.make_view("identity", B.DR_F32), B.DR_F32, workspace=ws,
                                               host_check=False))
    # two reads and two writes through the library (the broadcast multiply's
    # access pattern, with the identity view: gx = g * 1... written as a zip
    # of two inputs and two outputs): the ceiling of a 2-in-2-out stream
    src2 = torch.rand(N, device=dev)
    dst2 = torch.empty_like(src)
    t22 = B.segments([[src], [src2]], [[dst], [dst2]])
    g1 = torch.ones(1, dtype=torch.float64, device=dev)
    report("copy", "2 reads + 2 writes: broadcast multiply (mul view, g = 1) 2^28 f32", 16 * N,
           lambda: B.dr_broadcast_mul(t22, B.make_view("mul", B.DR_F32), g1, 2, workspace=ws, host_check=False))
    del src, dst, tcp, src2, dst2, t22

    # tiny: 2^20, 4 unequal segments, separate allocations and one carved buffer
    t = I.tiny()
    L = t["lengths"]
    n = sum(L)
    for layout in ("separate", "carved"):
        if layout == "separate":
            x = [to_dev(p.copy()) for p in I.split(t["x"], L)]
            y = [to_dev(p.copy()) for p in I.split(t["y"], L)]
            k = [to_dev(p.copy()) for p in I.split(t["k"], L)]
        else:
            x, y, k = (pieces(to_dev(t[nm]), L) for nm in ("x", "y", "k"))
        res = torch.zeros(1, dtype=torch.float64, device=dev)
        resi = torch.zeros(1, dtype=torch.int64, device=dev)
        ko = [torch.empty(p.numel(), dtype=torch.int32, device=dev) for p in k]
        tdot, tk, tks = B.segments([x, y]), B.segments([k]), B.segments([k], [ko])
        report("C1 tiny " + layout, "dot compensated", 8 * n, lambda: B.dr_transform_reduce(
            tdot, B.make_view("mul", B.DR_F32), B.DR_ACC_COMPENSATED, 0.0, res, workspace=ws, host_check=False),
            latency=True)
        report("C1 tiny " + layout, "int32 scan -> int32", 8 * n, lambda: B.dr_inclusive_scan(
            tks, B.make_view("identity", B.DR_I32), B.DR_I32, workspace=ws, host_check=False), latency=True)
        report("C1 tiny " + layout, "int sum", 4 * n, lambda: B.dr_transform_reduce(
            tk, B.make_view("identity", B.DR_I32), 0, 0, resi, workspace=ws, host_check=False), latency=True)
    del t

    # C2 triad + dot: 2^28, 8 equal segments
    t = I.triad()
    L = t["lengths"]
    b, c = to_dev(t["b"]), to_dev(t["c"])
    a = torch.empty_like(b)
    s = t["s"]
    del t
    res = torch.zeros(1, dtype=torch.float64, device=dev)
    ttr, tdot = B.segments([pieces(b, L), pieces(c, L)], [pieces(a, L)]), B.segments([pieces(b, L), pieces(c, L)])
    report("C2 triad", "for_each a = b + 3c", 12 * N, lambda: B.dr_for_each(
        ttr, B.make_view("axpy", B.DR_F32, s), B.DR_F32, workspace=ws, host_check=False))
    for acc in ("compensated", "plain"):
        report("C2 triad", f"dot {acc}", 8 * N, lambda: B.dr_transform_reduce(
            tdot, B.make_view("mul", B.DR_F32), B.ACCS[acc], 0.0, res, workspace=ws, host_check=False))
    del a, b, c, ttr, tdot

    # C3 scans: int32 2^30 (16 Dirichlet segments) and binary32 2^28 (its own 16)
    t = I.scan_int()
    L = t["lengths"]
    k = to_dev(t["k"])
    del t
    nk = k.numel()
    for odt, ob in ((B.DR_I64, 8), (B.DR_I32, 4)):
        out = torch.empty(nk, dtype=B.TORCH_DTYPE[odt], device=dev)
        tab = B.segments([pieces(k, L)], [pieces(out, L)])
        report("C3 scan", f"int32 2^30 -> {'int64' if odt == B.DR_I64 else 'int32 (wrap)'}", (4 + ob) * nk,
               lambda: B.dr_inclusive_scan(tab, B.make_view("identity", B.DR_I32), odt, workspace=ws,
                                           host_check=False), n_reps=max(5, reps // 4))
        del out, tab
    del k
    t = I.scan_fp()
    L = t["lengths"]
    x = to_dev(t["x"])
    del t
    out = torch.empty_like(x)
    tab = B.segments([pieces(x, L)], [pieces(out, L)])
    for fl, nm in ((0, "binary64 carries"), (B.DR_SCAN_CARRY_F32, "binary32 carries")):
        report("C3 scan", f"f32 2^28, {nm}", 8 * x.numel(), lambda: B.dr_inclusive_scan(
            tab, B.make_view("identity", B.DR_F32), B.DR_F32, fl, workspace=ws, host_check=False))
    vid = B.make_view("identity", B.DR_F32)
    report("C3 scan", "f32 2^28, exclusive sum with init", 8 * x.numel(), lambda: B.dr_scan(
        tab, vid, B.DR_F32, B.DR_COMBINE_SUM, B.DR_SCAN_EXCLUSIVE, 1.5, workspace=ws, host_check=False))
    report("C3 scan", "f32 2^28, inclusive max", 8 * x.numel(), lambda: B.dr_scan(
        tab, vid, B.DR_F32, B.DR_COMBINE_MAX, 0, None, workspace=ws, host_check=False))
    tx = B.segments([pieces(x, L)])
    rm = torch.zeros(1, dtype=torch.float64, device=dev)
    for cm, nm in ((B.DR_COMBINE_MAX, "max"), (B.DR_COMBINE_MIN, "min")):
        report("C3 scan", f"f32 2^28, reduce {nm}", 4 * x.numel(), lambda: B.dr_reduce(
            tx, vid, cm, 0, None, rm, workspace=ws, host_check=False))
    del x, out, tab, tx

    # C4 precision: 2^29 mixture, binary32 and bfloat16, plain vs compensated
    t = I.precision()
    L = t["lengths"]
    n4 = sum(L)
    for dt, (xs, ys), eb in (("f32", (t["x"], t["y"]), 4), ("bf16", (t["x_bf16"], t["y_bf16"]), 2)):
        xd, yd = to_dev(xs), to_dev(ys)
        bdt = B.DR_F32 if dt == "f32" else B.DR_BF16
        t1, t2 = B.segments([pieces(xd, L)]), B.segments([pieces(xd, L), pieces(yd, L)])
        for acc in ("compensated", "plain"):
            report("C4 precision", f"{dt} sum of squares {acc}", eb * n4, lambda: B.dr_transform_reduce(
                t1, B.make_view("square", bdt), B.ACCS[acc], 0.0, res, workspace=ws, host_check=False))
            report("C4 precision", f"{dt} dot {acc}", 2 * eb * n4, lambda: B.dr_transform_reduce(
                t2, B.make_view("mul", bdt), B.ACCS[acc], 0.0, res, workspace=ws, host_check=False))
        del xd, yd, t1, t2
    del t

    # C5 batch: 10,000 ragged ranges (2^28 total), fused scan + dot, backward
    t = I.batch()
    L = t["lengths"]
    x, y = to_dev(t["x"]), to_dev(t["y"])
    del t
    n5 = x.numel()
    s5 = torch.empty_like(x)
    r5 = torch.zeros(len(L), dtype=torch.float64, device=dev)
    ws5 = B.Workspace(dev)
    tab = B.segments([pieces(x, L), pieces(y, L)], [pieces(s5, L)], mode="batch")
    tsc = B.segments([pieces(x, L)], [pieces(s5, L)], mode="batch")
    tdt = B.segments([pieces(x, L), pieces(y, L)], mode="batch")
    vid, vmul = B.make_view("identity", B.DR_F32), B.make_view("mul", B.DR_F32)
    fused = lambda: B.dr_scan_reduce(tab, vid, vmul, B.DR_ACC_COMPENSATED, 0.0, r5, workspace=ws5,
                                     host_check=False)
    report("C5 batch", "fused scan + dot, eager", 12 * n5, fused)
    fused()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fused()
    torch.cuda.current_stream().wait_stream(side)
    with torch.cuda.graph(g):
        fused()
    report("C5 batch", "fused scan + dot, hipGraph replay", 12 * n5, g.replay)
    # the autotuner's shape (as in the bench step), eager and from a graph
    from paper_2406_00158_amd import autotune as AT
    tu = AT.tune(B.DR_ALGO_SCAN_REDUCE, vid, B.DR_F32, tab, lambda t_: B.dr_scan_reduce(
        tab, vid, vmul, B.DR_ACC_COMPENSATED, 0.0, r5, workspace=ws5, host_check=False, tuning=t_))
    fused_t = lambda: B.dr_scan_reduce(tab, vid, vmul, B.DR_ACC_COMPENSATED, 0.0, r5, workspace=ws5,
                                       host_check=False, tuning=tu)
    report("C5 batch", f"fused scan + dot, autotuned {AT.label(tu)}, eager", 12 * n5, fused_t)
    fused_t()
    torch.cuda.synchronize()
    gt = torch.cuda.CUDAGraph()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fused_t()
    torch.cuda.current_stream().wait_stream(side)
    with torch.cuda.graph(gt):
        fused_t()
    report("C5 batch", f"fused scan + dot, autotuned {AT.label(tu)}, hipGraph replay", 12 * n5, gt.replay)
    ws_s, ws_d, ws_b, ws_r = (B.Workspace(dev) for _ in range(4))
    report("C5 batch", "unfused: scan, then dot (two calls)", 16 * n5, lambda: (
        B.dr_inclusive_scan(tsc, vid, B.DR_F32, workspace=ws_s, host_check=False),
        B.dr_transform_reduce(tdt, vmul, B.DR_ACC_COMPENSATED, 0.0, r5, workspace=ws_d, host_check=False)))
    gx, gy = torch.empty_like(x), torch.empty_like(y)
    gg = torch.ones(len(L), dtype=torch.float64, device=dev)
    tbm = B.segments([pieces(x, L), pieces(y, L)], [pieces(gx, L), pieces(gy, L)], mode="batch")
    trs = B.segments([pieces(s5, L)], [pieces(gx, L)], mode="batch")
    report("C5 batch", "backward: dot adjoint (broadcast multiply)", 16 * n5, lambda: B.dr_broadcast_mul(
        tbm, vmul, gg, 2, workspace=ws_b, host_check=False))
    report("C5 batch", "backward: scan adjoint (reverse scan)", 8 * n5, lambda: B.dr_inclusive_scan(
        trs, vid, B.DR_F32, B.DR_SCAN_REVERSE, workspace=ws_r, host_check=False))
    tr = AT.tune(B.DR_ALGO_SCAN, vid, B.DR_F32, trs, lambda t_: B.dr_inclusive_scan(
        trs, vid, B.DR_F32, B.DR_SCAN_REVERSE, workspace=ws_r, host_check=False, tuning=t_), extra="reverse")
    report("C5 batch", f"backward: scan adjoint (reverse scan), autotuned {AT.label(tr)}", 8 * n5,
           lambda: B.dr_inclusive_scan(trs, vid, B.DR_F32, B.DR_SCAN_REVERSE, workspace=ws_r, host_check=False,
                                       tuning=tr))
    per = [(B.segments([[xs], [ys]], [[ss]]), r5[i:i + 1]) for i, (xs, ys, ss) in
           enumerate(zip(pieces(x, L), pieces(y, L), pieces(s5, L)))]
    ws1 = B.Workspace(dev)
    ws1.for_call(B.DR_ALGO_SCAN_REDUCE, per[int(np.argmax(L))][0], vid, None)
    report("C5 batch", "fused scan + dot, one call per range (10,000 calls)", 12 * n5, lambda: [
        B.dr_scan_reduce(tb, vid, vmul, B.DR_ACC_COMPENSATED, 0.0, rr, workspace=ws1, host_check=False)
        for tb, rr in per], n_reps=2)
    del x, y, s5, gx, gy, per, tab, tsc, tdt, tbm, trs

    # Black-Scholes for_each (the paper's Black Scholes benchmark): 2^28
    # options, 8 equal segments; 16 bytes read and 8 written per option
    t = I.options()
    L = t["lengths"]
    ins = [to_dev(t[n]) for n in ("S", "K", "T", "V")]
    call, put = torch.empty_like(ins[0]), torch.empty_like(ins[0])
    tbs = B.segments([pieces(a, L) for a in ins], [pieces(call, L), pieces(put, L)])
    report("Black-Scholes", "2^28 options: call and put", 24 * sum(L), lambda: B.dr_for_each(
        tbs, B.make_view("black_scholes", B.DR_F32, t["r"]), B.DR_F32, workspace=ws, host_check=False))
    del t, ins, call, put, tbs

    flags = B.dr_check_device_error(dev)
    for w_ in (ws, ws5, ws1, ws_s, ws_d, ws_b, ws_r):
        flags |= w_.device_status()
    print(json.dumps({"device_fault_flags": flags}), flush=True)
    return 0 if flags == 0 else 1


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU leg (oracle baseline and error figures)")
    ap.add_argument("--copy-only", action="store_true",
                    help="run only a plain copy (for_each identity, 2^28 f32) K times: the known-size "
                         "kernel that calibrates the HBM byte counters")
    ap.add_argument("--accuracy", metavar="PATH",
                    help="also write the accuracy record (every result against the binary64 oracle) as "
                         "markdown to PATH (needs the CPU leg)")
    ap.add_argument("--configs", action="store_true",
                    help="time every workload alone at full size and print one JSON line per case instead "
                         "of the step line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (each GPU would scan its own "
              "segments and exchange only segment totals); run with --gpus 1", file=sys.stderr)
        return 2

    if args.configs:
        return configs_report(max(args.steps, 5))

    import torch

    from paper_2406_00158_amd import binding as B

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    if args.copy_only:
        N = 1 << 28
        b = torch.rand(N, device=dev)
        a = torch.empty(N, device=dev)
        t_copy = B.segments([[b]], [[a]])
        v_copy = B.make_view("identity", B.DR_F32)
        ws = B.Workspace(dev)
        for _ in range(args.warmup + args.steps):
            B.dr_for_each(t_copy, v_copy, B.DR_F32, workspace=ws, host_check=False)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 8 * N, "launches": args.warmup + args.steps}), flush=True)
        return 0

    if not os.environ.get("DR_TUNE_CACHE"):
        import tempfile
        os.environ["DR_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="dr_tune_"), "tune.json")
    t_setup = time.perf_counter()
    print("[bench] generating the seeded inputs of the four workloads", file=sys.stderr, flush=True)
    ops, host, out = setup(dev)
    t_setup = time.perf_counter() - t_setup
    print(f"[bench] setup {t_setup:.1f} s; {len(ops)} operations per step", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream(dev)
    step_bytes = sum(o.nbytes for o in ops)

    for _ in range(args.warmup):
        for o in ops:
            o.fn()
    torch.cuda.synchronize()

    # timed region: K whole steps, with per-operation HIP events on the launch stream
    ev = [[] for _ in ops]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(args.steps):
        for i, o in enumerate(ops):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            o.fn()
            e1.record(stream)
            ev[i].append((e0, e1))
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = start.elapsed_time(stop) / args.steps
    op_ms = [sum(e0.elapsed_time(e1) for e0, e1 in v) / len(v) for v in ev]
    value = step_bytes / (ms_per_step * 1e-3) / 1e9
    flags = B.dr_check_device_error(dev)
    for w_ in out["workspaces"]:
        flags |= w_.device_status()
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.3f} ms per step", file=sys.stderr, flush=True)

    per_op = {}
    for o, ms in zip(ops, op_ms):
        gbs = o.nbytes / (ms * 1e-3) / 1e9
        per_op[o.name] = {"ms": round(ms, 4), "bytes": o.nbytes, "GB/s": round(gbs, 1),
                          "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}

    # roofline: the longest-running operation that is one kernel launch (the
    # reductions and the single-pass scans add a 2-5 us prologue that zeroes
    # their counters); the two-pass scans are three launches per call: those
    # are reported per op only
    single = [(ms, o) for o, ms in zip(ops, op_ms) if o.kernel]
    dom_ms, dom = max(single, key=lambda p: p[0])
    achieved = dom.nbytes / (dom_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom.kernel, "op": dom.name, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": load_traffic(dom.kernel), "algorithmic_bytes_per_launch": dom.nbytes}
    scan_ops = {o.name: per_op[o.name]["frac_of_peak"] for o in ops if "scan" in o.name}

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "the four full-size workloads in one step: triad (2^28 f32, 8 segments: for_each "
                               "a = b + 3c, compensated dot), scan (2^30 int32 in 16 Dirichlet segments -> int64 "
                               "and -> int32; 2^28 f32 in 16 segments with f64 and with f32 carries), precision "
                               "(2^29 mixture, f32 and bf16: sum of squares and dot, compensated and plain), "
                               "batch (10,000 ragged ranges, 2^28 f32: fused scan + dot from a hipGraph, "
                               "backward: broadcast multiply and reverse scan)",
                   "bytes_per_step": step_bytes, "frac_of_peak": round(value / HBM_PEAK_GBS, 4),
                   "dominant_op": ops[max(range(len(ops)), key=lambda i: op_ms[i])].name,
                   "scan_ops_frac_of_peak": scan_ops,
                   "per_op": per_op, "autotuned": out["tuning"], "device_fault_flags": flags,
                   "wall_s": round(wall, 3),
                   "setup_s": round(t_setup, 1)},
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if not args.no_cpu:
        print("[bench] per-range check: 64 batch ranges alone", file=sys.stderr, flush=True)
        per_range = per_range_leg(host, out, dev)
        flags |= per_range["status"]
        print("[bench] CPU leg: oracle (serial), oracle on every core, plain loops", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        errs, base = cpu_leg(host, out, per_range)
        for name, e in errs.items():
            per_op[name]["error_vs_fp64_oracle"] = e
        base["leg_s"] = round(time.perf_counter() - t0, 1)
        line["cpu_baseline"] = base
        line["config"]["device_fault_flags"] = flags
    print(json.dumps(line), flush=True)
    if args.accuracy:
        if args.no_cpu:
            print("[bench] --accuracy needs the CPU leg: no record written", file=sys.stderr, flush=True)
        else:
            write_accuracy(args.accuracy, line, torch.cuda.get_device_name(dev))
    return 0 if flags == 0 else 1


if __name__ == "__main__":
    sys.exit(main())
