#!/usr/bin/env python3
"""Benchmark of the segmented for_each / transform_reduce / inclusive_scan
path on one MI355X.

Workload ("stream triad + dot", 2^28 binary32 elements, 8 equal segments,
uniform[-1, 1), s = 3): one step is one pass of the whole hot path over it:

  1. for_each      a = b + s*c                     (zip | transform | for_each)
  2. reduce        R = dot(b, c), compensated       (zip | transform(mul) | reduce)
  3. scan          S = inclusive_scan(a), binary64 carries across tiles/segments
  4. batched       per segment: scan(b) and dot(b, c) fused in one launch
  5. backward      dR/db = g*c, dR/dc = g*b (broadcast multiply), and the scan
                   adjoint: reverse inclusive scan of an upstream gradient

`value` is the whole step's algorithmic HBM bytes (each input read once, each
output written once) divided by its time. `roofline` is for the kernel that
takes the largest share of the step, timed with HIP events on its stream.
`cpu_baseline` times the serial CPU oracle on a bounded sample of the same
workload. Inputs are resident in HBM before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2406_00158_amd.traffic import sources_hash  # noqa: E402 (no torch import)

METRIC = "effective HBM GB/s (% of peak) for fused reduce/scan; batched+compensated vs plain"
HBM_PEAK_GBS = 8000.0
N = 1 << 28
SEGMENTS = 8
SCALAR = 3.0


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


def cpu_baseline(reps: int = 3) -> dict:
    """The serial oracle (plain C, one thread) on the same workload (all
    2^28 elements, same segments), the same five steps, `reps` times."""
    import numpy as np

    import oracle as O
    from paper_2406_00158_amd import inputs as I

    t = I.triad(n=N, segments=SEGMENTS)
    L = t["lengths"]
    b, c = I.split(t["b"], L), I.split(t["c"], L)
    g = np.ones(1)
    t0 = time.perf_counter()
    for _ in range(reps):
        a = O.for_each(b, c, O.F32, O.AXPY, O.F32, alpha=SCALAR)
        O.reduce(b, c, O.F32, O.MUL)
        O.scan(a, None, O.F32, O.IDENTITY)
        O.scan(b, None, O.F32, O.IDENTITY, mode=O.BATCH)
        O.reduce(b, c, O.F32, O.MUL, mode=O.BATCH)
        O.reduce_grad(b, c, O.F32, O.MUL, g, 0)
        O.reduce_grad(b, c, O.F32, O.MUL, g, 1)
        O.scan(a, None, O.F32, O.IDENTITY, reverse=True)
        del a
    dt = time.perf_counter() - t0
    return {"value": round(reps * step_bytes(N) / dt / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"the whole workload (2^28 elements, {SEGMENTS} segments), the same five steps "
                      f"{reps} times, serial C oracle (gcc -O2, binary64/int64 arithmetic), one thread, "
                      f"{dt:.2f} s"}


BYTES_PER_ELEM = {"for_each": 12, "reduce": 8, "scan": 8, "batched": 12, "backward_mul": 16, "backward_scan": 8}


def step_bytes(n: int) -> int:
    return n * sum(BYTES_PER_ELEM.values())


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--copy-only", action="store_true",
                    help="run only a plain copy (for_each identity, 2^28 f32) K times: the known-size "
                         "kernel that calibrates the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (see DESIGN.md for how the "
              "path would shard); run with --gpus 1", file=sys.stderr)
        return 2

    import torch

    from paper_2406_00158_amd import binding as B

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(1002)
    b = torch.rand(N, device=dev, generator=gen) * 2 - 1
    c = torch.rand(N, device=dev, generator=gen) * 2 - 1
    a = torch.empty(N, device=dev)
    s = torch.empty(N, device=dev)
    sb = torch.empty(N, device=dev)
    gb = torch.empty(N, device=dev)
    gc = torch.empty(N, device=dev)
    gs = torch.empty(N, device=dev)
    up = torch.ones(N, device=dev)          # upstream gradient of S

    def seg(t):
        k = N // SEGMENTS
        return [t[i * k:(i + 1) * k] for i in range(SEGMENTS)]

    if args.copy_only:
        t_copy = B.segments([seg(b)], [seg(a)])
        v_copy = B.make_view("identity", B.DR_F32)
        for _ in range(args.warmup + args.steps):
            B.dr_for_each(t_copy, v_copy, B.DR_F32, host_check=False)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 8 * N, "launches": args.warmup + args.steps}), flush=True)
        return 0

    t_triad = B.segments([seg(b), seg(c)], [seg(a)])
    t_dot = B.segments([seg(b), seg(c)])
    t_scan = B.segments([seg(a)], [seg(s)])
    t_batch = B.segments([seg(b), seg(c)], [seg(sb)], mode="batch")
    t_grad = B.segments([seg(b), seg(c)], [seg(gb), seg(gc)])
    t_rscan = B.segments([seg(up)], [seg(gs)])
    ws = B.Workspace(dev)
    ws_b = B.Workspace(dev)
    R = torch.zeros(1, dtype=torch.float64, device=dev)
    Rp = torch.zeros(1, dtype=torch.float64, device=dev)
    Rb = torch.zeros(SEGMENTS, dtype=torch.float64, device=dev)
    g = torch.ones(1, dtype=torch.float64, device=dev)
    v_axpy = B.make_view("axpy", B.DR_F32, SCALAR)
    v_mul = B.make_view("mul", B.DR_F32)
    v_id = B.make_view("identity", B.DR_F32)

    ops = {
        "for_each": lambda: B.dr_for_each(t_triad, v_axpy, B.DR_F32, host_check=False),
        "reduce": lambda: B.dr_transform_reduce(t_dot, v_mul, B.DR_ACC_COMPENSATED, 0.0, R, workspace=ws,
                                                host_check=False),
        "scan": lambda: B.dr_inclusive_scan(t_scan, v_id, B.DR_F32, 0, workspace=ws, host_check=False),
        "batched": lambda: B.dr_scan_reduce(t_batch, v_id, v_mul, B.DR_ACC_COMPENSATED, 0.0, Rb, 0,
                                            workspace=ws_b, host_check=False),
        "backward_mul": lambda: B.dr_broadcast_mul(t_grad, v_mul, g, 2, host_check=False),
        "backward_scan": lambda: B.dr_inclusive_scan(t_rscan, v_id, B.DR_F32, B.DR_SCAN_REVERSE, workspace=ws,
                                                     host_check=False),
    }

    def step():
        for fn in ops.values():
            fn()

    stream = torch.cuda.current_stream(dev)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K whole steps, with per-kernel HIP events on the launch stream
    ev = {k: [] for k in ops}
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(args.steps):
        for k, fn in ops.items():
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            ev[k].append((e0, e1))
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start.elapsed_time(stop)
    ms_per_step = total_ms / args.steps
    per_op_ms = {k: sum(e0.elapsed_time(e1) for e0, e1 in v) / len(v) for k, v in ev.items()}
    value = step_bytes(N) / (ms_per_step * 1e-3) / 1e9

    # plain binary32 dot for the accuracy / cost contrast (outside the step)
    for _ in range(3):
        B.dr_transform_reduce(t_dot, v_mul, B.DR_ACC_PLAIN, 0.0, Rp, workspace=ws, host_check=False)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        B.dr_transform_reduce(t_dot, v_mul, B.DR_ACC_PLAIN, 0.0, Rp, workspace=ws, host_check=False)
    e1.record(stream)
    torch.cuda.synchronize()
    plain_ms = e0.elapsed_time(e1) / 10
    flags = ws.device_status() | ws_b.device_status()

    # roofline: the longest-running single kernel of the step. The ops
    # below are one main kernel launch each (the reduce adds a 2-5 us
    # counter-zeroing prologue), so HIP events around the op time that
    # kernel; the scans are several passes in one call and are reported per
    # op (per_op) and per kernel in the committed kernel-trace profile.
    single = {"for_each": "k_for_each", "reduce": "k_reduce_stream", "backward_mul": "k_broadcast_mul"}
    dom = max(single, key=lambda k: per_op_ms[k])
    kernel_name = single[dom]
    achieved = BYTES_PER_ELEM[dom] * N / (per_op_ms[dom] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": kernel_name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": load_traffic(kernel_name),
                "algorithmic_bytes_per_launch": BYTES_PER_ELEM[dom] * N}

    per_op = {k: {"ms": round(v, 4), "GB/s": round(BYTES_PER_ELEM[k] * N / (v * 1e-3) / 1e9, 1),
                  "frac_of_peak": round(BYTES_PER_ELEM[k] * N / (v * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
              for k, v in per_op_ms.items()}
    per_op["reduce_plain"] = {"ms": round(plain_ms, 4),
                              "GB/s": round(8 * N / (plain_ms * 1e-3) / 1e9, 1),
                              "frac_of_peak": round(8 * N / (plain_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

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
        "config": {"workload": "stream triad + dot (2^28 f32, 8 equal segments, uniform[-1,1), s=3): "
                               "for_each, compensated dot, scan with f64 carries, batched fused scan+dot, "
                               "backward (dot adjoint + reverse scan)",
                   "elements": N, "segments": SEGMENTS, "bytes_per_step": step_bytes(N),
                   "frac_of_peak": round(value / HBM_PEAK_GBS, 4), "dominant_kernel": kernel_name,
                   "dominant_op": max(per_op_ms, key=per_op_ms.get),
                   "per_op": per_op, "device_fault_flags": flags, "wall_s": round(wall, 3)},
        "roofline": roofline,
        "cpu_baseline": None,
    }
    del a, s, sb, gb, gc, gs, up
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
