"""Summaries of rocprofv3 runs: HBM traffic per kernel launch from the
hardware counters, and kernel durations from a kernel trace.

Traffic: two counter runs of the benchmark (FETCH_SIZE, then WRITE_SIZE;
KiB per dispatch) are scaled by what the same counters read for a plain copy
kernel of known size (`bench.py --copy-only`: a for_each identity over 2^28
binary32 elements, 1 GiB read and 1 GiB written per launch), and written to
profiles/traffic.json together with a hash of the kernel sources (bench.py
reports the figure only while the sources are unchanged) and a text summary.

    python -m paper_2406_00158_amd.traffic FETCH_DIR WRITE_DIR COPY_FETCH_DIR COPY_WRITE_DIR [OUT_MD]

Durations: the `--stats` table of a `rocprofv3 --kernel-trace --stats
--output-format csv` run, the library's kernels only, as a markdown table.

    python -m paper_2406_00158_amd.traffic --kernels TRACE_DIR [OUT_MD]
"""
from __future__ import annotations

import collections
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["dr_device.hpp", "dr_internal.hpp", "dr_combine.hpp", "k_scan_core.hpp", "k_elementwise.hip",
                  "k_reduce.hip", "k_scan.hip", "k_scan_wide.hip", "k_scan_chain.hip", "k_plan.hip", "dr_api.cpp",
                  "dr_static.hip"]
COPY_ELEMS = 1 << 28


def sources_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2406_00158_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(kernel: str) -> str:
    """`void dr::k_scan_apply<1, 1, ...>(dr::LaunchArgs)` -> `k_scan_apply<1, 1, ...>`."""
    k = kernel.split("(")[0].replace("void ", "").replace("dr::", "")
    return k.strip()


def _rows(d: str) -> list[dict]:
    out = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            out += list(csv.DictReader(fh))
    return out


def _per_kernel(rows: list[dict], counter: str) -> dict[str, list[float]]:
    acc: dict[str, list[float]] = collections.defaultdict(list)
    for r in rows:
        if r.get("Counter_Name") == counter:
            acc[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return acc


def summarize(fetch_dir: str, write_dir: str, copy_fetch_dir: str, copy_write_dir: str) -> dict:
    f_b, w_b = _per_kernel(_rows(fetch_dir), "FETCH_SIZE"), _per_kernel(_rows(write_dir), "WRITE_SIZE")
    f_c, w_c = _per_kernel(_rows(copy_fetch_dir), "FETCH_SIZE"), _per_kernel(_rows(copy_write_dir), "WRITE_SIZE")

    def copy_kib(d):
        vals = [v for k, vs in d.items() if k.startswith("k_for_each") for v in vs]
        if not vals:
            raise SystemExit("no k_for_each dispatch in the copy run")
        return sum(vals) / len(vals)

    fetch_factor = copy_kib(f_c) * 1024 / (4 * COPY_ELEMS)   # counter bytes per true byte
    write_factor = copy_kib(w_c) * 1024 / (4 * COPY_ELEMS)
    kernels = {}
    for k in sorted(set(f_b) | set(w_b)):
        fb = sum(f_b[k]) / len(f_b[k]) * 1024 / fetch_factor if f_b.get(k) else 0.0
        wb = sum(w_b[k]) / len(w_b[k]) * 1024 / write_factor if w_b.get(k) else 0.0
        kernels[k] = {"fetch_bytes": round(fb), "write_bytes": round(wb), "bytes_per_launch": round(fb + wb),
                      "dispatches": max(len(f_b.get(k, [])), len(w_b.get(k, [])))}
    # bench.py looks kernels up by base name; keep one entry per base name
    # when it is unambiguous
    by_base: dict[str, list[str]] = collections.defaultdict(list)
    for k in kernels:
        by_base[k.split("<")[0]].append(k)
    for base, ks in by_base.items():
        if len(ks) == 1 and base not in kernels:
            kernels[base] = kernels[ks[0]]
    return {"sources": sources_hash(),
            "calibration": {"fetch_factor": round(fetch_factor, 4), "write_factor": round(write_factor, 4),
                            "copy_bytes_each_way": 4 * COPY_ELEMS},
            "kernels": kernels}


def kernel_stats(trace_dir: str) -> list[dict]:
    """Rows of the kernel statistics CSV of a trace run (library kernels
    first by total time, then the rest), durations in microseconds."""
    rows = []
    for f in glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                rows.append({"kernel": short_name(r["Name"]), "calls": int(r["Calls"]),
                             "total_us": float(r["TotalDurationNs"]) / 1e3, "avg_us": float(r["AverageNs"]) / 1e3,
                             "min_us": float(r["MinNs"]) / 1e3, "max_us": float(r["MaxNs"]) / 1e3})
    rows.sort(key=lambda r: (not r["kernel"].startswith("k_"), -r["total_us"]))
    return rows


def kernels_md(trace_dir: str) -> str:
    lines = ["| kernel | calls | total us | avg us | min us | max us |", "|---|---|---|---|---|---|"]
    for r in kernel_stats(trace_dir):
        if r["kernel"].startswith("k_"):
            lines.append(f"| `{r['kernel']}` | {r['calls']} | {r['total_us']:.1f} | {r['avg_us']:.1f} | "
                         f"{r['min_us']:.1f} | {r['max_us']:.1f} |")
    return "\n".join(lines) + "\n"


def main(argv: list[str]) -> int:
    if argv and argv[0] == "--kernels":
        if len(argv) < 2:
            print(__doc__, file=sys.stderr)
            return 2
        text = kernels_md(argv[1])
        print(text)
        if len(argv) > 2:
            with open(argv[2], "w") as f:
                f.write(text)
        return 0
    if len(argv) < 4:
        print(__doc__, file=sys.stderr)
        return 2
    rec = summarize(*argv[:4])
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    lines = [f"calibration: FETCH_SIZE reads {rec['calibration']['fetch_factor']} counter bytes and "
             f"WRITE_SIZE {rec['calibration']['write_factor']} per true byte of the 1 GiB + 1 GiB copy", "",
             "| kernel | dispatches | fetch GB/launch | write GB/launch |", "|---|---|---|---|"]
    for k, v in rec["kernels"].items():
        if "<" in k or k.startswith("k_prologue") or k.startswith("k_zero"):
            lines.append(f"| `{k}` | {v['dispatches']} | {v['fetch_bytes'] / 1e9:.4f} | {v['write_bytes'] / 1e9:.4f} |")
    text = "\n".join(lines) + "\n"
    print(text)
    if len(argv) > 4:
        with open(argv[4], "w") as f:
            f.write(text)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
