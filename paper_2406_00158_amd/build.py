"""Build of the HIP library libdr.so for gfx950 (hipcc, in-tree).

    python -m paper_2406_00158_amd.build

Every source is compiled with -ffp-contract=off (the stream triad must
round twice: a = fl(b + fl(s*c))) and without packed binary32 instructions.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libdr.so")
OBJDIR = os.path.join(HERE, "_build")

SOURCES = ["dr_api.cpp", "k_elementwise.hip", "k_reduce.hip", "k_scan.hip", "k_scan_wide.hip", "k_scan_chain.hip",
           "k_plan.hip", "dr_static.hip"]
HEADERS = ["dr_device.hpp", "dr_internal.hpp", "dr_combine.hpp", "k_scan_core.hpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",
    "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-I", INCLUDE,
    "-I", CSRC,
]


def _obj(src: str) -> str:
    return os.path.join(OBJDIR, src + ".o")


def _compile(src: str) -> tuple[str, str]:
    out = _obj(src)
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    noise = "'-packed-fp32-ops' is not a recognized feature"
    err = "\n".join(l for l in r.stderr.splitlines() if noise not in l)
    return src, err


def build(jobs: int | None = None, verbose: bool = False) -> str:
    """Compile every source and link libdr.so. Always recompiles."""
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for src, err in ex.map(_compile, SOURCES):
            if err.strip() and verbose:
                print(f"[{src}]\n{err}", file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *[_obj(s) for s in SOURCES]]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
