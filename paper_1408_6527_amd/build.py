"""Build libpfmm.so (HIP for gfx950) in-tree.

    python -m paper_1408_6527_amd.build          # compile every source, link the library

The library is linked against the HIP runtime by its SONAME (libamdhip64.so.7), so a process
that has already loaded PyTorch's HIP runtime reuses it instead of loading a second copy.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build", "pfmm")
LIB = os.path.join(HERE, "libpfmm.so")
ARCH = os.environ.get("PFMM_ARCH", "gfx950")

SOURCES = ["tables.cpp", "tree.hip", "expansions.hip", "m2l.hip", "mac.hip", "p2p.hip", "solver.hip", "api.hip"]
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-Wno-unused-function"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _scratch_users(remarks: str):
    """Library kernels (namespace pfmm) whose compiled code needs a private (scratch) segment."""
    out, name = [], None
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name and "4pfmm" in name and int(m.group(1)) > 0:
            out.append((name, int(m.group(1))))
    return out


# The M2L schedule and the fixed-order L2P are fully unrolled, compile-time table-driven loops; their
# unrolled size exceeds the default limit for pragma-directed unrolling at the higher orders.
EXTRA = {"m2l.hip": ["-mllvm", "-pragma-unroll-threshold=60000"],
         "expansions.hip": ["-mllvm", "-pragma-unroll-threshold=200000"]}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *FLAGS, *EXTRA.get(src, []), "-Rpass-analysis=kernel-resource-usage", "-x", "hip", "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{r.stderr}")
    spill = _scratch_users(r.stderr)
    if spill:
        # Every kernel of the library is designed to fit in registers; a private segment means
        # register spills, which also put the dispatch's scratch demand far above what any kernel
        # here has been validated with.
        raise RuntimeError(f"{src}: kernels need scratch memory: {spill}")
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libpfmm.so failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    try:
        build()
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
