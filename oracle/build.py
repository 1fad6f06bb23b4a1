"""Build the C++/OpenMP part of the CPU oracle (liborcdirect.so) in-tree.

TEST INFRASTRUCTURE ONLY: the library is the direct-summation oracle used for systems too large for
the dense solve; nothing in the product path loads it.

    python -m oracle.build

Compiled with g++ for generic x86-64-v3 (AVX2 + FMA), without fast-math, so that the same binary
runs on any current host and its arithmetic stays IEEE float64.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "direct_sum.cpp")
LIB = os.path.join(HERE, "liborcdirect.so")
FLAGS = ["-O3", "-std=c++17", "-march=x86-64-v3", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-Wall"]


def build(verbose: bool = True) -> str:
    tmp = LIB + ".tmp"
    cmd = [os.environ.get("CXX", "g++"), *FLAGS, SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"building the oracle library failed:\n{r.stderr}")
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
