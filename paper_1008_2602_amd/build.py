"""Build libfdtd.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libfdtd.so")
SOURCES = ["fdtd_kernels.hip", "fdtd_kernels2.hip", "fdtd_kernels_eps.hip", "fdtd_noalloc.hip",
           "fdtd_host.cpp"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off: plain scalar FP32 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit FMA contraction: every fused multiply-add is an explicit fmaf,
    # so a cell's arithmetic is identical in every code path and tile shape
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, *[f"-D{d}" for d in defines], "-I", INCLUDE, "-I", CSRC,
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, stdout=None if verbose else subprocess.DEVNULL)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
