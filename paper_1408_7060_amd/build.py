"""Build libetaim.so in-tree with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libetaim.so")
ARCH = os.environ.get("ETAIM_OFFLOAD_ARCH", "gfx950")


def command(out: str = LIB) -> list[str]:
    return [
        "hipcc", "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared", "-fopenmp",
        # separate roundings by default; kernels opt in to contraction where it measured faster
        "-ffp-contract=off",
        # no packed FP32 instructions in device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(HERE, "..", "include"),
        os.path.join(CSRC, "etaim.hip"), os.path.join(CSRC, "setup.cpp"),
        "-Wl,-rpath,/opt/rocm/llvm/lib", "-o", out,
    ]


def build(verbose: bool = True) -> str:
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
