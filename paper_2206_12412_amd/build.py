"""Builds liblbmcrack.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbmcrack.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
SOURCES = ["api.cpp", "sweep.hip", "sweep2.hip", "crack.hip", "batch.hip", "io.hip", "adjoint.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into liblbmcrack.so (always recompiles)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    tmp = LIB + ".tmp"
    cmd = [hipcc, *FLAGS, "-I" + INCLUDE, "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building liblbmcrack.so")
    os.replace(tmp, LIB)
    del objs
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
