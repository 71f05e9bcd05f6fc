"""Builds liblbmcrack.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbmcrack.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
SOURCES = ["api.cpp", "sweep.hip", "sweep2.hip", "sweep_block_f64.hip", "sweep_block_f32.hip",
           "sweep_block_f16.hip", "sweep_block_f16_t8.hip", "sweep_block_bf16.hip", "crack.hip",
           "batch.hip", "io.hip", "adjoint.hip", "macro_bc.hip"]
# per-source flags: the FP16 sweep of eight steps unrolls its 24-row march in
# full (see that file)
EXTRA = {"sweep_block_f16_t8.hip": ["-mllvm", "-pragma-unroll-threshold=65536"]}
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into liblbmcrack.so (always recompiles): one
    hipcc process per source in parallel (objects under _build/), then one
    link."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    compile_flags = [f for f in FLAGS if f != "-shared"]
    cmds = [[hipcc, *compile_flags, *EXTRA.get(src, []), "-I" + INCLUDE, "-c", os.path.join(CSRC, src),
             "-o", os.path.join(bdir, src + ".o")] for src in SOURCES]
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
    for c, res in zip(cmds, results):
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError(f"hipcc failed on {os.path.basename(c[-3])}")
    tmp = LIB + ".tmp"
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-o", tmp] + [c[-1] for c in cmds]
    if verbose:
        print(" ".join(link), flush=True)
    res = subprocess.run(link, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("linking liblbmcrack.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
