"""Builds libscan.so (the HIP library) in place with hipcc for gfx950."""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libscan.so")
SOURCES = ["api.hip", "build.hip", "intersect.hip", "segsort.hip", "query.hip", "server.hip", "quality.hip",
           "weighted.hip", "lsh.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -O3, no fast-math, no FP contraction (the FP64 similarity must round like
# the host), packed FP32 instructions disabled.
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]
# The atomic optimizer folds a wavefront's uniform atomics into one (DPP).
# intersect.hip issues its few wavefront-level LDS atomics from one lane by
# hand and reads their results later, which the optimizer would defeat (it
# broadcasts each result, and so waits for it, right after the atomic).
ATOMIC_STRATEGY = {"intersect.hip": "None"}


def flags_for(src: str) -> list:
    return [*FLAGS, "-mllvm", f"-amdgpu-atomic-optimizer-strategy={ATOMIC_STRATEGY.get(src, 'DPP')}"]


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *flags_for(src), "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
