"""Build libsn.so (HIP, gfx950) in-tree with hipcc.

Every HIP source is compiled for gfx950 with packed-FP32 instructions
disabled (the packed forms are avoided on this hardware), then linked into
one shared library next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsn.so")
SOURCES = ["sweep.hip", "flux.hip", "dsa.hip", "hp.hip", "noalloc.hip", "capi.hip"]
HOST_ONLY = {"capi.hip"}  # host code only: no device compilation pass
# The sweeps issue from one or two waves per SIMD, so their speed depends on how
# well independent instructions are interleaved in the in-order stream; the
# iterative ILP machine scheduler measured 167 -> 161 us (FP64) and 119 -> 116
# us (FP32) on the 256^2 S8 2D sweep, and no change on the 3D sweeps.
EXTRA = {"sweep.hip": ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"]}
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(HERE, "..", "include")]


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, src.replace(".hip", ".o"))
    extra = ["--cuda-host-only"] if src in HOST_ONLY else []
    extra += EXTRA.get(src, [])
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
