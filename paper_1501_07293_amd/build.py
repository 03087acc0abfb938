"""Build libmmag.so (the HIP library) in-tree for gfx950 with hipcc.

Usage: python -m paper_1501_07293_amd.build   (or build() from Python).
Every call recompiles; objects go to paper_1501_07293_amd/_build/.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmmag.so")
# the two largest first, so that the pool compiles them side by side
SOURCES = ["mm_fast.hip", "mm_fused.hip", "mm_api.hip", "mm_passes.hip", "mm_tensor.hip", "mm_llg.hip",
           "mm_adjoint.hip", "mm_batch.hip"]
ARCH = os.environ.get("MMAG_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # keep hipcc from forming packed FP32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


# The size-specialised FFT bodies feed literal zeros (the padding half of a line)
# into their first stage; with signed zeros ignored the compiler drops the
# additions of those zeros.  Only the sign of a zero result can differ.
EXTRA = {"mm_fast.hip": ["-fno-signed-zeros"], "mm_fused.hip": ["-fno-signed-zeros"],
         "mm_batch.hip": ["-fno-signed-zeros"]}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [HIPCC, *FLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
