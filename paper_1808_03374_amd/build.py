"""Build libgkl.so (gfx950) from the HIP sources in csrc/ with hipcc.

Each source compiles to its own object in parallel, then one link step makes
the shared library next to this file.  Called by __graft_entry__.build() and
by the binding when no library is present.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgkl.so")
BUILD_DIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("GKL_OFFLOAD_ARCH", "gfx950")

SOURCES = ["engine.hip", "k_stats.hip", "k_matvec.hip", "k_ortho.hip", "k_svd.hip", "k_pro.hip",
           "k_mixed.hip", "k_block.hip", "k_batch.hip", "mixed.hip", "batched.hip"]

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # packed-FP32 instructions are disabled on purpose (see the design notes)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # matrix-core operands and accumulators in VGPRs: with the default
         # heuristic the loop-carried accumulators of every matrix-core loop were
         # rotated through 24-64 v_accvgpr moves per iteration
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-Wall", "-Wno-unused-function", "-Wno-unused-result"]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
