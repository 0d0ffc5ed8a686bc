"""Build ``libchebdm.so`` (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Usage: ``python -m paper_2306_12616_amd.build`` (or ``__graft_entry__.build()``).
Every call recompiles all sources; objects go to ``_build/`` at the repo root.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB_PATH = os.path.join(HERE, "libchebdm.so")

SOURCES = ["api.hip", "api_batch.hip", "api_mlp.hip", "api_noalloc.hip", "k_batch.hip", "k_bounds.hip", "k_check.hip", "k_cheb.hip", "k_combine.hip",
           "k_gemm.hip", "k_lanczos.hip", "k_mlp.hip"]
ARCH = os.environ.get("CHEBDM_OFFLOAD_ARCH", "gfx950")

# -packed-fp32-ops: keep the compiler from forming packed FP32 VALU ops.
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", INCLUDE, "-I", CSRC,
]
# MFMA accumulators in VGPRs.  With its own heuristic the compiler kept the K loop's
# loop-carried accumulators in VGPRs but ran the MFMAs on AGPR copies, moving all 128
# accumulator registers in and out on every iteration of the float64 product loop (N = 4000,
# three products per launch: 3.41 -> 3.08 ms; N = 2000, four: 0.831 -> 0.751 ms).  Not for the
# batched product kernel: it gains nothing there at one wavefront per SIMD (512-problem batch:
# 4588 -> 4573 DM/s), and where its float32 tiles fit two wavefronts per SIMD the persistent
# grid doubles, which measured slower (4593 -> 3292 DM/s).
VGPR_FORM = ["-mllvm", "-amdgpu-mfma-vgpr-form"]
NO_VGPR_FORM = {"k_batch.hip"}


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the HIP toolchain is required to build libchebdm.so")
    return path


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    extra = [] if src in NO_VGPR_FORM else VGPR_FORM
    cmd = [hipcc(), *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = min(len(SOURCES), max(1, (os.cpu_count() or 2)))
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB_PATH)
    if verbose:
        print(f"built {LIB_PATH}")
    return LIB_PATH


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
