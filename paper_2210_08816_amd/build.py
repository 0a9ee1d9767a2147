"""Build the gfx950 shared library libkv_hip.so in-tree with hipcc.

Usage: python -m paper_2210_08816_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkv_hip.so")

SOURCES = ["kv_capi.cpp", "kv_eig1d.cpp", "kv_stencil.hip", "kv_fd.hip", "kv_fd_split.hip", "kv_vec.hip",
           "kv_hess.hip", "kv_transfer.hip", "kvnn.hip", "kv_static.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
    "-Wall", "-Wno-unused-function",
    # packed FP32 arithmetic is kept off for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in ordinary VGPRs: without it the compiler keeps the
    # FD kernels' loop-carried accumulators in VGPRs and copies them into and
    # out of the AGPRs around every K chunk (twice the registers and 128 extra
    # moves per chunk in the inverse passes)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
]


def hipcc() -> str:
    for cand in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *FLAGS, "-I", os.path.join(HERE, "..", "include"), *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libkv_hip.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
