"""Builds the HIP library ``libhnv.so`` in-tree for gfx950 with hipcc.

The library is the host C++ (validation, coarsening, plan) plus the HIP
kernels, linked into one shared object that exports the C ABI declared in
``include/hnv.h``.  Packed FP32 instructions are disabled for device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libhnv.so")
SOURCES = [os.path.join(CSRC, "hnv_host.cpp"), os.path.join(CSRC, "hnv_kernels.hip")]
ARCH = os.environ.get("HNV_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def command(out: str) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function",
            "-I", INCLUDE, "-I", CSRC, "-o", out] + SOURCES


def build(verbose: bool = False) -> str:
    """Compiles every time it is called (the result replaces libhnv.so atomically)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
