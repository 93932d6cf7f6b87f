"""Builds the HIP library ``libhnv.so`` in-tree for gfx950 with hipcc.

The library is the host C++ (validation, coarsening, plan) plus the HIP
kernels (refinement, scoring, GPU coarsening), compiled in parallel and
linked into one shared object that exports the C ABI declared in
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
SOURCES = [os.path.join(CSRC, "hnv_host.cpp"), os.path.join(CSRC, "hnv_kernels.hip"),
           os.path.join(CSRC, "hnv_coarsen.hip"), os.path.join(CSRC, "hnv_devplan.hip")]
ARCH = os.environ.get("HNV_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC]


def compile_command(src: str, obj: str) -> list:
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    return [hipcc(), f"--offload-arch={ARCH}"] + FLAGS + ["-c"] + lang + [src, "-o", obj]


def link_command(objs: list, out: str) -> list:
    return [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out] + objs


def build(verbose: bool = False) -> str:
    """Compiles every time it is called (the result replaces libhnv.so atomically)."""
    tag = "tmp%d" % os.getpid()
    objs = [os.path.join(CSRC, os.path.basename(src) + "." + tag + ".o") for src in SOURCES]
    tmp = LIB + "." + tag
    try:
        jobs = []
        for src, obj in zip(SOURCES, objs):
            cmd = compile_command(src, obj)
            if verbose:
                print(" ".join(cmd), file=sys.stderr)
            jobs.append((cmd, subprocess.Popen(cmd)))
        for cmd, job in jobs:
            if job.wait() != 0:
                raise subprocess.CalledProcessError(job.returncode, cmd)
        cmd = link_command(objs, tmp)
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    finally:
        for f in objs + [tmp]:
            if os.path.exists(f):
                os.remove(f)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
