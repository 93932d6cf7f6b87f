"""Address and undefined-behaviour sanitizer runs of the host-side code (CPU
only): the FP64 oracle with gcc, and the library's host C++ (validation,
coarsening, plan sizing, the error paths of plan creation, score-plan
sizing) with g++, each driven over seeded random hypergraphs by a small
program under tests/sanitize/.  Device code is not part of these builds."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-O1", "-g"]


def _run(cmd, exe):
    build = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], cwd=ROOT, capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, (run.stdout + run.stderr)[-4000:]
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr
    return run.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    out = _run(["gcc", "-std=c11", "-Wall", "-Wno-unknown-pragmas"] + SAN +
               ["oracle/hnv_oracle.c", "tests/sanitize/oracle_sanitize.c", "-lm", "-o", exe], exe)
    assert "ok" in out


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"),
                    reason="g++ or the HIP headers not available")
def test_host_library_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_san")
    out = _run(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", "include", "-I", "paper_2103_09660_amd/csrc",
                "-I", "/opt/rocm/include"] + SAN +
               ["paper_2103_09660_amd/csrc/hnv_host.cpp", "tests/sanitize/host_sanitize.cpp", "-o", exe], exe)
    assert "ok" in out
