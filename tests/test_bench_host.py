"""Host-side parts of bench.py: the one-GPU rule, the byte models of the
roofline, and the counter file check (traffic is reported only for the
kernel source it was measured on)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_byte_models():
    import bench
    # one hyperedge {0, 1} over two nodes, d = 8, BF16: 2 nnz, 3 rows, 1 hyperedge
    n_nodes, n_edges, nnz, d, s = 2, 1, 2, 8, 2
    assert bench.sweep_stream_bytes(n_nodes, n_edges, nnz, d, s) == 2 * nnz * (d * s + 4) + 3 * (2 * d * s + 12) + 4
    assert bench.sweep_min_bytes(n_nodes, n_edges, nnz, d, s) == 3 * (2 * d * s + 12) + 8 * nnz + 4
    # the stream model never undercuts the compulsory one
    for args in ((2_000_000, 1_500_000, 13_088_147, 128, 2), (10, 0, 0, 32, 4), (1, 1, 1, 8, 4)):
        assert bench.sweep_stream_bytes(*args) >= bench.sweep_min_bytes(*args)


def test_counters_follow_the_kernel_source(tmp_path, monkeypatch):
    import bench
    path = tmp_path / "counters.txt"
    path.write_text("# header\nhbm_bytes_per_launch = 1.5e9\nkernel_source_sha256 = %s\n" % bench.kernel_source_digest())
    monkeypatch.setitem(bench.COUNTERS_FILES, "x", str(path))
    assert bench.read_counters("x") == pytest.approx(1.5e9)
    path.write_text("hbm_bytes_per_launch = 1.5e9\nkernel_source_sha256 = 0000\n")
    assert bench.read_counters("x") is None
    assert bench.read_counters("no-such-workload") is None

