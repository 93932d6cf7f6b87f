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
    path.write_text("# header\nbf16.traffic_bytes_per_launch = 1.5e9\nbf16.l2_hit_rate = 0.25\n"
                    "kernel_source_sha256 = %s\n" % bench.kernel_source_digest())
    monkeypatch.setitem(bench.COUNTERS_FILES, "x", str(path))
    got = bench.read_counters("x", "bf16")
    assert got["traffic_bytes_per_launch"] == pytest.approx(1.5e9) and got["l2_hit_rate"] == 0.25
    assert bench.read_counters("x", "f32") is None
    path.write_text("bf16.traffic_bytes_per_launch = 1.5e9\nkernel_source_sha256 = 0000\n")
    assert bench.read_counters("x", "bf16") is None
    assert bench.read_counters("no-such-workload", "bf16") is None


def _write_pass(d, rows):
    import csv
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "1_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], r)))


def test_counter_summary_bytes_from_sized_requests(tmp_path):
    """Bytes per launch from the size-split request counts, averaged over the
    kernel's dispatches, for the sweep kernel and the copy calibration."""
    import bench
    k = bench.SWEEP_KERNELS["bf16"]
    cp = "__amd_rocclr_copyBuffer"
    reads = []
    for disp, (r128, r64, r32) in ((1, (100, 10, 4)), (2, (300, 30, 0))):
        reads += [(disp, k, "TCC_EA0_RDREQ_sum", r128 + r64 + r32), (disp, k, "TCC_EA0_RDREQ_128B_sum", r128),
                  (disp, k, "TCC_EA0_RDREQ_64B_sum", r64), (disp, k, "TCC_EA0_RDREQ_32B_sum", r32)]
    reads += [(9, cp, "TCC_EA0_RDREQ_sum", 8), (9, cp, "TCC_EA0_RDREQ_128B_sum", 8),
              (9, cp, "TCC_EA0_RDREQ_64B_sum", 0), (9, cp, "TCC_EA0_RDREQ_32B_sum", 0)]
    writes = []
    for disp, (w, w64) in ((1, (50, 40)), (2, (70, 70))):
        writes += [(disp, k, "TCC_EA0_WRREQ_sum", w), (disp, k, "TCC_EA0_WRREQ_64B_sum", w64),
                   (disp, k, "TCC_EA0_RDREQ_DRAM_32B_sum", 4 * 100), (disp, k, "TCC_EA0_WRREQ_WRITE_DRAM_32B_sum", 8)]
    writes += [(9, cp, "TCC_EA0_WRREQ_sum", 16), (9, cp, "TCC_EA0_WRREQ_64B_sum", 16),
               (9, cp, "TCC_EA0_RDREQ_DRAM_32B_sum", 32), (9, cp, "TCC_EA0_WRREQ_WRITE_DRAM_32B_sum", 32)]
    l2 = []
    for disp in (1, 2, 9):
        kn = cp if disp == 9 else k
        l2 += [(disp, kn, "TCC_REQ_sum", 10), (disp, kn, "TCC_HIT_sum", 3), (disp, kn, "TCC_MISS_sum", 7),
               (disp, kn, "TCC_READ_sum", 9)]
    dirs = [str(tmp_path / n) for n in ("reads", "writes", "l2")]
    for d, rows in zip(dirs, (reads, writes, l2)):
        _write_pass(d, rows)
    text = bench.counter_summary(dirs, "zipf-2m", ["cmd one", "cmd two"])
    kv = dict(l.split(" = ", 1) for l in text.splitlines() if " = " in l and not l.startswith("#"))
    rd = ((128 * 100 + 64 * 10 + 32 * 4) + (128 * 300 + 64 * 30)) / 2
    wr = ((64 * 40 + 32 * 10) + 64 * 70) / 2
    assert float(kv["bf16.read_bytes_per_launch"]) == pytest.approx(rd)
    assert float(kv["bf16.write_bytes_per_launch"]) == pytest.approx(wr)
    assert float(kv["bf16.traffic_bytes_per_launch"]) == pytest.approx(rd + wr)
    assert float(kv["bf16.l2_hit_rate"]) == pytest.approx(0.3)
    assert float(kv["copy.read_bytes_per_launch"]) == 1024 and float(kv["copy.write_bytes_per_launch"]) == 1024
    assert kv["kernel_source_sha256"] == bench.kernel_source_digest()
    assert "#   cmd one" in text


def test_trace_summary_table(tmp_path):
    import csv
    import bench
    d = tmp_path / "trace"
    d.mkdir()
    with open(d / "x_kernel_stats.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs",
                                          "MaxNs", "StdDev"])
        w.writeheader()
        w.writerow(dict(Name="k_small", Calls=10, TotalDurationNs=1000, AverageNs=100, Percentage=10, MinNs=90,
                        MaxNs=110, StdDev=1))
        w.writerow(dict(Name="k_big", Calls=3, TotalDurationNs=9000, AverageNs=3000, Percentage=90, MinNs=2900,
                        MaxNs=3100, StdDev=1))
    text = bench.trace_summary([str(d)], "t", ["cmd"])
    lines = [l for l in text.splitlines() if l.startswith("| `")]
    assert lines[0].startswith("| `k_big` | 3 | 3.0 |") and lines[0].endswith("| 90.0 |")
    assert lines[1].startswith("| `k_small` | 10 | 0.1 |")
    assert "    cmd" in text and bench.kernel_source_digest() in text
    ex = bench.trace_summary([str(d)], "t", ["cmd"], exclude="big")
    rows = [l for l in ex.splitlines() if l.startswith("| `")]
    assert len(rows) == 1 and rows[0].startswith("| `k_small` | 10 |") and rows[0].endswith("| 100.0 |")
