"""Host-side checks of bench.py (no GPU): the one-GPU guard and the byte models behind the roofline figures."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_byte_models():
    # one fragment, no pixels: the two passes read 12 + 24 bytes (one channel), 20 + 32 (three)
    assert bench.algorithmic_bytes(1, 0, 1, 64) == 36
    assert bench.algorithmic_bytes(1, 0, 3, 192) == 52
    # one pixel, no fragments: coefficients written and read, accumulation written and read, composite written
    assert bench.algorithmic_bytes(0, 1, 1, 64) == 2 * 64 + 2 * 16 + 12
    assert bench.algorithmic_bytes(0, 1, 3, 192) == 2 * 192 + 2 * 32 + 12
    # the fused tile kernel: the stream twice, the coefficients and composite once
    assert bench.render_kernel_bytes(1, 1, 1, 64) == 36 + 64 + 12
    # the scatter: read and write one record (24 B at one channel, 32 B at three)
    assert bench.scatter_kernel_bytes(1, 1) == 48 and bench.scatter_kernel_bytes(1, 3) == 64
    # the one-pass render: the stream once, previous coefficients read, this frame's written, composite
    assert bench.temporal_bytes(1, 1, 1, 64) == 24 + 2 * 64 + 12
    # the smoke frame's whole-path figure quoted in the design notes (132.7 M fragments, rank 3, FP32)
    assert bench.algorithmic_bytes(132_689_233, 1920 * 1080, 1, 64) == pytest.approx(5.13e9, rel=2e-3)


def test_traffic_is_keyed_to_the_sources():
    """A counter summary taken on other kernel sources is not reported."""
    assert len(bench.sources_digest()) == 64
    assert bench.measured_traffic("k_scatter_staged", "no_such_workload") is None


def test_roofline_is_the_path_bytes_over_the_dominant_kernel():
    """achieved = the path's algorithmic bytes per frame over the dominant kernel's mean launch time; frac = that
    over 8 TB/s. The smoke frame's 5.134 GB over a 1.705 ms scatter is 0.376 of peak, not the scatter's own
    48 B/fragment record model (0.47)."""
    F, P = 132_689_233, 1920 * 1080
    b_alg = bench.algorithmic_bytes(F, P, 1, 64)
    r = bench.roofline(b_alg, "k_scatter_staged", 1.705, None)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["achieved"] == pytest.approx(b_alg / 1.705e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["frac"] == pytest.approx(0.376, abs=2e-3)
    assert r["alg_bytes_per_launch"] == b_alg and r["avg_ms"] == 1.705 and r["traffic"] is None
    # per-fragment figure of the path: 38.7 B at rank 3, FP32
    assert b_alg / F == pytest.approx(38.7, abs=0.05)


def test_cpu_model_is_named():
    assert isinstance(bench.cpu_model(), str) and bench.cpu_model()


def test_overlap_summary_of_a_kernel_trace(tmp_path):
    """The serving overlap figures from a kernel trace: busy time is the union of kernel intervals, overlap the
    time kernels of two streams run together; torch's own kernels are left out."""
    import csv
    p = tmp_path / "kernel_trace.csv"
    rows = [("KERNEL_DISPATCH", 1, "void wt::k_render<1, float, true>(x)", 0, 100),
            ("KERNEL_DISPATCH", 2, "wt::k_scan(x)", 50, 150),
            ("KERNEL_DISPATCH", 1, "void wt::k_hist_lds<256>(x)", 200, 300),
            ("KERNEL_DISPATCH", 3, "void at::native::fill(x)", 0, 1000)]
    with open(p, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kind", "Stream_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writerows(rows)
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--mode", "overlap", "--trace", str(p)],
                         capture_output=True, text=True, timeout=120)
    import json
    r = json.loads(out.stdout)
    assert r["kernels"] == 3 and r["streams"] == 2 and r["max_streams_at_once"] == 2
    assert r["busy_ms"] == pytest.approx(250e-6) and r["two_or_more_streams_ms"] == pytest.approx(50e-6)
    assert r["kernels_overlapping_another_streams_kernel"] == 2
