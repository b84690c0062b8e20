"""Host-side logic of the library that does not need a GPU, compiled for the host from the library's own header:
the per-frame fast division used to turn pixel ids into tile coordinates, checked against the hardware divide, and
the absorbance -ln(1 - alpha), checked against log1p."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_fastdiv_matches_hardware_divide(tmp_path):
    exe = tmp_path / "fastdiv_check"
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2201_00094_amd", "csrc"),
                           os.path.join(ROOT, "tests", "host", "fastdiv_check.cpp"), "-o", str(exe)],
                          stderr=subprocess.DEVNULL)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout
    assert "bad 0" in res.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_neg_log1m_matches_log1p(tmp_path):
    """The library's own -ln(1 - alpha), the absorbance the binning pass stores, is within 4 ulp of log1p."""
    exe = tmp_path / "neglog_check"
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2201_00094_amd", "csrc"),
                           os.path.join(ROOT, "tests", "host", "neglog_check.cpp"), "-o", str(exe)],
                          stderr=subprocess.DEVNULL)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout
    assert "series: max" in res.stdout
