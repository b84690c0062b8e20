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


def _round_inputs():
    """FP64 values that exercise the FP16 and BF16 rounding: random magnitudes over both formats' ranges, the
    midpoints between neighbouring values of each format and the FP64 values one step either side of them, the
    subnormal ranges, the overflow edges, signed zeros, infinities and NaN."""
    import numpy as np
    rng = np.random.default_rng(5)
    vals = [rng.uniform(-1, 1, 4000) * np.exp2(rng.uniform(-30, 17, 4000)),
            rng.uniform(-1, 1, 2000) * np.exp2(rng.uniform(-140, -110, 2000))]
    h = np.arange(0, 0x7c00, 7, dtype=np.uint16).view(np.float16).astype(np.float64)
    hn = np.nextafter(h.astype(np.float16), np.float16(np.inf)).astype(np.float64)
    mid16 = (h + hn) / 2
    b = (np.arange(0, 0x7f80, 5, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)
    bn = ((np.arange(0, 0x7f80, 5, dtype=np.uint32) + 1) << 16).view(np.float32).astype(np.float64)
    mid_b = (b + bn) / 2
    for m in (mid16, mid_b):
        vals += [m, np.nextafter(m, np.inf), np.nextafter(m, -np.inf), -m]
    # midpoints moved by less than half an FP32 step, where an intermediate FP32 rounding lands on the midpoint
    for m in (mid16, mid_b):
        vals += [m * (1 + 2.0 ** -30), m * (1 - 2.0 ** -30), -m * (1 + 2.0 ** -40)]
    vals.append(np.array([0.0, -0.0, 65504.0, 65519.99, 65520.0, 65536.0, 2.0 ** -24, 2.0 ** -25, 2.0 ** -26,
                          3 * 2.0 ** -26, 2.0 ** -14, 1e300, -1e300, 5e-324, 3.3e38, 3.39e38, 3.402823e38, 3.5e38,
                          -3.5e38, 2.0 ** -149, 2.0 ** -150, 3 * 2.0 ** -151, 2.0 ** -133, 1.5 * 2.0 ** -133,
                          np.inf, -np.inf, np.nan]))
    return np.concatenate(vals)


def _bf16_nearest(v, table):
    """Nearest BF16 value to v (ties to the even bit pattern) by search over every finite positive BF16 value,
    with the distances compared exactly (fractions); inf beyond the overflow threshold."""
    import bisect
    import math
    from fractions import Fraction
    a = abs(v)
    sign = 0x8000 if math.copysign(1.0, v) < 0 else 0
    top = Fraction(table[-1]) + Fraction(2) ** (127 - 8)  # largest finite + half its spacing
    if math.isinf(a) or Fraction(a) >= top:
        return 0x7f80 | sign
    i = bisect.bisect_left(table, a)
    cands = [k for k in (i - 1, i) if 0 <= k < len(table)]
    best = min(cands, key=lambda k: (abs(Fraction(table[k]) - Fraction(a)), k & 1))
    return best | sign


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_round_f64_to_f16_bf16(tmp_path):
    """The library rounds FP64 sums to FP16 / BF16 storage once (FP32 rounded to odd, then to nearest): bit-equal
    to NumPy's binary16 conversion of the FP64 value, and to the exactly nearest BF16 value (ties to even) found by
    search, also for values one FP64 step off a midpoint of either format, which a plain FP64 -> FP32 -> narrow
    conversion would round the wrong way."""
    import numpy as np
    exe = tmp_path / "round_check"
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2201_00094_amd", "csrc"),
                           os.path.join(ROOT, "tests", "host", "round_check.cpp"), "-o", str(exe)],
                          stderr=subprocess.DEVNULL)
    x = _round_inputs()
    inp = "\n".join("%016x" % u for u in x.view(np.uint64)) + "\n"
    res = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0
    got = np.array([[int(w, 16) for w in ln.split()] for ln in res.stdout.split("\n") if ln])
    assert got.shape == (x.size, 2)
    with np.errstate(over="ignore"):
        ref16 = x.astype(np.float16).view(np.uint16)
    nan = np.isnan(x)
    assert (got[~nan, 0] == ref16[~nan]).all()
    assert ((got[nan, 0] & 0x7c00) == 0x7c00).all() and ((got[nan, 0] & 0x3ff) != 0).all()
    table = list(((np.arange(0, 0x7f80, dtype=np.uint32) << 16).view(np.float32)).astype(np.float64))
    for v, g in zip(x[~nan], got[~nan, 1]):
        assert g == _bf16_nearest(float(v), table), (float(v), hex(g))
    assert ((got[nan, 1] & 0x7f80) == 0x7f80).all() and ((got[nan, 1] & 0x7f) != 0).all()


def _e5_inputs():
    """FP32 triples that exercise the shared-exponent packing: random magnitudes over the format's range and beyond,
    triples whose largest value rounds up to the next exponent, values exactly halfway between two mantissas (and
    one FP32 step either side), the smallest exponent's range and FP32 subnormals, the clamp at 65408, zeros,
    negatives, infinities and NaN."""
    import numpy as np
    rng = np.random.default_rng(11)
    n = 6000
    mag = np.exp2(rng.uniform(-30, 18, (n, 3))) * rng.uniform(0.5, 1.0, (n, 3))
    spread = np.exp2(rng.uniform(-30, 18, (n, 1))) * np.exp2(-rng.uniform(0, 12, (n, 3)))
    t = [mag, spread]
    e = rng.integers(-16, 16, 2000)
    m = rng.integers(0, 512, (2000, 3)).astype(np.float64)
    half = (m + 0.5) * np.exp2(e[:, None] - 8.0)
    t += [half, np.nextafter(half.astype(np.float32), np.float32(np.inf)).astype(np.float64),
          np.nextafter(half.astype(np.float32), np.float32(0)).astype(np.float64)]
    top = (511.5 + rng.uniform(-0.01, 0.01, (2000, 1))) * np.exp2(e[:, None] - 8.0) * np.array([1.0, 0.3, 0.01])
    t.append(top)
    t.append(rng.uniform(0, 2.0 ** -16, (1000, 3)))
    t.append(rng.uniform(0, 1, (500, 3)) * 2.0 ** -130)
    sign = np.where(rng.random((3000, 3)) < 0.3, -1.0, 1.0)
    t.append(sign * np.exp2(rng.uniform(-20, 17, (3000, 3))))
    t.append(np.array([[0.0, 0.0, 0.0], [-0.0, 1.0, 2.0], [65408.0, 1.0, 0.5], [65409.0, 65535.0, 1e30],
                       [np.inf, 1.0, 2.0], [-np.inf, 3.0, np.nan], [np.nan, np.nan, np.nan], [2.0 ** -16, 0, 0],
                       [2.0 ** -16 * 511.5 / 512, 0, 0], [511.5 * 2.0 ** -24, 1e-45, 0], [1.0, 1.0, 1.0]]))
    return np.concatenate(t).astype(np.float32)


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_e5_pack_matches_the_oracle(tmp_path):
    """The kernels' E5B9G9R9 packing (FP32 scaling, FP64 round-half-up, exponent from the FP32 bit pattern) gives,
    word for word, the oracle's packing (FP64 scaling, exponent by frexp), over the format's whole range and its
    rounding and clamping edges."""
    import numpy as np
    import oracle
    exe = tmp_path / "e5_check"
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2201_00094_amd", "csrc"),
                           os.path.join(ROOT, "tests", "host", "e5_check.cpp"), "-o", str(exe)],
                          stderr=subprocess.DEVNULL)
    x = _e5_inputs()
    bits = x.view(np.uint32)
    inp = "\n".join("%08x %08x %08x" % tuple(r) for r in bits) + "\n"
    res = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0
    got = [int(w, 16) for w in res.stdout.split()]
    assert len(got) == len(x)
    want = [oracle.pack_e5b9g9r9(*(float(v) for v in r)) for r in x]
    bad = [(tuple(x[i]), hex(got[i]), hex(want[i])) for i in range(len(x)) if got[i] != want[i]]
    assert not bad, bad[:5]


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_workspace_stamps_tell_layouts_and_streams_apart(tmp_path):
    """The stamps the binning leaves in the workspace header: every description a caller could confuse with the
    one a stream was binned under (rank, frame size, channels, depth bounds, one-pass tiles, gradient records,
    workspace size) stamps differently, and a count is tied to the stream it counted (size and array addresses)."""
    exe = tmp_path / "stamp_check"
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2201_00094_amd", "csrc"),
                           os.path.join(ROOT, "tests", "host", "stamp_check.cpp"), "-o", str(exe)],
                          stderr=subprocess.DEVNULL)
    res = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout
    assert "bad 0" in res.stdout
