"""The FP64 C oracle against its scalar pure-Python twin (oracle/ref_tiny.py) on tiny frames: the twin reaches the
coefficients from the cell means of the absorbance step function and the Haar analysis, where the oracle adds the
closed forms of section 2.3.1, so a slip in either (a term, a sign, an index, a level scale) shows as a
difference. Coefficients, composites and the exact A-buffer, one and three visibility channels, ranks 0 to 5,
with and without per-pixel depth bounds, and frames with edge values and dropped fragments."""
import numpy as np
import pytest

import oracle
import synth
from oracle import ref_tiny


def _compare(f, rank, channels, tight=False, orc=oracle):
    o = orc.resolve(f.width, f.height, rank, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg, channels=channels,
                       want=("coeffs", "out"), tight=tight)
    cf, out, dropped = ref_tiny.resolve(f.width, f.height, rank, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg,
                                        channels=channels, tight=tight)
    P = f.width * f.height
    twin_c = np.array([cf[p] for p in range(P)])
    twin_o = np.array([out[p] for p in range(P)])
    assert o["dropped"] == dropped
    scale = max(1.0, float(np.abs(o["coeffs"]).max()))
    np.testing.assert_allclose(twin_c, o["coeffs"], rtol=1e-12, atol=1e-13 * scale)
    np.testing.assert_allclose(twin_o, o["out"], rtol=0, atol=1e-12)
    if not tight:
        a = orc.abuffer(f.width, f.height, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg, channels=channels)
        ta, td = ref_tiny.abuffer(f.width, f.height, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg, channels=channels)
        assert td == a["dropped"]
        np.testing.assert_allclose(np.array([ta[p] for p in range(P)]), a["out"], rtol=0, atol=1e-12)


@pytest.mark.parametrize("rank", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("tight", [False, True])
def test_one_channel(rank, tight):
    f = synth.frame_c1(seed=100 + rank, width=7, height=5, rank=rank, mean=5.0)
    _compare(f, rank, 1, tight)


@pytest.mark.parametrize("rank", [1, 3, 4])
@pytest.mark.parametrize("tight", [False, True])
def test_three_channels(rank, tight):
    f = synth.frame_c3(seed=200 + rank, width=6, height=4, rank=rank, particles=4.0)
    _compare(f, rank, 3, tight)


def test_edge_values_and_drops():
    """Depths at and beyond both ends, equal depths, alphas at 0, 1 and beyond, NaN depth and alpha, pixel ids past
    the frame: clamped, tied or dropped the same way by both."""
    depth = np.array([0.0, 1.0, -0.5, 1.5, 0.25, 0.25, 0.5, np.nan, 0.3, 0.7, 0.125, 0.875, 0.6], dtype=np.float32)
    alpha = np.array([0.3, 0.4, 0.0, 1.0, 0.2, 0.2, 1.7, 0.5, np.nan, -0.2, 0.999, 0.05, 0.5], dtype=np.float32)
    pixel = np.array([0, 0, 1, 1, 2, 2, 3, 3, 0, 1, 2, 3, 99], dtype=np.uint32)
    rgb = np.linspace(0.1, 0.9, 3 * len(depth)).reshape(-1, 3).astype(np.float32)
    f = synth.Frame(2, 2, 3, 1, pixel, depth, alpha, rgb, (0.2, 0.3, 0.4), "edges")
    for rank in (0, 3, 4):
        _compare(f, rank, 1)
        _compare(f, rank, 1, tight=True)


# Slips planted in a copy of the C oracle (as in test_oracle_mutations.py): the comparison with the twin catches
# each, although the twin shares none of the oracle's code.
TWIN_MUTATIONS = [
    ("level scale left out", "coef[s + k] += half_pow2(n) * X;", "coef[s + k] += X;", 0),
    ("wavelet index one level off", "int k = (int)floor(s * x[i]);", "int k = (int)floor(s * x[i] * 0.5);", 0),
    ("scaling coefficient without its 1 - x factor", "coef[0] += a[i] * (1.0 - x[i]);", "coef[0] += a[i];", 0),
    ("interpolation from cell j instead of j - 1", "double lo = (j == 0) ? 0.0 : cells[j - 1];",
     "double lo = cells[j];", 0),
]


@pytest.mark.parametrize("what,old,new,occurrence", TWIN_MUTATIONS, ids=[m[0] for m in TWIN_MUTATIONS])
def test_twin_catches_planted_oracle_mistakes(tmp_path, what, old, new, occurrence):
    from test_oracle_mutations import _mutant
    mod = _mutant(tmp_path, old, new, occurrence)
    f = synth.frame_c1(seed=7, width=5, height=4, rank=3, mean=5.0)
    with pytest.raises(AssertionError):
        _compare(f, 3, 1, orc=mod)
