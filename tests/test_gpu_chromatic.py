"""Parity of the chromatic-aberration composite (wt_resolve_chromatic, through the C ABI) with the FP64 oracle.

The accumulated colour and absorbance, the background image and the refraction offsets are seeded inputs handed
to both sides as the same float32 values; the composite must agree within 1e-4 absolute.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import assert_close_abs, device_frags, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_00094_amd as wt
    wt.load_library()


def _inputs(seed, W, H, channels, max_off):
    rng = np.random.default_rng(seed)
    P = W * H
    S = rng.random((P, 3), dtype=np.float32)
    suma = rng.uniform(0.0, 3.0, (P, channels)).astype(np.float32)
    # a smooth field plus texel noise: high contrast between neighbours, as at refracted edges
    y, x = np.divmod(np.arange(P), W)
    smooth = 0.5 + 0.4 * np.sin(x[:, None] * np.array([0.05, 0.09, 0.13]) + y[:, None] * np.array([0.07, 0.03, 0.11]))
    bg = (0.7 * smooth + 0.3 * rng.random((P, 3))).astype(np.float32)
    off = rng.uniform(-max_off, max_off, (P, 2)).astype(np.float32)
    return S, suma, bg, off


def _accum(S, suma, channels):
    P = S.shape[0]
    if channels == 1:
        return np.concatenate([S, suma], axis=1).astype(np.float32)
    acc = np.zeros((P, 8), np.float32)
    acc[:, :3] = S
    acc[:, 4:7] = suma
    return acc


def _gpu_chromatic(W, H, channels, acc, bg, off, disp, taps):
    import torch
    import paper_2201_00094_amd as wt
    spec = wt.FrameSpec(W, H, 3, channels)
    out = wt.resolve_chromatic(spec, torch.from_numpy(acc).cuda(), torch.from_numpy(bg).cuda(),
                               torch.from_numpy(off).cuda(), dispersion=disp, taps=taps)
    torch.cuda.synchronize()
    return out.cpu().double().numpy()


@pytest.mark.parametrize("channels,taps,disp,max_off", [(1, 5, 0.5, 25.0), (3, 5, 0.5, 25.0), (1, 3, 1.3, 8.0),
                                                        (3, 9, 0.0, 40.0), (1, 7, 2.0, 300.0), (3, 63, 0.25, 0.0)])
def test_chromatic_parity(orc, channels, taps, disp, max_off):
    """97 x 61 pixels (a partial last workgroup), offsets reaching past every edge."""
    W, H = 97, 61
    say("case chromatic", channels, taps, disp, max_off)
    S, suma, bg, off = _inputs(80 + taps, W, H, channels, max_off)
    g = _gpu_chromatic(W, H, channels, _accum(S, suma, channels), bg, off, disp, taps)
    o = orc.resolve_chromatic(W, H, S, suma, bg, off, dispersion=disp, taps=taps, channels=channels)
    err = assert_close_abs(g, o, 1e-4, what="chromatic out")
    say("  max |out - oracle| = %.2e" % err)


@pytest.mark.parametrize("W,H", [(1920, 1080), (3840, 2160)])
def test_chromatic_full_frame(orc, W, H):
    """Whole 1080p and 4K frames (three channels, five taps), every pixel against the oracle."""
    say("case chromatic full frame", W, H)
    S, suma, bg, off = _inputs(W, W, H, 3, 20.0)
    g = _gpu_chromatic(W, H, 3, _accum(S, suma, 3), bg, off, 0.5, 5)
    o = orc.resolve_chromatic(W, H, S, suma, bg, off, dispersion=0.5, taps=5, channels=3)
    err = assert_close_abs(g, o, 1e-4, what="chromatic out")
    say("  max |out - oracle| = %.2e" % err)


def test_chromatic_after_build_and_evaluate(orc):
    """End to end on a glass frame: build + evaluate on the GPU, then the chromatic composite of their accumulation,
    against the oracle's resolve followed by its chromatic composite."""
    import torch
    import paper_2201_00094_amd as wt
    f = synth.frame_c3(seed=90, width=75, height=44, rank=3, particles=6.0)
    say("case chromatic end to end F", f.count)
    spec = wt.FrameSpec(f.width, f.height, 3, 3)
    fr = device_frags(f)
    ws = wt.Workspace(spec, f.count)
    coeffs = spec.new_coeffs()
    accum = spec.new_accum()
    wt.build(spec, fr, coeffs, ws)
    wt.evaluate(spec, fr, coeffs, accum, ws)
    _, _, bg, off = _inputs(91, f.width, f.height, 3, 12.0)
    out = wt.resolve_chromatic(spec, accum, torch.from_numpy(bg).cuda(), torch.from_numpy(off).cuda(),
                               dispersion=0.8, taps=5)
    torch.cuda.synchronize()
    r = orc.resolve(f.width, f.height, 3, f.pixel, f.depth, f.alpha, f.rgb, channels=3, want=("accum", "suma"))
    o = orc.resolve_chromatic(f.width, f.height, r["accum"], r["suma"], bg, off, dispersion=0.8, taps=5, channels=3)
    assert_close_abs(out.cpu().double().numpy(), o, 1e-4, what="end-to-end chromatic out")
