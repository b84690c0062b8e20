"""The largest inputs a call takes. WT_MAX_FRAGMENTS = 2^32 - 2^20 fragments over the 1920x1080 rank-3 frame in
the benchmark's launch configuration (about 2,071 fragments per pixel: 103 GB of input and a 120 GB workspace), so
the 32-bit record indices and segment offsets reach the top of their range; the largest frame, 65535 x 65537 =
2^32 - 1 pixels; and three channels past 2^31 fragments through the two-level binning. Pixels are checked whole
against the oracle."""
import numpy as np
import pytest

import synth
from gpu_helpers import assert_close_abs, assert_coeffs, say

pytestmark = pytest.mark.gpu


def test_stream_at_the_fragment_limit(orc):
    """No drops; signs of every stored coefficient; the pixels of the first and last fragment, both sides of the
    ragged edge (the pixels before it hold one fragment more) and random ones, each with its whole list of about
    2,071 fragments, against the oracle. Skipped where the device has no room for the 224 GB this takes."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_00094_amd as wt
    from paper_2201_00094_amd import _lib
    W, H, F = 1920, 1080, _lib.WT_MAX_FRAGMENTS
    P = W * H
    spec = wt.FrameSpec(W, H, 3, 1, "f32")
    need = 24 * F + wt.workspace_bytes(spec, F) + (64 + 12) * P + (8 << 30)
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip("needs %.0f GB of device memory, %.0f GB free" % (need / 1e9, free / 1e9))
    say("case stream at the fragment limit: F", F)
    pixel, depth, alpha, rgb, A, B = synth.scrambled_stream(7, W, H, F)
    fr = wt.Fragments(pixel, depth, alpha, rgb)
    ws = wt.Workspace(spec, F)
    coeffs = spec.new_coeffs()
    bg = (0.25, 0.2, 0.15)
    out = wt.render(spec, fr, bg, ws, coeffs=coeffs)
    torch.cuda.synchronize()
    assert wt.dropped_count(ws) == 0
    c = coeffs[:, 0, :]
    assert bool((c[:, 0] >= 0).all()) and bool((c[:, 1:] <= 0).all())
    # the pixel of fragment i is (A i + B) mod P; pixel p holds the fragments i_p + k P
    rag = F % P
    rng = np.random.default_rng(7)
    firsts = np.unique(np.concatenate([[0, P - 1, rag - 1, rag, (F - 1) % P], rng.choice(P, 27, replace=False)]))
    sel = (A * firsts + B) % P
    parts = []
    for j, ip in enumerate(firsts):
        idx = torch.arange(int(ip), F, P, device=pixel.device)
        parts.append((np.full(idx.numel(), j, np.uint32), depth[idx].cpu().numpy(), alpha[idx].cpu().numpy(),
                      rgb[idx].cpu().numpy()))
    assert sum(p[0].size for p in parts) == sum(F // P + (ip < rag) for ip in firsts)
    mp, md, ma, mc = (np.concatenate([p[k] for p in parts]) for k in range(4))
    o = orc.resolve(len(parts), 1, 3, mp, md, ma, mc, bg=bg, want=("coeffs", "out"))
    sel_t = torch.from_numpy(sel).to(pixel.device)
    assert_coeffs(coeffs[sel_t].cpu().double().numpy(), o["coeffs"])
    err = assert_close_abs(out[sel_t].cpu().double().numpy(), o["out"], 1e-4)
    say("  %d pixels with %d-%d fragments each: max |out - oracle| %.2e" %
        (len(parts), min(p[0].size for p in parts), max(p[0].size for p in parts), err))
    del pixel, depth, alpha, rgb, fr, ws, coeffs, out, c
    torch.cuda.empty_cache()


def test_frame_at_the_pixel_limit(orc):
    """65535 x 65537 = 2^32 - 1 pixels at rank 0 (4.2 M tiles, binned with one global atomic per fragment) with
    fragments on about 2,000 pixels, among them the first and the last pixel, the ends of the first and last rows
    and both sides of 2^31: those pixels against the oracle, and every other pixel of the frame shows the
    background over zero coefficients. Skipped where the device has no room for the 103 GB this takes."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_00094_amd as wt
    W, H = 65535, 65537
    P = W * H
    spec = wt.FrameSpec(W, H, 0, 1, "f32")
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    need = (8 + 12 + 3) * P + (4 << 30)
    if free < need:
        pytest.skip("needs %.0f GB of device memory, %.0f GB free" % (need / 1e9, free / 1e9))
    rng = np.random.default_rng(11)
    special = [0, 1, W - 1, W, (1 << 31) - 1, 1 << 31, (1 << 31) + 1, P - W, P - 2, P - 1]
    pix = np.unique(np.concatenate([special, rng.integers(0, P, 2000)]))
    pixel, depth, alpha, rgb = synth.sparse_stream(11, W, H, pix)
    say("case frame at the pixel limit: P", P, "F", pixel.size)
    fr = wt.Fragments.from_numpy(pixel, depth, alpha, rgb)
    ws = wt.Workspace(spec, pixel.size)
    coeffs = spec.new_coeffs()
    bg = (0.3, 0.5, 0.7)
    out = wt.render(spec, fr, bg, ws, coeffs=coeffs)
    torch.cuda.synchronize()
    assert wt.dropped_count(ws) == 0
    sel_t = torch.from_numpy(pix.astype(np.int64)).cuda()
    go = out[sel_t].cpu().double().numpy()
    gc = coeffs[sel_t].cpu().double().numpy()
    # the oracle over the same fragments with the listed pixels renumbered 0..n-1
    o = orc.resolve(pix.size, 1, 0, np.searchsorted(pix, pixel).astype(np.uint32), depth, alpha, rgb, bg=bg,
                    want=("coeffs", "out"))
    assert_coeffs(gc, o["coeffs"])
    err = assert_close_abs(go, o["out"], 1e-4)
    # every other pixel: the background, over zero coefficients
    bg_t = torch.tensor(bg, dtype=torch.float32, device="cuda")
    out[sel_t] = bg_t
    coeffs[sel_t] = 0
    assert bool((out == bg_t).all()), "a pixel without fragments does not show the background"
    assert bool((coeffs == 0).all()), "a pixel without fragments has a non-zero coefficient"
    say("  %d pixels against the oracle: max |out - oracle| %.2e; the other %d show the background" %
        (pix.size, err, P - pix.size))
    del fr, ws, coeffs, out
    torch.cuda.empty_cache()


def test_three_channel_stream_past_2_31_fragments(orc):
    """Three visibility channels, 2^31 + 12,345 fragments over the 1920x1080 rank-3 frame: 8,160 tiles of 256
    pixels, so the stream takes the two-level binning (super-tiles, then the split into tiles), whose record
    indices and offsets run past 2^31 at both levels. No drops, and about 40 pixels with their whole lists of
    about 1,036 fragments against the oracle. Skipped where the device has no room for the 231 GB this takes."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_00094_amd as wt
    W, H, F = 1920, 1080, (1 << 31) + 12345
    P = W * H
    spec = wt.FrameSpec(W, H, 3, 3, "f32")
    need = 32 * F + wt.workspace_bytes(spec, F) + (3 * 16 * 4 + 12) * P + (8 << 30)
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip("needs %.0f GB of device memory, %.0f GB free" % (need / 1e9, free / 1e9))
    say("case three channels past 2^31: F", F)
    pixel, depth, alpha, rgb, A, B = synth.scrambled_stream(9, W, H, F, channels=3)
    torch.cuda.empty_cache()  # the generator's temporaries
    fr = wt.Fragments(pixel, depth, alpha, rgb)
    ws = wt.Workspace(spec, F)
    coeffs = spec.new_coeffs()
    bg = (0.1, 0.2, 0.3)
    out = wt.render(spec, fr, bg, ws, coeffs=coeffs)
    torch.cuda.synchronize()
    assert wt.dropped_count(ws) == 0
    assert bool((coeffs[:, :, 0] >= 0).all()) and bool((coeffs[:, :, 1:] <= 0).all())
    rag = F % P
    rng = np.random.default_rng(9)
    firsts = np.unique(np.concatenate([[0, P - 1, rag - 1, rag, (F - 1) % P], rng.choice(P, 35, replace=False)]))
    sel = (A * firsts + B) % P
    parts = []
    for j, ip in enumerate(firsts):
        idx = torch.arange(int(ip), F, P, device=pixel.device)
        parts.append((np.full(idx.numel(), j, np.uint32), depth[idx].cpu().numpy(), alpha[idx].cpu().numpy(),
                      rgb[idx].cpu().numpy()))
    mp, md, ma, mc = (np.concatenate([p[k] for p in parts]) for k in range(4))
    o = orc.resolve(len(parts), 1, 3, mp, md, ma, mc, bg=bg, channels=3, want=("coeffs", "out"))
    sel_t = torch.from_numpy(sel).to(pixel.device)
    assert_coeffs(coeffs[sel_t].cpu().double().numpy(), o["coeffs"])
    err = assert_close_abs(out[sel_t].cpu().double().numpy(), o["out"], 1e-4)
    say("  %d pixels with %d-%d fragments each: max |out - oracle| %.2e" %
        (len(parts), min(p[0].size for p in parts), max(p[0].size for p in parts), err))
    del pixel, depth, alpha, rgb, fr, ws, coeffs, out
    torch.cuda.empty_cache()

