"""Parity of the one-pass render against the previous frame (wt_render_temporal, through the C ABI) with the
FP64 oracle's shade_prev.

The previous frame's coefficients handed to the GPU are the oracle's (rounded to the storage type, which is what a
stored buffer holds), and the oracle shades with exactly those stored values. Contract as for the two-pass path:
composite within 1e-4 absolute; this frame's coefficients within 1e-5 relative (FP32), one storage step (FP16,
BF16) or one shared-exponent step (E5B9G9R9) of the oracle at that storage.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import STORAGE_ATOL, assert_close_abs, assert_coeffs, device_frags, e5_decode, say

pytestmark = pytest.mark.gpu

STEP = {"f32": 0.0, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_00094_amd as wt
    wt.load_library()


def _frame(channels, seed, width, height, rank, mean=8.0):
    if channels == 1:
        return synth.frame_c1(seed=seed, width=width, height=height, rank=rank, mean=mean)
    return synth.frame_c3(seed=seed, width=width, height=height, rank=rank, particles=mean)


def _stored(orc, coeffs, dtype):
    """Oracle coefficients [P, C, M] at storage precision -> (values as stored, FP64; device tensor)."""
    import torch
    if dtype == "f32":
        vals = coeffs.astype(np.float32).astype(np.float64)
        return vals, torch.from_numpy(vals.astype(np.float32)).cuda()
    if dtype == "f16":
        return coeffs, torch.from_numpy(coeffs.astype(np.float16)).cuda()
    if dtype == "bf16":
        t = torch.from_numpy(coeffs).to(torch.bfloat16)
        assert np.array_equal(t.double().numpy(), coeffs)  # already bf16 values: the conversion is exact
        return coeffs, t.cuda()
    P, C, M = coeffs.shape
    words = np.array([[orc.pack_e5b9g9r9(*np.abs(coeffs[p, :, m])) for m in range(M)] for p in range(P)],
                     dtype=np.uint32)
    assert np.array_equal(e5_decode(orc, words), coeffs)  # already E5B9G9R9 values: the packing is exact
    return coeffs, torch.from_numpy(words.view(np.int32)).cuda()


def _spec(f, dtype, rank=None):
    import paper_2201_00094_amd as wt
    return wt.FrameSpec(f.width, f.height, f.rank if rank is None else rank, f.channels, dtype, temporal=True)


def _gpu_temporal(f, dtype, prev_dev, prev_pixel=None, in_place=False):
    import torch
    import paper_2201_00094_amd as wt
    spec = _spec(f, dtype)
    fr = device_frags(f)
    ws = wt.Workspace(spec, max(1, f.count))
    if in_place:
        coeffs = prev_dev
    else:
        coeffs = spec.new_coeffs()
    pp = None if prev_pixel is None else torch.from_numpy(prev_pixel.astype(np.uint32).view(np.int32)).cuda()
    out = wt.render_temporal(spec, fr, f.bg, ws, prev=prev_dev, coeffs=coeffs, prev_pixel=pp)
    torch.cuda.synchronize()
    res = {"out": out.cpu().double().numpy(), "dropped": wt.dropped_count(ws)}
    if dtype == "e5b9g9r9":
        res["words"] = coeffs.cpu().numpy().view(np.uint32)
    else:
        res["coeffs"] = coeffs.float().cpu().double().numpy()
    return res


def _check_coeffs(orc, g, f, dtype):
    o = orc.resolve(f.width, f.height, f.rank, f.pixel, f.depth, f.alpha, f.rgb, channels=f.channels,
                    want=("coeffs",), storage="exact" if dtype == "f32" else dtype)["coeffs"]
    if dtype == "e5b9g9r9":
        ex = orc.resolve(f.width, f.height, f.rank, f.pixel, f.depth, f.alpha, f.rgb, channels=3,
                         want=("coeffs",))["coeffs"]
        tmax = np.abs(ex).max(axis=1, keepdims=True)
        assert np.all(np.abs(e5_decode(orc, g["words"]) - o) <= tmax / 255.0 * (1 + 1e-6) + 1e-30)
    else:
        assert_coeffs(g["coeffs"], o, rel=2 * STEP[dtype] + 1e-5, what=dtype + " coeffs", atol=STORAGE_ATOL[dtype])


@pytest.mark.parametrize("channels,rank,dtype", [(1, 3, "f32"), (1, 0, "f32"), (1, 4, "f16"), (1, 2, "bf16"),
                                                 (3, 3, "bf16"), (3, 4, "f32"), (3, 3, "e5b9g9r9"),
                                                 (3, 4, "e5b9g9r9")])
def test_temporal_parity(orc, channels, rank, dtype):
    """70 x 45 pixels (partial tiles on two edges): frame t shaded with frame t-1's stored coefficients."""
    prev_f = _frame(channels, 30 + rank, 70, 45, rank)
    f = _frame(channels, 130 + rank, 70, 45, rank)
    say("case temporal", channels, rank, dtype, "F", f.count)
    po = orc.resolve(prev_f.width, prev_f.height, rank, prev_f.pixel, prev_f.depth, prev_f.alpha, prev_f.rgb,
                     channels=channels, want=("coeffs",), storage="exact" if dtype == "f32" else dtype)["coeffs"]
    vals, dev = _stored(orc, po, dtype)
    g = _gpu_temporal(f, dtype, dev)
    o = orc.shade_prev(f.width, f.height, rank, f.pixel, f.depth, f.alpha, f.rgb, prev=vals, bg=f.bg,
                       channels=channels, want=("out",))
    assert g["dropped"] == 0
    err = assert_close_abs(g["out"], o["out"], 1e-4, what="temporal out")
    say("  max |out - oracle| = %.2e" % err)
    _check_coeffs(orc, g, f, dtype)


@pytest.mark.parametrize("channels", [1, 3])
def test_temporal_reprojection_map_and_no_history(orc, channels):
    """A motion of (+5, -3) pixels: pixel (x, y) reads the previous buffer at (x - 5, y + 3); pixels whose source
    lies off screen have no history. Then a first frame without any previous buffer."""
    W, H, rank = 53, 41, 3
    prev_f = _frame(channels, 40, W, H, rank)
    f = _frame(channels, 41, W, H, rank)
    say("case temporal map channels", channels)
    po = orc.resolve(W, H, rank, prev_f.pixel, prev_f.depth, prev_f.alpha, prev_f.rgb, channels=channels,
                     want=("coeffs",))["coeffs"]
    vals, dev = _stored(orc, po, "f32")
    y, x = np.divmod(np.arange(W * H), W)
    sx, sy = x - 5, y + 3
    inside = (sx >= 0) & (sx < W) & (sy >= 0) & (sy < H)
    pmap = np.where(inside, sy * W + sx, 0xFFFFFFFF).astype(np.uint32)
    g = _gpu_temporal(f, "f32", dev, prev_pixel=pmap)
    o = orc.shade_prev(W, H, rank, f.pixel, f.depth, f.alpha, f.rgb, prev=vals, prev_pixel=pmap, bg=f.bg,
                       channels=channels, want=("out",))
    assert_close_abs(g["out"], o["out"], 1e-4, what="mapped out")
    _check_coeffs(orc, g, f, "f32")
    g0 = _gpu_temporal(f, "f32", None)
    o0 = orc.shade_prev(W, H, rank, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg, channels=channels, want=("out",))
    assert_close_abs(g0["out"], o0["out"], 1e-4, what="first-frame out")
    # this frame's coefficients do not depend on history
    np.testing.assert_allclose(g0["coeffs"], g["coeffs"], rtol=1e-6, atol=0)


@pytest.mark.parametrize("dtype", ["f32", "e5b9g9r9"])
def test_temporal_in_place(orc, dtype):
    """prev and coeffs one buffer (identity map): the same result as two buffers."""
    channels = 3 if dtype == "e5b9g9r9" else 1
    prev_f = _frame(channels, 50, 64, 40, 3)
    f = _frame(channels, 51, 64, 40, 3)
    say("case temporal in place", dtype)
    po = orc.resolve(64, 40, 3, prev_f.pixel, prev_f.depth, prev_f.alpha, prev_f.rgb, channels=channels,
                     want=("coeffs",), storage="exact" if dtype == "f32" else dtype)["coeffs"]
    vals, dev = _stored(orc, po, dtype)
    a = _gpu_temporal(f, dtype, dev.clone())
    b = _gpu_temporal(f, dtype, dev, in_place=True)
    # FP64 sums in another order may round to a neighbouring FP32 value: compare to within that
    if dtype == "e5b9g9r9":
        assert int((a["words"] != b["words"]).sum()) <= max(1, a["words"].size // 10000)
    else:
        np.testing.assert_allclose(a["coeffs"], b["coeffs"], rtol=1e-6, atol=0)
    np.testing.assert_allclose(a["out"], b["out"], rtol=0, atol=1e-6)
    _check_coeffs(orc, b, f, dtype)
    o = orc.shade_prev(64, 40, 3, f.pixel, f.depth, f.alpha, f.rgb, prev=vals, bg=f.bg, channels=channels,
                       want=("out",))
    assert_close_abs(b["out"], o["out"], 1e-4, what="in-place out")


def test_temporal_sequence_ping_pong(orc):
    """Four frames, the coefficient buffers swapped each frame on the GPU and in the oracle."""
    import torch
    import paper_2201_00094_amd as wt
    W, H, rank = 57, 38, 3
    frames = [_frame(1, 60 + t, W, H, rank) for t in range(4)]
    spec = _spec(frames[0], "f32")
    ws = wt.Workspace(spec, max(fr.count for fr in frames))
    bufs = [spec.new_coeffs(), spec.new_coeffs()]
    prev_o = None
    for t, f in enumerate(frames):
        say("case temporal sequence frame", t)
        out = wt.render_temporal(spec, device_frags(f), f.bg, ws, prev=bufs[1] if t else None, coeffs=bufs[0])
        torch.cuda.synchronize()
        o = orc.shade_prev(W, H, rank, f.pixel, f.depth, f.alpha, f.rgb, prev=prev_o, bg=f.bg, want=("out",))
        assert_close_abs(out.cpu().double().numpy(), o["out"], 1e-4, what="frame %d out" % t)
        co = orc.resolve(W, H, rank, f.pixel, f.depth, f.alpha, f.rgb, want=("coeffs",))["coeffs"]
        assert_coeffs(bufs[0].cpu().double().numpy(), co, what="frame %d coeffs" % t)
        prev_o = co.astype(np.float32).astype(np.float64)
        bufs.reverse()


def test_temporal_empty_frame(orc):
    import torch
    import paper_2201_00094_amd as wt
    f = synth.frame_c1(seed=70, width=33, height=17, mean=4.0)
    spec = _spec(f, "f32")
    ws = wt.Workspace(spec, 1)
    empty = wt.Fragments(torch.zeros(0, dtype=torch.int32, device="cuda"), torch.zeros(0, device="cuda"),
                         torch.zeros(0, device="cuda"), torch.zeros((0, 3), device="cuda"))
    prev = torch.full(spec.coeff_shape(), -0.25, device="cuda")
    coeffs = torch.full(spec.coeff_shape(), 7.0, device="cuda")
    out = wt.render_temporal(spec, empty, f.bg, ws, prev=prev, coeffs=coeffs)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), np.tile(np.array(f.bg, np.float32), (f.pixels, 1)))
    assert bool((coeffs == 0).all())


def test_temporal_static_smoke_1080p(orc):
    """The benchmark workload (1920 x 1080, Poisson(64 g) fragments/px, rank 3) in the one-pass configuration. A
    static scene: shaded against the two-pass render's own stored coefficients, every pixel matches the two-pass
    composite (the same stored coefficients, the same cells). Against the oracle: 1500 sampled pixels plus the 100
    densest, with the oracle's coefficients of those pixels as the previous buffer."""
    import torch
    import paper_2201_00094_amd as wt
    f = synth.frame_c2(seed=0, rank=3)
    say("case temporal static smoke 1080p F", f.count)
    fr = device_frags(f)
    spec2 = wt.FrameSpec(f.width, f.height, 3)
    ws2 = wt.Workspace(spec2, f.count)
    c2 = spec2.new_coeffs()
    out2 = wt.render(spec2, fr, f.bg, ws2, coeffs=c2)
    del ws2
    spec = _spec(f, "f32")
    ws = wt.Workspace(spec, f.count)
    c1 = spec.new_coeffs()
    out1 = wt.render_temporal(spec, fr, f.bg, ws, prev=c2, coeffs=c1)
    torch.cuda.synchronize()
    assert wt.dropped_count(ws) == 0
    d_out = float((out1 - out2).abs().max())
    d_c = float(((c1 - c2).abs() - 1e-5 * c2.abs()).max())
    say("  static scene: max |out1 - out2| = %.2e" % d_out)
    assert d_out <= 1e-5
    assert d_c <= 0.0
    cnt = np.bincount(f.pixel, minlength=f.pixels)
    rng = np.random.default_rng(3)
    sel = np.unique(np.concatenate([rng.choice(f.pixels, 1500, replace=False), np.argsort(cnt)[-100:]]))
    mask = np.zeros(f.pixels, bool)
    mask[sel] = True
    co = orc.resolve(f.width, f.height, 3, f.pixel, f.depth, f.alpha, f.rgb, mask=mask, want=("coeffs",))["coeffs"]
    vals, dev = _stored(orc, co, "f32")
    out3 = wt.render_temporal(spec, fr, f.bg, ws, prev=dev, coeffs=c1)
    torch.cuda.synchronize()
    o = orc.shade_prev(f.width, f.height, 3, f.pixel, f.depth, f.alpha, f.rgb, prev=vals, bg=f.bg, mask=mask,
                       want=("out",))
    err = assert_close_abs(out3.cpu().double().numpy(), o["out"], 1e-4, sel=sel)
    say("  max |out - oracle| on %d sampled pixels: %.2e" % (sel.size, err))
    assert_coeffs(c1.cpu().double().numpy(), co, sel=sel)
    del fr, ws, c1, c2, out1, out2, out3, dev
    torch.cuda.empty_cache()
