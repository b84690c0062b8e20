"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Contract: coefficients within 1e-5 relative per element (exact zeros stay zero); composite rgb within 1e-4
absolute; accumulations within 2e-5 relative. FP16/BF16 storage is compared with the oracle run at the same
storage precision (coefficients within one storage rounding step), and its error against the exact oracle is
reported.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import (STORAGE_ATOL, accum_to_oracle_layout, assert_close_abs, assert_coeffs, assert_within, e5_decode,
                         gpu_passes, gpu_render, oracle_frame, say, spec_of, storage_out_bound)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2201_00094_amd as wt
    wt.load_library()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_c1_render(orc, seed):
    f = synth.frame_c1(seed=seed)
    say("case c1 render seed", seed, "F", f.count)
    g = gpu_render(f)
    o = oracle_frame(orc, f)
    assert g["dropped"] == 0
    assert_coeffs(g["coeffs"], o["coeffs"])
    assert_close_abs(g["out"], o["out"], 1e-4)


def test_c1_three_passes(orc):
    f = synth.frame_c1(seed=3)
    say("case c1 build/evaluate/resolve")
    g = gpu_passes(f)
    o = oracle_frame(orc, f)
    assert_coeffs(g["coeffs"], o["coeffs"])
    S, sa = accum_to_oracle_layout(g["accum"], 1)
    np.testing.assert_allclose(S, o["accum"], rtol=2e-5, atol=1e-7)
    np.testing.assert_allclose(sa, o["suma"], rtol=2e-5, atol=1e-7)
    assert_close_abs(g["out"], o["out"], 1e-4)


@pytest.mark.parametrize("rank", [0, 1, 2, 3, 4, 5, 6])
def test_ragged_frame_all_ranks(orc, rank):
    """70 x 45 pixels: partial tiles on the right and bottom edges for every tile shape."""
    f = synth.frame_c1(seed=10 + rank, width=70, height=45, rank=rank, mean=6.0)
    say("case ragged 70x45 rank", rank)
    g = gpu_render(f)
    o = oracle_frame(orc, f)
    assert_coeffs(g["coeffs"], o["coeffs"])
    assert_close_abs(g["out"], o["out"], 1e-4)
    p = gpu_passes(f)
    assert_coeffs(p["coeffs"], o["coeffs"])
    assert_close_abs(p["out"], o["out"], 1e-4)


@pytest.mark.parametrize("rank", [8, 10])
def test_high_rank_tiny_frame(orc, rank):
    f = synth.frame_c1(seed=rank, width=9, height=7, rank=rank, mean=12.0)
    say("case high rank", rank)
    g = gpu_render(f)
    o = oracle_frame(orc, f)
    assert_coeffs(g["coeffs"], o["coeffs"])
    assert_close_abs(g["out"], o["out"], 1e-4)


@pytest.mark.parametrize("rank", [3, 4])
def test_three_channels(orc, rank):
    f = synth.frame_c3(seed=rank, width=50, height=37, rank=rank, particles=8.0)
    say("case three channels rank", rank, "F", f.count)
    g = gpu_render(f)
    o = oracle_frame(orc, f)
    assert_coeffs(g["coeffs"], o["coeffs"])
    assert_close_abs(g["out"], o["out"], 1e-4)
    p = gpu_passes(f)
    S, sa = accum_to_oracle_layout(p["accum"], 3)
    np.testing.assert_allclose(S, o["accum"], rtol=2e-5, atol=1e-7)
    np.testing.assert_allclose(sa, o["suma"], rtol=2e-5, atol=1e-7)
    assert_close_abs(p["out"], o["out"], 1e-4)


@pytest.mark.parametrize("dtype,step", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
@pytest.mark.parametrize("channels", [1, 3])
def test_reduced_precision_storage(orc, dtype, step, channels):
    f = synth.frame_c1(seed=7, width=61, height=33) if channels == 1 else \
        synth.frame_c3(seed=7, width=61, height=33, particles=8.0)
    say("case storage", dtype, "channels", channels)
    g = gpu_render(f, dtype=dtype)
    o = oracle_frame(orc, f, storage=dtype)
    ex = oracle_frame(orc, f, want=("out",))
    # one storage rounding step apart at most: FP32 accumulation can move a value across a rounding boundary
    assert_coeffs(g["coeffs"], o["coeffs"], rel=2 * step + 1e-5, what=dtype + " coeffs", atol=STORAGE_ATOL[dtype])
    tol = storage_out_bound(orc, f.rank, o["coeffs"], o["accum"], channels, 2 * step + 1e-5,
                            atol=STORAGE_ATOL[dtype])
    err_same, _ = assert_within(g["out"], o["out"], tol, what=dtype + " out vs oracle at storage precision")
    err_exact = float(np.abs(g["out"] - ex["out"]).max())
    say("  %s: max |out - oracle(%s)| = %.2e, max |out - oracle(exact)| = %.2e" % (dtype, dtype, err_same, err_exact))
    p = gpu_passes(f, dtype=dtype)
    np.testing.assert_allclose(p["out"], g["out"], rtol=0, atol=1e-3)


def _midpoint_picks(x32, xn, dtype):
    """Elements whose FP32 storage value x32 lies exactly halfway between two neighbouring values of the narrow
    format: (number of such elements, how many of them the narrow storage xn holds as the odd neighbour). Raises if
    a narrow value there is not one of the two neighbours."""
    u = x32.astype(np.float32).view(np.uint32).astype(np.int64)
    mag = np.abs(x32)
    if dtype == "bf16":
        mid = ((u & 0xffff) == 0x8000) & (mag < 3.3e38)
        nb = xn[mid].astype(np.float32).view(np.uint32).astype(np.int64)
        assert ((nb & 0xffff) == 0).all()
        hi = nb >> 16
        lo = u[mid] >> 16
        assert np.isin(hi - lo, [0, 1]).all(), "a narrow value at a midpoint is not one of its neighbours"
        return int(mid.sum()), int((hi & 1).sum())
    normal = mag >= 2.0 ** -14
    mid = np.where(normal, (u & 0x1fff) == 0x1000, np.mod(mag * 2.0 ** 25, 2.0) == 1.0) & (mag < 65504)
    half = np.where(normal, np.exp2(np.floor(np.log2(np.maximum(mag, 2.0 ** -14))) - 11), 2.0 ** -25)[mid]
    assert np.allclose(np.abs(xn[mid] - x32[mid]), half, rtol=0, atol=0), \
        "a narrow value at a midpoint is not one of its neighbours"
    bits = xn[mid].astype(np.float16).view(np.uint16)
    return int(mid.sum()), int((bits & 1).sum())


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_storage_rounds_once(dtype):
    """Reduced storage holds the FP64 on-chip sum rounded once. Where the FP32 storage of the same frame holds a
    value exactly halfway between two neighbouring values of the narrow format, the FP64 sum lay within half an
    FP32 step of that midpoint, on either side of it, so a single rounding picks the odd neighbour about as often as
    the even one; rounding through FP32 would pick the even one every time. 1024 x 512 pixels, rank 3: 8.4 M
    coefficients, about a thousand such midpoints for FP16 and a hundred for BF16."""
    f = synth.frame_c1(seed=31, width=1024, height=512, mean=16.0)
    say("case storage rounds once", dtype, "F", f.count)
    x32 = gpu_render(f, dtype="f32")["coeffs"]
    xn = gpu_render(f, dtype=dtype)["coeffs"]
    n, odd = _midpoint_picks(x32.ravel(), xn.ravel(), dtype)
    say("  %s: %d FP32 values on a midpoint, %d stored as the odd neighbour" % (dtype, n, odd))
    assert n >= (400 if dtype == "f16" else 40)
    assert 0.2 * n <= odd <= 0.8 * n


@pytest.mark.parametrize("rank", [1, 3, 4])
def test_e5b9g9r9_storage(orc, rank):
    """Packed three-channel storage (section 2.1): the decoded coefficients are within one step of the shared
    exponent (max |triple| / 255) of the oracle run at the same storage; the words equal the oracle's packing of
    the GPU's own FP32 coefficients of the same frame, bit for bit; the composite is within 2e-3 of the oracle at
    E5B9G9R9 storage, and its error against the exact oracle is reported."""
    f = synth.frame_c3(seed=20 + rank, width=45, height=29, rank=rank, particles=8.0)
    say("case e5b9g9r9 rank", rank, "F", f.count)
    g = gpu_render(f, dtype="e5b9g9r9")
    o = oracle_frame(orc, f, storage="e5b9g9r9", want=("coeffs", "out"))
    ex = oracle_frame(orc, f, want=("coeffs", "out"))
    dec = e5_decode(orc, g["words"])
    tmax = np.abs(ex["coeffs"]).max(axis=1, keepdims=True)
    assert np.all(np.abs(dec - o["coeffs"]) <= tmax / 255.0 * (1 + 1e-6) + 1e-30)
    assert np.all(dec[:, :, 0] >= 0) and np.all(dec[:, :, 1:] <= 0)
    err_same = assert_close_abs(g["out"], o["out"], 2e-3, what="e5 out vs oracle at e5 storage")
    say("  e5b9g9r9: max |out - oracle(e5)| = %.2e, max |out - oracle(exact)| = %.2e"
        % (err_same, float(np.abs(g["out"] - ex["out"]).max())))
    f32 = gpu_render(f, dtype="f32")["coeffs"].reshape(-1, 3, f32_M(rank))
    words = np.array([[orc.pack_e5b9g9r9(*(abs(f32[p, :, m]))) for m in range(f32.shape[2])]
                      for p in range(f32.shape[0])], dtype=np.uint32)
    mism = int((words != g["words"]).sum())
    assert mism <= max(1, words.size // 10000), "%d of %d words differ from the oracle's packing" % (mism, words.size)
    # the separate passes store and reload the packed words
    p = gpu_passes(f, dtype="e5b9g9r9")
    assert np.array_equal(p["words"], g["words"]) or \
        np.abs(e5_decode(orc, p["words"]) - dec).max() <= tmax.max() / 255.0
    np.testing.assert_allclose(p["out"], g["out"], rtol=0, atol=2e-3)


def f32_M(rank):
    return 1 << (rank + 1)


@pytest.mark.parametrize("channels,rank", [(1, 0), (1, 3), (1, 4), (1, 6), (3, 3)])
def test_tight_depth_bounds(orc, channels, rank):
    """Per-pixel depth bounds (section 2.1, step 1) against the oracle with the same bounds: fused render and the
    separate passes, on a ragged frame; the plain and tight results differ."""
    f = (synth.frame_c1(seed=50 + rank, width=53, height=38, rank=rank, mean=9.0) if channels == 1 else
         synth.frame_c3(seed=50 + rank, width=53, height=38, rank=rank, particles=6.0))
    say("case tight depth channels", channels, "rank", rank)
    g = gpu_render(f, tight=True)
    o = oracle_frame(orc, f, tight=True)
    assert_coeffs(g["coeffs"], o["coeffs"])
    assert_close_abs(g["out"], o["out"], 1e-4)
    p = gpu_passes(f, tight=True)
    assert_coeffs(p["coeffs"], o["coeffs"])
    S, sa = accum_to_oracle_layout(p["accum"], channels)
    np.testing.assert_allclose(S, o["accum"], rtol=2e-5, atol=1e-7)
    assert_close_abs(p["out"], o["out"], 1e-4)
    plain = oracle_frame(orc, f, want=("out",))
    assert np.abs(plain["out"] - o["out"]).max() > 1e-3


def test_tight_depth_smoke_1080p_sampled(orc):
    """The smoke frame (depths concentrated around 0.5) with per-pixel bounds, on sampled pixels."""
    import torch
    import paper_2201_00094_amd as wt
    f = synth.frame_c2(seed=3, rank=3)
    say("case tight smoke 1080p F", f.count)
    spec = spec_of(f, tight=True)
    fr = wt.Fragments.from_numpy(f.pixel, f.depth, f.alpha, f.rgb)
    ws = wt.Workspace(spec, f.count)
    coeffs = spec.new_coeffs()
    out = wt.render(spec, fr, f.bg, ws, coeffs=coeffs)
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    sel = np.unique(rng.choice(f.pixels, 1500, replace=False))
    mask = np.zeros(f.pixels, bool)
    mask[sel] = True
    o = oracle_frame(orc, f, mask=mask, want=("coeffs", "out"), tight=True)
    assert_coeffs(coeffs.cpu().double().numpy(), o["coeffs"], sel=sel)
    assert_close_abs(out.cpu().double().numpy(), o["out"], 1e-4, sel=sel)
    del fr, ws, coeffs, out
    torch.cuda.empty_cache()


def test_order_independence_and_chunks(orc):
    """Permuted and chunked streams give the same result within the parity tolerance (P6, P10)."""
    f = synth.frame_c1(seed=11, width=90, height=70, mean=20.0)
    say("case permutation/chunks")
    o = oracle_frame(orc, f)
    base = gpu_passes(f)
    perm = f.subset(np.random.default_rng(1).permutation(f.count))
    permuted = gpu_passes(perm)
    chunked = gpu_passes(f, chunks=5)
    for r in (base, permuted, chunked):
        assert_coeffs(r["coeffs"], o["coeffs"])
        assert_close_abs(r["out"], o["out"], 1e-4)


def test_empty_frame_shows_background():
    import torch
    import paper_2201_00094_amd as wt
    say("case empty frame")
    spec = wt.FrameSpec(33, 17, 3)
    fr = wt.Fragments(torch.zeros(0, dtype=torch.int32, device="cuda"), torch.zeros(0, device="cuda"),
                      torch.zeros(0, device="cuda"), torch.zeros((0, 3), device="cuda"))
    ws = wt.Workspace(spec, 0)
    coeffs = spec.new_coeffs()
    coeffs.fill_(7.0)
    out = wt.render(spec, fr, (0.25, 0.5, 0.75), ws, coeffs=coeffs)
    torch.cuda.synchronize()
    assert (coeffs == 0).all()
    assert torch.equal(out.cpu(), torch.tensor([[0.25, 0.5, 0.75]]).expand(33 * 17, 3))
    assert wt.dropped_count(ws) == 0


def test_edge_values_and_drops(orc):
    W, H = 5, 4
    pix = np.array([0, 0, 0, 1, 1, 2, 3, 3, 7, 100, 5, 6, 6], np.uint32)
    depth = np.array([0.0, 1.0, 0.5, -3.0, 7.0, np.nan, 0.25, 0.75, 0.1, 0.2, 0.3, 0.6, 0.6], np.float32)
    alpha = np.array([0.3, 0.9, 0.0, 1.0, -0.5, 0.5, 2.0, 0.99999, np.nan, 0.3, 1e-7, 0.5, 0.5], np.float32)
    rgb = np.random.default_rng(0).random((13, 3), dtype=np.float32)
    f = synth.Frame(W, H, 3, 1, pix, depth, alpha, rgb, (0.1, 0.2, 0.3), "edges")
    say("case edge values")
    g = gpu_render(f)
    o = oracle_frame(orc, f, want=("coeffs", "out"))
    assert g["dropped"] == 3 and o["dropped"] == 3
    assert_coeffs(g["coeffs"], o["coeffs"])
    assert_close_abs(g["out"], o["out"], 1e-4)


@pytest.mark.parametrize("rank", [3, 4])
def test_smoke_1080p_64_full(orc, rank):
    """The benchmark workload (1920x1080, Poisson(64 g) fragments/px, 132.7 M fragments) in the benchmark's launch
    configuration: every coefficient and every composite pixel of the frame against the oracle, plus sign and
    monotonicity of the stored coefficients over the whole frame."""
    import torch
    import paper_2201_00094_amd as wt
    f = synth.frame_c2(seed=0, rank=rank)
    say("case smoke 1080p rank", rank, "F", f.count)
    spec = spec_of(f)
    fr = wt.Fragments.from_numpy(f.pixel, f.depth, f.alpha, f.rgb)
    ws = wt.Workspace(spec, f.count)
    coeffs = spec.new_coeffs()
    out = wt.render(spec, fr, f.bg, ws, coeffs=coeffs)
    torch.cuda.synchronize()
    assert wt.dropped_count(ws) == 0
    c = coeffs[:, 0, :]
    assert bool((c[:, 0] >= 0).all()) and bool((c[:, 1:] <= 0).all())
    # P5 over the whole frame: the cell values of the stored coefficients (the level-scaled inverse Haar transform,
    # children = parent +/- d) never decrease with depth, up to the FP32 rounding of the stored values
    v = c[:, :1].double()
    for n in range(rank + 1):
        d = c[:, (1 << n):(2 << n)].double()
        v = torch.stack([v + d, v - d], dim=2).reshape(c.shape[0], 2 << n)
    tol = 4 * 2.0 ** -24 * v.abs().amax(dim=1, keepdim=True)
    assert bool(((v[:, 1:] - v[:, :-1]) >= -tol).all()), "cell values decrease with depth"
    del v, d
    o = oracle_frame(orc, f, want=("coeffs", "out"))
    gc = coeffs.cpu().double().numpy()
    go = out.cpu().double().numpy()
    assert_coeffs(gc, o["coeffs"])
    err = assert_close_abs(go, o["out"], 1e-4)
    say("  max |out - oracle| over all %d pixels: %.2e" % (f.pixels, err))
    del fr, ws, coeffs, out, o, gc, go
    torch.cuda.empty_cache()


@pytest.mark.parametrize("width,height", [(1200, 1100), (2000, 1100), (3840, 2160)])
def test_many_tiles(orc, width, height):
    """Three channels at rank 4 use 16 x 8 tiles: about 10,000, 17,000 and 64,800 tiles (at 3840 x 2160), each binned
    in two levels (super-tiles of up to 64 tiles, then a split into tiles)."""
    f = synth.frame_c3(seed=width, width=width, height=height, rank=4, particles=1.0)
    say("case many tiles", width, height, "F", f.count)
    g = gpu_render(f)
    rng = np.random.default_rng(width)
    sel = np.unique(rng.choice(f.pixels, 3000, replace=False))
    mask = np.zeros(f.pixels, bool)
    mask[sel] = True
    o = oracle_frame(orc, f, mask=mask, want=("coeffs", "out"))
    assert g["dropped"] == 0
    assert_coeffs(g["coeffs"], o["coeffs"], sel=sel)
    assert_close_abs(g["out"], o["out"], 1e-4, sel=sel)


@pytest.fixture(scope="module")
def glass_4k():
    """The glass + particles frame at full size, generated once for the module."""
    import paper_2201_00094_amd as wt
    f = synth.frame_c3(seed=0, rank=3)
    return f, wt.Fragments.from_numpy(f.pixel, f.depth, f.alpha, f.rgb)


@pytest.mark.parametrize("dtype,rel", [("f32", 1e-5), ("f16", 2 * 2.0 ** -11 + 1e-5), ("bf16", 2 * 2.0 ** -8 + 1e-5)])
def test_glass_4k_full(orc, glass_4k, dtype, rel):
    """The glass + particles workload at full size (3840x2160, rank 3, 2-4 glass layers with per-channel alpha plus
    Poisson(24) particles per pixel, about 224 M fragments) in the benchmark's launch configuration (bin count,
    bin scatter, render over the binned stream; two-level binning), FP32, FP16 and BF16 storage: every coefficient
    and every composite pixel against the oracle (FP16 and BF16 against the oracle at the same storage precision)."""
    import torch
    import paper_2201_00094_amd as wt
    f, fr = glass_4k
    say("case glass 4K F", f.count, "storage", dtype)
    sel = None
    spec = wt.FrameSpec(f.width, f.height, 3, 3, dtype)
    ws = wt.Workspace(spec, f.count)
    coeffs = spec.new_coeffs()
    out = torch.empty((spec.pixels, 3), dtype=torch.float32, device="cuda")
    wt.bin_count(spec, fr, ws)
    wt.bin_scatter(spec, fr, ws)
    wt.render_binned(spec, ws, f.bg, out, coeffs)
    torch.cuda.synchronize()
    assert wt.dropped_count(ws) == 0
    o = oracle_frame(orc, f, want=("coeffs", "accum", "out"), storage="exact" if dtype == "f32" else dtype)
    assert_coeffs(coeffs.float().cpu().double().numpy(), o["coeffs"], rel=rel, sel=sel, what=dtype + " coeffs",
                  atol=STORAGE_ATOL[dtype])
    if dtype == "f32":
        err = assert_close_abs(out.cpu().double().numpy(), o["out"], 1e-4, sel=sel, what=dtype + " out")
    else:
        tol = storage_out_bound(orc, 3, o["coeffs"], o["accum"], 3, rel, atol=STORAGE_ATOL[dtype])
        err, ratio = assert_within(out.cpu().double().numpy(), o["out"], tol, sel=sel, what=dtype + " out")
        say("  %s: largest error / derived bound %.2f" % (dtype, ratio))
    say("  %s: max |out - oracle| over all %d pixels: %.2e" % (dtype, f.pixels, err))
    del ws, coeffs, out, o
    torch.cuda.empty_cache()


def test_global_binning_fallback(orc):
    """More than 8192 super-tiles of 64 tiles: three channels at rank 8 use 8-pixel tiles (their FP64 coefficient
    sums take 12 KB of LDS per pixel), so a 2048 x 2064 frame has 528,384 tiles and 8,256 super-tiles, beyond one
    LDS table; the stream is then binned with one global atomic per fragment. The composite (no coefficient array
    is written) on 2,000 sampled pixels against the oracle."""
    f = synth.frame_c3(seed=5, width=2048, height=2064, rank=8, particles=0.3)
    say("case global binning fallback F", f.count)
    g = gpu_render(f, want_coeffs=False)
    assert g["dropped"] == 0
    rng = np.random.default_rng(5)
    sel = np.unique(rng.choice(f.pixels, 2000, replace=False))
    mask = np.zeros(f.pixels, bool)
    mask[sel] = True
    o = oracle_frame(orc, f, mask=mask, want=("out",))
    err = assert_close_abs(g["out"], o["out"], 1e-4, sel=sel)
    say("  max |out - oracle| on %d sampled pixels: %.2e" % (sel.size, err))


def test_stream_past_2_31_fragments(orc):
    """Maximum sizes: 2^31 + 12,345 fragments (about 1,036 per pixel: 51.5 GB of input and a 60 GB workspace) over
    the 1920x1080 rank-3 frame in the benchmark's launch configuration, so fragment indices, record slots and
    segment offsets run past 2^31, with a partial last chunk. No drops; signs of every stored coefficient; and
    about 48 pixels against the oracle: the pixels of the first and last fragment, both sides of the ragged edge
    (the pixels before it hold one fragment more) and 43 random ones, each with its whole list of fragments."""
    import torch
    import paper_2201_00094_amd as wt
    W, H, F = 1920, 1080, (1 << 31) + 12345
    P = W * H
    say("case stream past 2^31: F", F)
    pixel, depth, alpha, rgb, A, B = synth.scrambled_stream(5, W, H, F)
    spec = wt.FrameSpec(W, H, 3, 1, "f32")
    fr = wt.Fragments(pixel, depth, alpha, rgb)
    ws = wt.Workspace(spec, F)
    coeffs = spec.new_coeffs()
    bg = (0.2, 0.3, 0.4)
    out = wt.render(spec, fr, bg, ws, coeffs=coeffs)
    torch.cuda.synchronize()
    assert wt.dropped_count(ws) == 0
    c = coeffs[:, 0, :]
    assert bool((c[:, 0] >= 0).all()) and bool((c[:, 1:] <= 0).all())
    # the pixel of fragment i is (A i + B) mod P; pixel p holds the fragments i_p + k P
    rag = F % P
    rng = np.random.default_rng(5)
    firsts = np.unique(np.concatenate([[0, P - 1, rag - 1, rag, (F - 1) % P], rng.choice(P, 43, replace=False)]))
    sel = (A * firsts + B) % P
    dev = pixel.device
    parts = []
    for j, ip in enumerate(firsts):
        idx = torch.arange(int(ip), F, P, device=dev)
        parts.append((np.full(idx.numel(), j, np.uint32), depth[idx].cpu().numpy(), alpha[idx].cpu().numpy(),
                      rgb[idx].cpu().numpy()))
    n = len(parts)
    assert sum(p[0].size for p in parts) == sum(F // P + (ip < rag) for ip in firsts)
    mp, md, ma, mc = (np.concatenate([p[k] for p in parts]) for k in range(4))
    o = orc.resolve(n, 1, 3, mp, md, ma, mc, bg=bg, want=("coeffs", "out"))
    sel_t = torch.from_numpy(sel).to(dev)
    assert_coeffs(coeffs[sel_t].cpu().double().numpy(), o["coeffs"])
    err = assert_close_abs(out[sel_t].cpu().double().numpy(), o["out"], 1e-4)
    say("  %d pixels with %d-%d fragments each: max |out - oracle| %.2e" %
        (n, min(p[0].size for p in parts), max(p[0].size for p in parts), err))
    del pixel, depth, alpha, rgb, fr, ws, coeffs, out, c
    torch.cuda.empty_cache()
