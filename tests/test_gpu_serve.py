"""Serving on the GPU: every request's composite is the same alone and in a concurrent mix of frame sizes, ranks,
channel counts and storage types (FP32, FP16, BF16, E5B9G9R9; within the parity tolerance), and the mix really
overlaps on the device."""
import numpy as np
import pytest

import synth
from gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_served_results_match_solo(orc):
    import torch
    import paper_2201_00094_amd as wt
    from paper_2201_00094_amd.serve import FrameRequest, GpuExecutor, Server

    shapes = [(64, 48, 3, "f32", 1), (200, 120, 4, "f32", 1), (320, 240, 3, "f16", 1), (96, 96, 4, "bf16", 1),
              (257, 131, 3, "f32", 1), (500, 300, 4, "f16", 1), (150, 90, 3, "e5b9g9r9", 3), (120, 80, 4, "f32", 3)]
    pool = []
    for i, (w, h, rank, dt, ch) in enumerate(shapes):
        f = synth.frame_c4(seed=i, width=w, height=h, rank=rank, mean=24.0) if ch == 1 else \
            synth.frame_c3(seed=i, width=w, height=h, rank=rank, particles=12.0)
        fr = wt.Fragments.from_numpy(f.pixel, f.depth, f.alpha, f.rgb)
        spec = wt.FrameSpec(w, h, rank, ch, dt)
        solo = wt.render(spec, fr, f.bg, wt.Workspace(spec, f.count))
        pool.append((f, fr, spec, solo))
    torch.cuda.synchronize()
    say("case serving mix of", len(pool), "frames")
    srv = Server(GpuExecutor(slots=4), slots=4, budget_bytes=8 << 30)
    futs = []
    for rep in range(4):
        for i, (f, fr, spec, _) in enumerate(pool):
            futs.append(srv.submit(FrameRequest(spec.width, spec.height, spec.rank, fr, dtype=spec.dtype,
                                                channels=spec.channels, bg=f.bg, tag=(rep, i))))
    results = [fu.result(timeout=120) for fu in futs]
    srv.close()
    torch.cuda.synchronize()
    worst = 0.0
    for r in results:
        f, fr, spec, solo = pool[r.tag[1]]
        d = float((r.out - solo).abs().max())
        worst = max(worst, d)
        assert d <= 1e-5, (r.tag, d)
    # the first frame against the oracle too
    f, fr, spec, solo = pool[0]
    o = orc.resolve(f.width, f.height, f.rank, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg, want=("out",))["out"]
    assert np.abs(solo.cpu().double().numpy() - o).max() <= 1e-4
    s = srv.stats.summary()
    say("  served %d requests, worst |served - solo| %.2e, max in flight %d, p50 %.3f ms p99 %.3f ms" %
        (s["completed"], worst, s["max_inflight"], s["p50_ms"], s["p99_ms"]))
    assert s["completed"] == len(futs)
    assert s["max_inflight"] >= 2


def test_fragments_produced_on_a_side_stream(orc):
    """A client that produces a request's fragments on its own stream and submits while that work is still
    queued: the slot stream is ordered after it (the event recorded at submit on the client's current stream), and
    the composite matches the frame rendered alone after a synchronisation."""
    import torch
    import paper_2201_00094_amd as wt
    from paper_2201_00094_amd.serve import FrameRequest, GpuExecutor, Server

    f = synth.frame_c4(seed=7, width=320, height=200, rank=3, mean=24.0)
    src = wt.Fragments.from_numpy(f.pixel, f.depth, f.alpha, f.rgb)
    spec = wt.FrameSpec(f.width, f.height, f.rank)
    solo = wt.render(spec, src, f.bg, wt.Workspace(spec, f.count))
    torch.cuda.synchronize()
    say("case serving: fragments from a side stream, %d fragments" % f.count)
    srv = Server(GpuExecutor(slots=2), slots=2, budget_bytes=8 << 30)
    side = torch.cuda.Stream()
    futs = []
    with torch.cuda.stream(side):
        for rep in range(3):
            torch.cuda._sleep(20_000_000)  # keeps the copies below queued when submit returns
            dst = wt.Fragments(torch.empty_like(src.pixel), torch.empty_like(src.depth),
                               torch.empty_like(src.alpha), torch.empty_like(src.rgb))
            for a, b in ((dst.pixel, src.pixel), (dst.depth, src.depth), (dst.alpha, src.alpha),
                         (dst.rgb, src.rgb)):
                a.copy_(b, non_blocking=True)
            futs.append(srv.submit(FrameRequest(f.width, f.height, f.rank, dst, bg=f.bg, tag=rep)))
            del dst
    results = [fu.result(timeout=120) for fu in futs]
    srv.close()
    torch.cuda.synchronize()
    for r in results:
        d = float((r.out - solo).abs().max())
        assert d <= 1e-5, (r.tag, d)


def test_reserved_slots_and_client_result_buffers():
    """Slots reserved for the largest request allocate nothing when requests up to that size run (no growth), and a
    request that brings its own composite buffer gets its result written there, equal to the frame rendered alone;
    under the shortest-first policy as well. A wrongly shaped buffer is refused at submit."""
    import torch
    import paper_2201_00094_amd as wt
    from paper_2201_00094_amd.serve import FrameRequest, GpuExecutor, Server

    frames = []
    for i, (w, h, rank) in enumerate([(300, 200, 4), (160, 90, 3), (64, 64, 3)]):
        f = synth.frame_c4(seed=40 + i, width=w, height=h, rank=rank, mean=16.0)
        fr = wt.Fragments.from_numpy(f.pixel, f.depth, f.alpha, f.rgb)
        spec = wt.FrameSpec(w, h, rank)
        frames.append((f, fr, spec, wt.render(spec, fr, f.bg, wt.Workspace(spec, f.count))))
    say("case serving with reserved slots and client buffers")
    ex = GpuExecutor(slots=2)
    big = frames[0]
    ex.reserve(big[0].width, big[0].height, 4, big[0].count)
    held = ex.resident_bytes()
    for f, fr, spec, _ in frames:
        req = FrameRequest(f.width, f.height, spec.rank, fr, bg=f.bg)
        assert ex.growth(0, req) == 0 and ex.growth(1, req) == 0
    srv = Server(ex, slots=2, budget_bytes=4 << 30, policy="sjf")
    outs, futs = [], []
    for rep in range(3):
        for f, fr, spec, _ in frames:
            o = torch.full((spec.pixels, 3), float("nan"), device="cuda")
            outs.append(o)
            futs.append(srv.submit(FrameRequest(f.width, f.height, spec.rank, fr, bg=f.bg, out=o)))
    res = [fu.result(timeout=60) for fu in futs]
    srv.close()
    torch.cuda.synchronize()
    assert ex.resident_bytes() == held
    for k, r in enumerate(res):
        f, fr, spec, solo = frames[k % len(frames)]
        assert r.out.data_ptr() == outs[k].data_ptr()
        assert float((r.out - solo).abs().max()) <= 1e-5
    srv2 = Server(GpuExecutor(slots=1), slots=1)
    f, fr, spec, _ = frames[1]
    bad = torch.empty((spec.pixels + 1, 3), device="cuda")
    with pytest.raises(ValueError, match="FrameRequest.out"):
        srv2.submit(FrameRequest(f.width, f.height, spec.rank, fr, bg=f.bg, out=bad))
    srv2.close()
