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
