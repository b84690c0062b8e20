"""Gradient kernel (wt_backward, through WaveletComposite) against the oracle's FP64 gradient and against FP64
central finite differences of the oracle's forward pass."""
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


def _gpu_grads(f, rank, target, dtype="f32", tight=False):
    import torch
    import paper_2201_00094_amd as wt
    spec = wt.FrameSpec(f.width, f.height, rank, f.channels, dtype, tight)
    fr = wt.Fragments.from_numpy(f.pixel, f.depth, f.alpha, f.rgb)
    alpha = fr.alpha.clone().requires_grad_(True)
    rgb = fr.rgb.clone().requires_grad_(True)
    out = wt.composite(fr.pixel, fr.depth, alpha, rgb, spec, f.bg)
    tgt = torch.from_numpy(target).float().cuda()
    loss = ((out - tgt) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    return (out.detach().cpu().double().numpy(), alpha.grad.cpu().double().numpy().reshape(f.count, -1),
            rgb.grad.cpu().double().numpy())


@pytest.mark.parametrize("channels,rank,tight", [(1, 3, False), (1, 4, False), (1, 6, False), (3, 3, False),
                                                (1, 3, True), (3, 4, True)])
def test_backward_matches_oracle_gradient(orc, channels, rank, tight):
    if channels == 1:
        f = synth.frame_c5(seed=rank, width=45, height=38, rank=rank, mean=12.0)
    else:
        f = synth.frame_c3(seed=rank, width=45, height=38, rank=rank, particles=8.0)
    say("case backward channels", channels, "rank", rank, "tight", tight, "F", f.count)
    target = synth.target_image(rank, f.width, f.height)
    out, ga, gr = _gpu_grads(f, rank, target, tight=tight)
    o = orc.resolve(f.width, f.height, rank, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg, channels=channels,
                    want=("out",), tight=tight)
    np.testing.assert_allclose(out, o["out"], atol=1e-4, rtol=0)
    oa, orgb = orc.backward(f.width, f.height, rank, f.pixel, f.depth, f.alpha, f.rgb, 2.0 * (out - target), bg=f.bg,
                            channels=channels, tight=tight)
    sa, sr = np.abs(oa).max(), np.abs(orgb).max()
    np.testing.assert_allclose(ga, oa, rtol=1e-4, atol=2e-6 * sa)
    np.testing.assert_allclose(gr, orgb, rtol=1e-5, atol=1e-7 * sr)


@pytest.mark.parametrize("channels", [1, 3])
def test_backward_two_level_binning(orc, channels):
    """Frames whose gradient binning has more than 4096 tiles, so that the records that keep the stream index go
    through the two-level binning (super-tiles, then the split): 2100 x 1100 at one channel (512-pixel gradient
    tiles, 66 x 69 of them) and 1100 x 1000 at three (256-pixel tiles, 69 x 63). Every gradient element against the
    oracle's, as for the small frames."""
    if channels == 1:
        f = synth.frame_c5(seed=11, width=2100, height=1100, rank=3, mean=6.0)
    else:
        f = synth.frame_c3(seed=11, width=1100, height=1000, rank=3, particles=8.0)
    say("case backward two-level channels", channels, "F", f.count)
    target = synth.target_image(11, f.width, f.height)
    out, ga, gr = _gpu_grads(f, 3, target)
    o = orc.resolve(f.width, f.height, 3, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg, channels=channels,
                    want=("out",))
    np.testing.assert_allclose(out, o["out"], atol=1e-4, rtol=0)
    oa, orgb = orc.backward(f.width, f.height, 3, f.pixel, f.depth, f.alpha, f.rgb, 2.0 * (out - target), bg=f.bg,
                            channels=channels)
    sa, sr = np.abs(oa).max(), np.abs(orgb).max()
    np.testing.assert_allclose(ga, oa, rtol=1e-4, atol=2e-6 * sa)
    np.testing.assert_allclose(gr, orgb, rtol=1e-5, atol=1e-7 * sr)


def test_backward_finite_differences_512(orc):
    """512 x 512, Poisson(32) fragments/px, loss = squared error against a seeded target: gradients of 64 sampled
    fragments against FP64 central differences of the oracle (step 1e-6, the fragment's pixel re-resolved)."""
    f = synth.frame_c5(seed=0)
    say("case backward FD 512x512 F", f.count)
    target = synth.target_image(0, f.width, f.height)
    out, ga, gr = _gpu_grads(f, 3, target)
    rng = np.random.default_rng(5)
    order = rng.permutation(f.count)
    chosen = [i for i in order[:400] if 0.05 + 1e-3 < f.alpha[i] < 0.5 - 1e-3][:64]
    assert len(chosen) == 64
    eps = 1e-6
    worst = 0.0
    for i in chosen:
        p = f.pixel[i]
        idx = np.nonzero(f.pixel == p)[0]
        sub = f.subset(idx)
        k = int(np.nonzero(idx == i)[0][0])
        pix0 = np.zeros(sub.count, np.uint32)
        t = target[p]

        def loss(al, rgb):
            o = orc.resolve(1, 1, 3, pix0, sub.depth, al, rgb, bg=f.bg, want=("out",))["out"][0]
            return float(((o - t) ** 2).sum())

        ap, am = sub.alpha.copy(), sub.alpha.copy()
        ap[k] += eps
        am[k] -= eps
        fd = (loss(ap, sub.rgb) - loss(am, sub.rgb)) / (float(ap[k]) - float(am[k]))
        err = abs(ga[i, 0] - fd)
        worst = max(worst, err / (abs(fd) + 1e-3))
        assert err <= 1e-4 * abs(fd) + 2e-5, (i, ga[i, 0], fd)
        for q in range(3):
            rp, rm = sub.rgb.copy(), sub.rgb.copy()
            rp[k, q] += eps
            rm[k, q] -= eps
            fdr = (loss(sub.alpha, rp) - loss(sub.alpha, rm)) / (float(rp[k, q]) - float(rm[k, q]))
            assert abs(gr[i, q] - fdr) <= 1e-4 * abs(fdr) + 2e-6, (i, q, gr[i, q], fdr)
    say("  worst relative alpha-gradient error vs FD: %.2e" % worst)


def test_backward_zero_for_dropped_fragments():
    import torch
    import paper_2201_00094_amd as wt
    say("case backward dropped")
    W, H = 6, 5
    pix = np.array([0, 1, 99, 2, 2], np.uint32)
    depth = np.array([0.3, 0.6, 0.5, np.nan, 0.2], np.float32)
    alpha = np.array([0.3, 0.4, 0.5, 0.5, 0.2], np.float32)
    rgb = np.full((5, 3), 0.5, np.float32)
    spec = wt.FrameSpec(W, H, 3)
    fr = wt.Fragments.from_numpy(pix, depth, alpha, rgb)
    a = fr.alpha.clone().requires_grad_(True)
    c = fr.rgb.clone().requires_grad_(True)
    out = wt.composite(fr.pixel, fr.depth, a, c, spec, (0.1, 0.1, 0.1))
    out.sum().backward()
    torch.cuda.synchronize()
    assert float(a.grad[2]) == 0.0 and float(a.grad[3]) == 0.0
    assert torch.all(c.grad[2:4] == 0)
    assert float(a.grad[0]) != 0.0 and float(a.grad[4]) != 0.0
