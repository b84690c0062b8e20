"""The scrambled-order stream generator (used where a stream is too large to draw on the host): every pixel's
fragments sit at the indices its closed form names, each pixel receives its share, and the values lie in their
ranges. CPU only, small frames."""
import math

import numpy as np
import torch

import synth


def test_scrambled_stream_places_every_pixel_where_its_closed_form_says():
    for (w, h, count) in [(48, 30, 5000), (1920, 1080, 4_200_000), (7, 5, 35)]:
        P = w * h
        pixel, depth, alpha, rgb, A, B = synth.scrambled_stream(3, w, h, count, device="cpu", chunk=1 << 20)
        assert math.gcd(A, P) == 1 and A == synth.scrambled_multiplier(P)
        px = pixel.numpy().astype(np.int64)
        assert px.min() >= 0 and px.max() < P
        # each pixel holds count // P fragments, one more where i_p < count mod P
        per = np.bincount(px, minlength=P)
        ip = (pow(A, -1, P) * (np.arange(P) - B)) % P
        assert (per == count // P + (ip < count % P)).all()
        # the fragments of a pixel are exactly i_p + k P
        rng = np.random.default_rng(0)
        for p in rng.choice(P, min(P, 40), replace=False):
            where = np.flatnonzero(px == p)
            assert (where == np.arange(ip[p], count, P)).all()
        assert float(depth.min()) >= 0.0 and float(depth.max()) < 1.0
        assert float(alpha.min()) >= 0.0005 and float(alpha.max()) <= 0.003
        assert tuple(rgb.shape) == (count, 3) and rgb.dtype == torch.float32
        # the same seed draws the same stream
        again = synth.scrambled_stream(3, w, h, count, device="cpu", chunk=1 << 18)
        assert torch.equal(again[0], pixel) and torch.equal(again[1], depth) and torch.equal(again[3], rgb)
    three = synth.scrambled_stream(3, 48, 30, 5000, device="cpu", channels=3)
    assert tuple(three[2].shape) == (5000, 3) and torch.equal(three[0], synth.scrambled_stream(3, 48, 30, 5000,
                                                                                             device="cpu")[0])

