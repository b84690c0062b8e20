"""Synthetic frames: per-pixel fragment counts first, then attributes, then one global shuffle.

Workloads (all seeded with NumPy's PCG64 ``default_rng``):

* ``frame_c1`` -- 64x64, Poisson(8) fragments/px, depth in (0.05, 1], alpha U[0.05, 0.6], rgb U[0,1]^3.
* ``frame_c2`` -- smoke: 1920x1080, Poisson(64 g(x, y)) fragments/px with g a clipped sum of six seeded 2-D
  Gaussian blobs rescaled to mean 1, depth Normal(0.5, 0.1) clipped to (0, 1], alpha U[0.02, 0.1], grey-ish rgb.
* ``frame_c3`` -- glass + particles: 3840x2160, 2-4 glass layers/px with per-channel alpha U[0.3, 0.9] at depth
  U[0.2, 0.8], plus Poisson(24) particles/px with alpha U[0.02, 0.2] (same in every channel).
* ``frame_c4`` -- one serving request: Poisson(24) fragments/px with the c1 distributions.
* ``frame_c5`` -- differentiation: 512x512, Poisson(32) fragments/px, alpha U[0.05, 0.5].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

REQUEST_RESOLUTIONS = ((640, 360), (1280, 720), (1920, 1080), (3840, 2160))
TINY_DEPTH = np.float32(2.0 ** -24)


@dataclass
class Frame:
    width: int
    height: int
    rank: int
    channels: int
    pixel: np.ndarray
    depth: np.ndarray
    alpha: np.ndarray
    rgb: np.ndarray
    bg: tuple = (0.2, 0.2, 0.2)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def count(self) -> int:
        return int(self.pixel.shape[0])

    @property
    def pixels(self) -> int:
        return self.width * self.height

    def subset(self, idx) -> "Frame":
        """Frame holding the fragments ``idx`` (in that order) of this one."""
        return Frame(self.width, self.height, self.rank, self.channels, self.pixel[idx], self.depth[idx],
                     self.alpha[idx], self.rgb[idx], self.bg, self.name, dict(self.meta))


def _u(rng, lo, hi, n, dtype=np.float32):
    return (lo + (hi - lo) * rng.random(n, dtype=np.float64)).astype(dtype)


def make_frame(width, height, counts, rng, depth_fn, alpha_fn, rgb_fn, rank=3, channels=1, bg=(0.2, 0.2, 0.2),
               name="", shuffle=True) -> Frame:
    """Assemble a stream from per-pixel ``counts`` and attribute samplers ``fn(rng, F) -> array``."""
    counts = np.asarray(counts, dtype=np.int64).reshape(-1)
    assert counts.shape[0] == width * height
    F = int(counts.sum())
    pixel = np.repeat(np.arange(width * height, dtype=np.uint32), counts)
    depth = np.asarray(depth_fn(rng, F), dtype=np.float32)
    alpha = np.asarray(alpha_fn(rng, F), dtype=np.float32)
    rgb = np.asarray(rgb_fn(rng, F), dtype=np.float32).reshape(F, 3)
    if shuffle and F > 1:
        perm = rng.permutation(F)
        pixel, depth, alpha, rgb = pixel[perm], depth[perm], alpha[perm], rgb[perm]
    return Frame(width, height, rank, channels, np.ascontiguousarray(pixel), np.ascontiguousarray(depth),
                 np.ascontiguousarray(alpha), np.ascontiguousarray(rgb), tuple(bg), name)


def _depth_c1(rng, F):
    # 1 - 0.95 U[0,1): uniform on (0.05, 1]
    return (1.0 - 0.95 * rng.random(F, dtype=np.float64)).astype(np.float32)


def _rgb_uniform(rng, F):
    return rng.random((F, 3), dtype=np.float32)


def frame_c1(seed=0, width=64, height=64, rank=3, mean=8.0) -> Frame:
    """Plain method check: Poisson(8) fragments/px, depth (0.05, 1], alpha U[0.05, 0.6], rgb U[0,1]^3."""
    rng = np.random.default_rng(seed)
    counts = rng.poisson(mean, width * height)
    return make_frame(width, height, counts, rng, _depth_c1, lambda r, F: _u(r, 0.05, 0.6, F), _rgb_uniform, rank=rank,
                      name="c1_%dx%d_r%d" % (width, height, rank))


def smoke_density(rng, width, height, blobs=6, lo=0.1, hi=2.0):
    """Six seeded Gaussian blobs (centres uniform over the frame, sigma U[0.1, 0.3] * height, amplitude
    U[0.5, 1.5]), scaled by the factor that makes the mean of the clipped field 1 (found by bisection)."""
    cx = rng.uniform(0, width, blobs)
    cy = rng.uniform(0, height, blobs)
    sig = rng.uniform(0.1, 0.3, blobs) * height
    amp = rng.uniform(0.5, 1.5, blobs)
    ys = np.arange(height, dtype=np.float64)[:, None]
    xs = np.arange(width, dtype=np.float64)[None, :]
    G = np.zeros((height, width))
    for b in range(blobs):
        G += amp[b] * np.exp(-((xs - cx[b]) ** 2 + (ys - cy[b]) ** 2) / (2.0 * sig[b] ** 2))
    s_lo, s_hi = 0.0, 1.0
    while np.clip(s_hi * G, lo, hi).mean() < 1.0:
        s_hi *= 2.0
    for _ in range(60):
        s = 0.5 * (s_lo + s_hi)
        if np.clip(s * G, lo, hi).mean() < 1.0:
            s_lo = s
        else:
            s_hi = s
    return np.clip(0.5 * (s_lo + s_hi) * G, lo, hi).reshape(-1)


def _depth_smoke(rng, F):
    d = rng.normal(0.5, 0.1, F)
    return np.clip(d, float(TINY_DEPTH), 1.0).astype(np.float32)


def _rgb_grey(rng, F):
    grey = rng.uniform(0.4, 0.6, F).astype(np.float32)
    tint = rng.uniform(-0.05, 0.05, (F, 3)).astype(np.float32)
    return grey[:, None] + tint


def frame_c2(seed=0, width=1920, height=1080, rank=3, mean=64.0) -> Frame:
    """Smoke: Poisson(mean * g) fragments/px, depth Normal(0.5, 0.1) clipped to (0, 1], alpha U[0.02, 0.1]."""
    rng = np.random.default_rng(seed)
    g = smoke_density(rng, width, height)
    counts = rng.poisson(mean * g)
    f = make_frame(width, height, counts, rng, _depth_smoke, lambda r, F: _u(r, 0.02, 0.1, F), _rgb_grey, rank=rank,
                   name="c2_smoke_%dx%d_r%d" % (width, height, rank))
    f.meta["density_mean"] = float(g.mean())
    return f


def frame_uniform(seed=0, width=1920, height=1080, rank=3, mean=64.0) -> Frame:
    """Flat cross-check of the smoke workload: Poisson(mean) fragments/px with the smoke attributes."""
    rng = np.random.default_rng(seed)
    counts = rng.poisson(mean, width * height)
    return make_frame(width, height, counts, rng, _depth_smoke, lambda r, F: _u(r, 0.02, 0.1, F), _rgb_grey, rank=rank,
                      name="flat_%dx%d_r%d" % (width, height, rank))


def frame_c3(seed=0, width=3840, height=2160, rank=3, particles=24.0) -> Frame:
    """Glass + particles with per-channel transmittance (three visibility channels)."""
    rng = np.random.default_rng(seed)
    P = width * height
    n_glass = rng.integers(2, 5, P)
    n_part = rng.poisson(particles, P)
    Fg, Fp = int(n_glass.sum()), int(n_part.sum())
    pix = np.concatenate([np.repeat(np.arange(P, dtype=np.uint32), n_glass),
                          np.repeat(np.arange(P, dtype=np.uint32), n_part)])
    depth = np.concatenate([_u(rng, 0.2, 0.8, Fg), _depth_c1(rng, Fp)])
    alpha = np.concatenate([_u(rng, 0.3, 0.9, Fg * 3).reshape(Fg, 3),
                            np.repeat(_u(rng, 0.02, 0.2, Fp)[:, None], 3, axis=1)])
    rgb = rng.random((Fg + Fp, 3), dtype=np.float32)
    perm = rng.permutation(Fg + Fp)
    f = Frame(width, height, rank, 3, np.ascontiguousarray(pix[perm]), np.ascontiguousarray(depth[perm]),
              np.ascontiguousarray(alpha[perm]), np.ascontiguousarray(rgb[perm]), (0.2, 0.2, 0.2),
              "c3_glass_%dx%d_r%d" % (width, height, rank))
    f.meta["glass"] = Fg
    f.meta["particles"] = Fp
    return f


def frame_c4(seed, width, height, rank, mean=24.0) -> Frame:
    """One serving request: Poisson(mean) fragments/px with the c1 distributions."""
    f = frame_c1(seed=seed, width=width, height=height, rank=rank, mean=mean)
    f.name = "c4_%dx%d_r%d_s%d" % (width, height, rank, seed)
    return f


def frame_c5(seed=0, width=512, height=512, rank=3, mean=32.0) -> Frame:
    """Differentiation workload: Poisson(32) fragments/px, alpha U[0.05, 0.5], rgb U[0,1]^3."""
    rng = np.random.default_rng(seed)
    counts = rng.poisson(mean, width * height)
    return make_frame(width, height, counts, rng, _depth_c1, lambda r, F: _u(r, 0.05, 0.5, F), _rgb_uniform, rank=rank,
                      name="c5_%dx%d_r%d" % (width, height, rank))


def target_image(seed, width, height):
    """Seeded target image U[0,1]^3 for the differentiation loss."""
    rng = np.random.default_rng(seed + 1000003)
    return rng.random((width * height, 3))


def poisson_arrivals(seed, n, rate_hz, resolutions=REQUEST_RESOLUTIONS, ranks=(3, 4), dtypes=("f32", "f16")):
    """Serving trace: ``n`` requests with exponential inter-arrival times (``rate_hz``), each with a resolution,
    rank and coefficient storage type drawn uniformly, and a per-request frame seed."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, n))
    res = rng.integers(0, len(resolutions), n)
    rk = rng.integers(0, len(ranks), n)
    dt = rng.integers(0, len(dtypes), n)
    seeds = rng.integers(0, 2 ** 31 - 1, n)
    return [dict(t=float(t[i]), width=resolutions[res[i]][0], height=resolutions[res[i]][1], rank=ranks[rk[i]],
                 dtype=dtypes[dt[i]], seed=int(seeds[i])) for i in range(n)]


def torch_frame(seed, width, height, mean=24.0, rank=3, device="cuda"):
    """Device-side generator with the c1/c4 distributions (Poisson(mean) fragments/px, depth in (0.05, 1],
    alpha U[0.05, 0.6], rgb U[0,1]^3, shuffled), seeded with torch's generator on the device. Returns
    (pixel int32, depth, alpha, rgb) device tensors. Used where NumPy generation of many large frames would be
    too slow (serving traces); it is not bit-compatible with the NumPy streams."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    P = width * height
    counts = torch.poisson(torch.full((P,), float(mean), device=device), generator=g).to(torch.int64)
    pixel = torch.repeat_interleave(torch.arange(P, device=device, dtype=torch.int32), counts)
    F = int(pixel.numel())
    perm = torch.randperm(F, generator=g, device=device)
    pixel = pixel[perm].contiguous()
    del perm
    depth = (1.0 - 0.95 * torch.rand(F, generator=g, device=device)).contiguous()
    alpha = (0.05 + 0.55 * torch.rand(F, generator=g, device=device)).contiguous()
    rgb = torch.rand((F, 3), generator=g, device=device).contiguous()
    return pixel, depth, alpha, rgb



def scrambled_multiplier(P):
    """The multiplier of :func:`scrambled_stream`: the first integer at or above 0.618 P that is coprime to P, so
    that i -> (A i + B) mod P visits every pixel once per P consecutive fragments in a scattered order."""
    import math
    A = max(1, int(0.6180339887 * P))
    while math.gcd(A, P) != 1:
        A += 1
    return A


def scrambled_stream(seed, width, height, count, alpha=(0.0005, 0.003), device="cuda", chunk=1 << 28, channels=1):
    """Exactly ``count`` fragments spread evenly over the frame in a scrambled order, drawn on the device for streams
    too large to generate on the host (past 2^31 fragments). Fragment i lands on pixel (A i + B) mod P
    (A = :func:`scrambled_multiplier`, B from the seed), so pixel p holds the fragments i_p + k P, k = 0, 1, ...,
    with i_p = A^-1 (p - B) mod P: any pixel's fragments are gathered without a search, and the pixels with
    i_p < count mod P hold one fragment more. Depth U[0,1), alpha U[alpha] ([count] or, for three channels,
    [count, 3]), rgb U[0,1]^3 from torch's generator on the device (small alphas keep the deep per-pixel lists
    visible). Returns (pixel int32, depth, alpha, rgb, A, B) with the tensors on ``device``."""
    import torch
    P = width * height
    A = scrambled_multiplier(P)
    B = int(seed) * 7919 % P
    pixel = torch.empty(count, dtype=torch.int32, device=device)
    for s in range(0, count, chunk):
        e = min(count, s + chunk)
        i = torch.arange(s, e, dtype=torch.int64, device=device)
        pixel[s:e] = ((i * A + B) % P).to(torch.int32)
        del i
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    depth = torch.rand(count, generator=g, device=device)
    lo, hi = alpha
    al = torch.empty((count, 3) if channels == 3 else count, device=device).uniform_(float(lo), float(hi), generator=g)
    rgb = torch.rand((count, 3), generator=g, device=device)
    return pixel, depth, al, rgb, A, B


def sparse_stream(seed, width, height, pixels, mean=3.0):
    """Fragments on the listed pixels only, 1 + Poisson(mean) each, in shuffled order, with the c1 distributions
    (depth (0.05, 1], alpha U[0.05, 0.6], rgb U[0,1]^3): for frames too large to describe pixel by pixel (up to
    2^32 - 1 pixels). Returns (pixel uint32, depth, alpha, rgb) NumPy arrays."""
    rng = np.random.default_rng(seed)
    pixels = np.asarray(pixels, dtype=np.int64).reshape(-1)
    assert pixels.size == 0 or (pixels.min() >= 0 and pixels.max() < width * height)
    counts = 1 + rng.poisson(mean, pixels.size)
    pixel = np.repeat(pixels, counts)
    F = pixel.size
    perm = rng.permutation(F)
    pixel = np.ascontiguousarray(pixel[perm].astype(np.uint32))
    depth = _depth_c1(rng, F)
    alpha = _u(rng, 0.05, 0.6, F)
    rgb = _rgb_uniform(rng, F)
    return pixel, depth, alpha, rgb
