"""Pins of the FP64 oracle against what the paper and the mathematics fix (no GPU needed).

Each test checks the oracle against something other than itself: the worked example of section 1.2, the
inner-product definition of the Haar coefficients (section 2.3) evaluated by quadrature, the box-filter
closed form of the cell averages, the sign and locality statements of section 2.3.1, the exact A-buffer on
grid-aligned inputs, hand-worked cases, and finite differences for the gradient.
"""
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _haar_psi(n, k, z):
    """Textbook orthonormal Haar wavelet 2^(n/2) psi(2^n z - k), psi = +1 on [0, 1/2), -1 on [1/2, 1)."""
    u = (2.0 ** n) * z - k
    return (2.0 ** (0.5 * n)) * (((u >= 0) & (u < 0.5)).astype(float) - ((u >= 0.5) & (u < 1.0)).astype(float))


def _step_absorbance(z, x, a):
    """A(z) = sum_i a_i theta(z - x_i), evaluated on an array of z (section 2.2, discrete interfaces)."""
    return (a[None, :] * (z[:, None] > x[None, :])).sum(axis=1)


def _random_pixel(rng, k, lo=0.0, hi=1.0):
    x = rng.uniform(lo, hi, k)
    alpha = rng.uniform(0.02, 0.7, k)
    a = -np.log1p(-alpha)
    return x, alpha, a


# ---------------------------------------------------------------------------------------------- P1
def test_p1_worked_example_single_layer(orc):
    """Section 1.2: one 25%-opaque plane gives v = 1 in front of it and 0.75 behind it."""
    alpha, v_front, v_behind = np.loadtxt(os.path.join(GOLDEN, "single_layer_25pct.txt"))
    for rank in (0, 1, 3, 4, 6):
        M = 2 ** (rank + 1)
        for x in (0.0, 0.1, 0.37, 0.5, 0.8125, 0.93):
            a = orc.absorbance(alpha)
            cells = orc.cells_one(rank, orc.coeffs_one(rank, [x], [a]))
            j0 = int(np.floor(M * x))
            for z in np.linspace(0.0, 1.0, 257):
                v = np.exp(-orc.reconstruct(rank, cells, z))
                if z <= j0 / M:
                    assert v == pytest.approx(v_front, abs=1e-15)
                elif z >= (j0 + 2) / M:
                    assert v == pytest.approx(v_behind, abs=1e-14)
    # exact A-buffer: same numbers, with a probe layer of negligible alpha in front and behind
    pix = np.zeros(3, np.uint32)
    depth = np.array([0.5, 0.25, 0.75], np.float32)
    al = np.array([alpha, 1e-7, 1e-7], np.float32)
    rgb = np.ones((3, 3), np.float32)
    vis = orc.abuffer(1, 1, pix, depth, al, rgb, want_vis=True)["vis"][:, 0]
    assert vis[1] == pytest.approx(v_front, abs=1e-15)
    assert vis[2] == pytest.approx(v_behind, rel=1e-6)
    # the wavelet method on the grid: identical to the A-buffer (P8 on the worked example)
    w = orc.resolve(1, 1, 3, pix, depth, al, rgb, want=("vis",))["vis"][:, 0]
    assert w[1] == pytest.approx(v_front, abs=1e-15)
    assert w[2] == pytest.approx(vis[2], rel=1e-12)


# ---------------------------------------------------------------------------------------------- P2
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_p2_closed_forms_match_inner_products(orc, seed):
    """Section 2.3.1: chi = <A, phi_00> and X_nk = <A, psi_nk>, by midpoint quadrature of the step function."""
    rng = np.random.default_rng(seed)
    rank = 4
    x, _, a = _random_pixel(rng, 12)
    Q = 1 << 20
    z = (np.arange(Q) + 0.5) / Q
    A = np.zeros(Q)
    for xi, ai in zip(x, a):  # accumulate per layer to keep memory small
        A += ai * (z > xi)
    coef = orc.coeffs_one(rank, x, a)
    tol = 2.0 * a.sum() / Q
    assert coef[0] == pytest.approx(A.mean(), abs=tol)
    for n in range(rank + 1):
        for k in range(2 ** n):
            X_quad = (A * _haar_psi(n, k, z)).mean()
            X_closed = coef[2 ** n + k] / orc.level_scale(n)
            assert X_closed == pytest.approx(X_quad, abs=tol * 2.0 ** (0.5 * n))


def test_p2_Psi_is_antiderivative_of_psi(orc):
    """Psi_nk(x) = integral_0^x psi_nk, checked by quadrature at a few points."""
    Q = 1 << 16
    for n in range(4):
        for k in range(2 ** n):
            for x in (0.03, 0.26, 0.49, 0.51, 0.77, 1.0):
                z = (np.arange(Q) + 0.5) / Q * x
                integral = _haar_psi(n, k, z).mean() * x
                assert orc.Psi(n, k, x) == pytest.approx(integral, abs=4.0 * 2 ** (0.5 * n) / Q)
                assert orc.psi(n, k, (k + 0.25) / 2 ** n) == pytest.approx(2 ** (0.5 * n))


# ---------------------------------------------------------------------------------------------- P3
@pytest.mark.parametrize("rank", [0, 1, 3, 4, 7])
def test_p3_cell_averages_are_box_filtered_absorbance(orc, rank):
    """Inverse Haar of the coefficients = the average of A over each cell = sum a_i clamp((j+1) - M x_i, 0, 1)."""
    rng = np.random.default_rng(100 + rank)
    M = 2 ** (rank + 1)
    for trial in range(20):
        x, _, a = _random_pixel(rng, int(rng.integers(1, 40)))
        if trial == 0:
            x[:3] = [0.0, 1.0, 0.5]
        cells = orc.cells_one(rank, orc.coeffs_one(rank, x, a))
        j = np.arange(M)
        box = (a[None, :] * np.clip((j[:, None] + 1) - M * x[None, :], 0.0, 1.0)).sum(axis=1)
        np.testing.assert_allclose(cells, box, rtol=1e-12, atol=1e-13)


def test_p3_cell_averages_by_quadrature(orc):
    rng = np.random.default_rng(7)
    rank = 3
    M = 16
    x, _, a = _random_pixel(rng, 9)
    Q = 1 << 18
    cells = orc.cells_one(rank, orc.coeffs_one(rank, x, a))
    for j in range(M):
        z = (j + (np.arange(Q) + 0.5) / Q) / M
        assert cells[j] == pytest.approx(_step_absorbance(z, x, a).mean(), abs=2 * a.sum() / Q)


# ---------------------------------------------------------------------------------------------- P4
def test_p4_sign_of_coefficients(orc):
    """Section 2.3.1 (and the discussion): the scaling coefficient is >= 0, every wavelet coefficient <= 0."""
    f = synth.frame_c1(seed=3, width=16, height=16)
    r = orc.resolve(16, 16, 3, f.pixel, f.depth, f.alpha, f.rgb, want=("coeffs",))
    c = r["coeffs"][:, 0, :]
    assert (c[:, 0] >= 0).all()
    assert (c[:, 1:] <= 0).all()
    assert (c[:, 1:] < 0).any()


# ---------------------------------------------------------------------------------------------- P5
def test_p5_monotone_visibility(orc):
    rng = np.random.default_rng(11)
    for rank in (2, 3, 4):
        for _ in range(30):
            x, _, a = _random_pixel(rng, int(rng.integers(1, 30)))
            cells = orc.cells_one(rank, orc.coeffs_one(rank, x, a))
            assert (np.diff(cells) >= -1e-14).all()
            zs = np.linspace(0, 1, 513)
            At = np.array([orc.reconstruct(rank, cells, zz) for zz in zs])
            assert (np.diff(At) >= -1e-14).all()
            assert At[0] == 0.0


# ---------------------------------------------------------------------------------------------- P6
def test_p6_permutation_invariance_bit_exact(orc):
    f = synth.frame_c1(seed=5, width=24, height=20)
    r0 = orc.resolve(24, 20, 3, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg)
    perm = np.random.default_rng(9).permutation(f.count)
    g = f.subset(perm)
    r1 = orc.resolve(24, 20, 3, g.pixel, g.depth, g.alpha, g.rgb, bg=f.bg)
    for key in ("coeffs", "cells", "accum", "suma", "out"):
        assert np.array_equal(r0[key], r1[key]), key
    assert np.array_equal(r0["vis"][perm], r1["vis"])


# ---------------------------------------------------------------------------------------------- P7
def test_p7_logarithmic_locality(orc):
    """Section 2.3.1: a fragment updates the scaling coefficient and one wavelet per level: N+2 values."""
    rng = np.random.default_rng(13)
    for rank in (0, 3, 4, 9):
        for x in rng.uniform(0, 1, 50):
            c = orc.coeffs_one(rank, [x], [0.3])
            nz = np.count_nonzero(c)
            assert nz <= rank + 2
            M = 2 ** (rank + 1)
            if abs(M * x - round(M * x)) > 1e-9:  # off the finest grid: every level's tent is non-zero
                assert nz == rank + 2


# ---------------------------------------------------------------------------------------------- P8
@pytest.mark.parametrize("rank", [1, 3, 4])
def test_p8_grid_depths_reproduce_exact_abuffer(orc, rank):
    """All depths on the subdivision {m/M}: the interpolated wavelet result equals the exact A-buffer."""
    rng = np.random.default_rng(rank)
    W, H = 12, 10
    M = 2 ** (rank + 1)
    counts = rng.poisson(6, W * H)
    F = int(counts.sum())
    pix = np.repeat(np.arange(W * H, dtype=np.uint32), counts)
    depth = (rng.integers(0, M + 1, F) / M).astype(np.float32)
    al = rng.uniform(0.05, 0.8, F).astype(np.float32)
    rgb = rng.random((F, 3), dtype=np.float32)
    bg = (0.1, 0.3, 0.7)
    w = orc.resolve(W, H, rank, pix, depth, al, rgb, bg=bg)
    ab = orc.abuffer(W, H, pix, depth, al, rgb, bg=bg, want_vis=True)
    np.testing.assert_allclose(w["vis"], ab["vis"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(w["out"], ab["out"], rtol=1e-12, atol=1e-14)


def test_p8_grid_depths_three_channels(orc):
    """P8 with per-channel transmittance: each channel matches the exact A-buffer of that channel."""
    rng = np.random.default_rng(77)
    W, H, rank = 8, 6, 3
    M = 2 ** (rank + 1)
    counts = rng.poisson(5, W * H)
    F = int(counts.sum())
    pix = np.repeat(np.arange(W * H, dtype=np.uint32), counts)
    depth = (rng.integers(0, M + 1, F) / M).astype(np.float32)
    al = rng.uniform(0.05, 0.9, (F, 3)).astype(np.float32)
    rgb = rng.random((F, 3), dtype=np.float32)
    bg = (0.6, 0.1, 0.3)
    w = orc.resolve(W, H, rank, pix, depth, al, rgb, bg=bg, channels=3)
    ab = orc.abuffer(W, H, pix, depth, al, rgb, bg=bg, channels=3, want_vis=True)
    np.testing.assert_allclose(w["vis"], ab["vis"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(w["out"], ab["out"], rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------------------------------------- P9
def test_p9_error_envelope_against_abuffer(orc):
    """For z in cell j: |A~(z) - A(z-)| <= sum of a_i with x_i in [(j-1)/M, (j+1)/M]."""
    rng = np.random.default_rng(17)
    for rank in (1, 3, 4):
        M = 2 ** (rank + 1)
        for _ in range(40):
            x, _, a = _random_pixel(rng, int(rng.integers(1, 25)))
            cells = orc.cells_one(rank, orc.coeffs_one(rank, x, a))
            for z in rng.uniform(0, 1, 40):
                j = min(int(np.floor(M * z)), M - 1)
                exact = a[x < z].sum()
                window = a[(x >= (j - 1) / M) & (x <= (j + 1) / M)].sum()
                assert abs(orc.reconstruct(rank, cells, z) - exact) <= window + 1e-12


# ---------------------------------------------------------------------------------------------- P10
def test_p10_additivity(orc):
    f = synth.frame_c1(seed=21, width=16, height=16)
    half = f.count // 2
    a, b = f.subset(np.arange(half)), f.subset(np.arange(half, f.count))
    r = orc.resolve(16, 16, 3, f.pixel, f.depth, f.alpha, f.rgb, want=("coeffs", "suma"))
    ra = orc.resolve(16, 16, 3, a.pixel, a.depth, a.alpha, a.rgb, want=("coeffs", "suma"))
    rb = orc.resolve(16, 16, 3, b.pixel, b.depth, b.alpha, b.rgb, want=("coeffs", "suma"))
    np.testing.assert_allclose(ra["coeffs"] + rb["coeffs"], r["coeffs"], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(ra["suma"] + rb["suma"], r["suma"], rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------------------------------------- P11
def test_p11_three_channels_with_equal_alpha(orc):
    f = synth.frame_c1(seed=4, width=10, height=9)
    r1 = orc.resolve(10, 9, 3, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg)
    a3 = np.repeat(f.alpha[:, None], 3, axis=1)
    r3 = orc.resolve(10, 9, 3, f.pixel, f.depth, a3, f.rgb, bg=f.bg, channels=3)
    for c in range(3):
        np.testing.assert_array_equal(r3["coeffs"][:, c], r1["coeffs"][:, 0])
        np.testing.assert_array_equal(r3["vis"][:, c], r1["vis"][:, 0])
    np.testing.assert_allclose(r3["out"], r1["out"], rtol=1e-14)


# ---------------------------------------------------------------------------------------------- P12 / P13
def test_p12_empty_pixel_and_far_fragment(orc):
    pix = np.array([1, 1], np.uint32)
    depth = np.array([1.0, 1.0], np.float32)
    al = np.array([0.4, 0.0], np.float32)
    rgb = np.array([[0.9, 0.5, 0.1], [1.0, 1.0, 1.0]], np.float32)
    bg = (0.2, 0.3, 0.4)
    r = orc.resolve(2, 1, 3, pix, depth, al, rgb, bg=bg)
    assert (r["coeffs"] == 0).all()  # P13: depth 1 changes no coefficient; pixel 0 is empty
    np.testing.assert_array_equal(r["out"][0], np.array(bg))  # empty pixel shows the background exactly
    a = np.float64(np.float32(0.4))
    expect = a * rgb[0].astype(np.float64) + np.array(bg) * (1.0 - a)
    np.testing.assert_allclose(r["out"][1], expect, rtol=1e-14)


def test_p13_far_fragment_leaves_coefficients(orc):
    rng = np.random.default_rng(3)
    x, _, a = _random_pixel(rng, 10)
    c0 = orc.coeffs_one(4, x, a)
    c1 = orc.coeffs_one(4, np.append(x, 1.0), np.append(a, 2.0))
    np.testing.assert_array_equal(c0, c1)


# ---------------------------------------------------------------------------------------------- hand-worked
def test_hand_worked_off_grid_single_layer(orc):
    """alpha 0.25 at depth 0.3, rank 0 (M = 2): chi = 0.7a, d_00 = -0.3a, cells (0.4a, a),
    A~(0.3) = 0.6 * 0.4a, v = 0.75^0.24."""
    a = -np.log(0.75)
    c = orc.coeffs_one(0, [0.3], [a])
    np.testing.assert_allclose(c, [0.7 * a, -0.3 * a], rtol=1e-14)
    cells = orc.cells_one(0, c)
    np.testing.assert_allclose(cells, [0.4 * a, a], rtol=1e-14)
    assert np.exp(-orc.reconstruct(0, cells, 0.3)) == pytest.approx(0.75 ** 0.24, rel=1e-14)


def test_hand_worked_mid_layer_rank3(orc):
    """alpha 0.25 at depth 0.5, rank 3: only chi = a/2 and d_00 = -a/2 are non-zero; cells 0 then a."""
    a = -np.log(0.75)
    c = orc.coeffs_one(3, [0.5], [a])
    expect = np.zeros(16)
    expect[0], expect[1] = 0.5 * a, -0.5 * a
    np.testing.assert_allclose(c, expect, rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(orc.cells_one(3, c), np.r_[np.zeros(8), np.full(8, a)], rtol=1e-14, atol=1e-16)


def test_absorbance_and_clamps(orc):
    assert orc.absorbance(0.25) == pytest.approx(-np.log(0.75), rel=1e-15)
    assert orc.absorbance(-0.3) == 0.0
    assert orc.absorbance(1.0) == pytest.approx(24 * np.log(2.0), rel=1e-7)
    assert orc.alpha_used(2.0) == 1.0 - 2.0 ** -24


def test_dropped_fragments(orc):
    pix = np.array([0, 5, 1, 1], np.uint32)  # 5 is outside a 2x1 frame
    depth = np.array([0.5, 0.5, np.nan, 0.2], np.float32)
    al = np.array([0.5, 0.5, 0.5, np.nan], np.float32)
    rgb = np.ones((4, 3), np.float32)
    r = orc.resolve(2, 1, 3, pix, depth, al, rgb, bg=(0, 0, 0))
    assert r["dropped"] == 3
    assert np.isnan(r["vis"][1:]).all() and not np.isnan(r["vis"][0]).any()
    assert r["out"][1].tolist() == [0.0, 0.0, 0.0]


# ---------------------------------------------------------------------------------------------- storage precision
def test_storage_rounding_matches_ieee_conversions(orc):
    """FP16 rounding against NumPy's binary16 conversion, BF16 against torch's (both round to nearest even)."""
    import torch
    rng = np.random.default_rng(5)
    vals = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.uniform(-9, 4, 4000),
                           [0.0, -0.0, 1.0, 65504.0, 65519.0, 65520.0, 2.0 ** -24, 2.0 ** -25, 3 * 2.0 ** -26]])
    vals = vals.astype(np.float32).astype(np.float64)  # exactly representable in FP32: one rounding step
    f16 = np.array([orc.round_storage(v, "f16") for v in vals])
    np.testing.assert_array_equal(f16, vals.astype(np.float16).astype(np.float64))
    b16 = np.array([orc.round_storage(v, "bf16") for v in vals])
    ref = torch.from_numpy(vals.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(b16, ref)


def test_storage_rounding_in_resolve(orc):
    f = synth.frame_c1(seed=2, width=8, height=8)
    ex = orc.resolve(8, 8, 3, f.pixel, f.depth, f.alpha, f.rgb, want=("coeffs", "out"))
    h = orc.resolve(8, 8, 3, f.pixel, f.depth, f.alpha, f.rgb, want=("coeffs", "out"), storage="f16")
    np.testing.assert_array_equal(h["coeffs"], ex["coeffs"].astype(np.float16).astype(np.float64))
    assert 0 < np.abs(h["out"] - ex["out"]).max() < 1e-2


def test_e5b9g9r9_hand_worked(orc):
    """Shared-exponent words worked by hand: (1, 1/2, 1/4) has exponent field 16 and mantissas 256, 128, 64;
    1 - 2^-11 rounds up to 512 at the first exponent, so the exponent is bumped and it decodes to 1; values
    clamp at 511/512 * 2^16; zero, negative and NaN inputs store 0."""
    assert orc.pack_e5b9g9r9(1.0, 0.5, 0.25) == (16 << 27) | (64 << 18) | (128 << 9) | 256
    w = orc.pack_e5b9g9r9(1.0 - 2.0 ** -11, 0.0, 0.0)
    assert w >> 27 == 16 and orc.unpack_e5b9g9r9(w) == (1.0, 0.0, 0.0)
    assert orc.pack_e5b9g9r9(1e9, 0.0, 0.0) == (31 << 27) | 511
    assert orc.unpack_e5b9g9r9((31 << 27) | 511)[0] == 65408.0
    assert orc.pack_e5b9g9r9(0.0, 0.0, 0.0) == 0
    assert orc.pack_e5b9g9r9(-1.0, float("nan"), 2.0 ** -30) == 0
    assert orc.unpack_e5b9g9r9(orc.pack_e5b9g9r9(3.0, 2.0, 1.0)) == (3.0, 2.0, 1.0)


def test_e5b9g9r9_is_nearest_at_smallest_exponent(orc):
    """Brute force over the 32 exponents: the packed word uses the smallest exponent at which the largest
    (clamped) value is within 9 bits after rounding half up, and every component decodes to the nearest
    multiple of that exponent's step (ties up)."""
    rng = np.random.default_rng(11)
    trip = (rng.random((3000, 3)) * 10.0 ** rng.uniform(-7, 5, (3000, 1))).astype(np.float32)
    trip[::7, 1] = 0.0
    trip[::11] *= np.float32(2.0 ** 10)
    vmax = 511.0 / 512.0 * 65536.0
    for r, g, b in trip:
        v = np.minimum(np.array([r, g, b], np.float64), vmax)
        w = orc.pack_e5b9g9r9(r, g, b)
        e = w >> 27
        fits = [ex for ex in range(32) if v.max() < 511.5 * 2.0 ** (ex - 24)]
        assert e == fits[0]
        step = 2.0 ** (e - 24)
        dec = np.array(orc.unpack_e5b9g9r9(w))
        assert np.all(dec - v <= step / 2) and np.all(dec - v > -step / 2)
        assert np.all(np.abs(dec / step - np.round(dec / step)) == 0)


def test_e5b9g9r9_in_resolve(orc):
    """Three channels stored as E5B9G9R9: signs are kept (chi >= 0, d <= 0, stored as magnitudes) and each
    coefficient is within half a step of the shared exponent, i.e. within max|triple| / 511."""
    f = synth.frame_c3(seed=4, width=12, height=9, particles=6.0)
    ex = orc.resolve(12, 9, 3, f.pixel, f.depth, f.alpha, f.rgb, channels=3, want=("coeffs", "out"))
    e5 = orc.resolve(12, 9, 3, f.pixel, f.depth, f.alpha, f.rgb, channels=3, want=("coeffs", "out"),
                     storage="e5b9g9r9")
    c, q = ex["coeffs"], e5["coeffs"]
    assert np.all(q[:, :, 0] >= 0) and np.all(q[:, :, 1:] <= 0)
    tmax = np.abs(c).max(axis=1, keepdims=True)
    assert np.all(np.abs(q - c) <= tmax / 511.0 * (1 + 1e-6) + 1e-30)
    assert 0 < np.abs(e5["out"] - ex["out"]).max() < 2e-2
    with pytest.raises(Exception):
        orc.resolve(4, 4, 3, f.pixel[:0], f.depth[:0], f.alpha[:0, 0], f.rgb[:0], storage="e5b9g9r9")


# ---------------------------------------------------------------------------------------------- A-buffer
def test_abuffer_golden_two_layers(orc):
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "two_layer_abuffer.txt")) if ln.strip() and ln[0] != "#"]
    frags = np.array([[float(v) for v in r] for r in rows if r[0] not in ("bg", "out")])
    bg = [float(v) for v in rows[-2][1:]]
    expect = [float(v) for v in rows[-1][1:]]
    F = frags.shape[0]
    for perm in ([0, 1], [1, 0]):
        fr = frags[perm]
        out = orc.abuffer(1, 1, np.zeros(F, np.uint32), fr[:, 0].astype(np.float32), fr[:, 1].astype(np.float32),
                          fr[:, 2:5].astype(np.float32), bg=bg)["out"][0]
        np.testing.assert_allclose(out, expect, rtol=1e-15)


def test_abuffer_sorted_equals_brute_force(orc):
    rng = np.random.default_rng(23)
    W, H = 9, 7
    counts = rng.poisson(7, W * H)
    F = int(counts.sum())
    pix = np.repeat(np.arange(W * H, dtype=np.uint32), counts)
    depth = (rng.integers(0, 12, F) / 11).astype(np.float32)  # many ties
    al = rng.uniform(0, 0.9, (F, 3)).astype(np.float32)
    rgb = rng.random((F, 3), dtype=np.float32)
    for C in (1, 3):
        a = al if C == 3 else al[:, 0].copy()
        s = orc.abuffer(W, H, pix, depth, a, rgb, bg=(0.3, 0.2, 0.1), channels=C, want_vis=True)
        b = orc.abuffer(W, H, pix, depth, a, rgb, bg=(0.3, 0.2, 0.1), channels=C, want_vis=True, brute=True)
        np.testing.assert_allclose(s["out"], b["out"], rtol=1e-13)
        np.testing.assert_allclose(s["vis"], b["vis"], rtol=1e-13)


# ---------------------------------------------------------------------------------------------- P14 (oracle side)
@pytest.mark.parametrize("channels", [1, 3])
def test_p14_backward_matches_finite_differences(orc, channels, tight=False):
    rng = np.random.default_rng(31 + channels)
    W, H, rank = 6, 5, 3
    f = synth.frame_c5(seed=channels, width=W, height=H, rank=rank, mean=9)
    alpha = f.alpha if channels == 1 else np.ascontiguousarray(
        np.clip(f.alpha[:, None] * rng.uniform(0.6, 1.4, (f.count, 3)), 0.05, 0.5).astype(np.float32))
    target = synth.target_image(3, W, H)
    bg = (0.2, 0.5, 0.8)

    def loss(al, rgb):
        out = orc.resolve(W, H, rank, f.pixel, f.depth, al, rgb, bg=bg, channels=channels, want=("out",),
                          tight=tight)["out"]
        return ((out - target) ** 2).sum()

    out = orc.resolve(W, H, rank, f.pixel, f.depth, alpha, f.rgb, bg=bg, channels=channels, want=("out",),
                      tight=tight)["out"]
    ga, gr = orc.backward(W, H, rank, f.pixel, f.depth, alpha, f.rgb, 2.0 * (out - target), bg=bg, channels=channels,
                          tight=tight)
    # FD in FP64 needs FP64 inputs: perturb through float64 copies by evaluating the oracle's steps on the
    # perturbed value directly (the FP32 stream is promoted exactly, so a float32 perturbation would round).
    eps = 1e-3
    for i in rng.choice(f.count, 12, replace=False):
        for c in range(channels):
            ap, am = alpha.copy(), alpha.copy()
            if channels == 1:
                ap[i] += eps
                am[i] -= eps
                h = float(ap[i]) - float(am[i])
            else:
                ap[i, c] += eps
                am[i, c] -= eps
                h = float(ap[i, c]) - float(am[i, c])
            fd = (loss(ap, f.rgb) - loss(am, f.rgb)) / h
            assert ga[i, c] == pytest.approx(fd, rel=2e-3, abs=2e-5)
        for q in range(3):
            rp, rm = f.rgb.copy(), f.rgb.copy()
            rp[i, q] += eps
            rm[i, q] -= eps
            fd = (loss(alpha, rp) - loss(alpha, rm)) / (float(rp[i, q]) - float(rm[i, q]))
            assert gr[i, q] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_p14_backward_with_tight_depth_bounds(orc):
    test_p14_backward_matches_finite_differences(orc, 1, tight=True)


# ---------------------------------------------------------------------------------------------- tight depth bounds
def _two_depth_frame(rng, W, H, channels=1):
    """Every pixel holds 1-5 fragments at exactly two distinct depths (ties included)."""
    pix, dep = [], []
    for p in range(W * H):
        z = np.sort(rng.choice(np.arange(1, 255), 2, replace=False) / 256.0)
        k = rng.integers(2, 6)
        d = np.concatenate([z, rng.choice(z, k - 2)])
        pix += [p] * k
        dep += list(d)
    F = len(pix)
    alpha = rng.uniform(0.05, 0.8, (F, channels) if channels == 3 else F).astype(np.float32)
    return (np.array(pix, np.uint32), np.array(dep, np.float32), alpha, rng.random((F, 3), dtype=np.float32))


@pytest.mark.parametrize("channels", [1, 3])
def test_tight_depth_two_layers_are_exact(orc, channels):
    """With per-pixel bounds two distinct depths land on 0 and 1: the near group sees v = 1 (the knot at 0) and the
    far group sees the full near absorbance (the last cell average), which is exactly the sorted A-buffer."""
    rng = np.random.default_rng(40 + channels)
    W, H = 7, 5
    pix, dep, al, rgb = _two_depth_frame(rng, W, H, channels)
    t = orc.resolve(W, H, 3, pix, dep, al, rgb, bg=(0.3, 0.2, 0.1), channels=channels, want=("out", "vis"), tight=True)
    a = orc.abuffer(W, H, pix, dep, al, rgb, bg=(0.3, 0.2, 0.1), channels=channels, want_vis=True)
    np.testing.assert_allclose(t["vis"], a["vis"], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(t["out"], a["out"], rtol=1e-12, atol=1e-15)
    plain = orc.resolve(W, H, 3, pix, dep, al, rgb, bg=(0.3, 0.2, 0.1), channels=channels, want=("out",))
    assert np.abs(plain["out"] - a["out"]).max() > 1e-4  # off-grid depths are approximated without the bounds


def test_tight_depth_affine_invariance(orc):
    """The tight result depends on depth only through each pixel's relative position: x -> 1/8 + x/2 (exact on a
    dyadic grid) leaves every output bit-identical, while the plain result changes."""
    rng = np.random.default_rng(44)
    f = synth.frame_c1(seed=44, width=9, height=8, mean=7.0)
    dep = (np.floor(f.depth * 256.0) / 256.0).astype(np.float32)
    dep2 = (0.125 + dep / 2.0).astype(np.float32)
    a = orc.resolve(9, 8, 3, f.pixel, dep, f.alpha, f.rgb, bg=f.bg, want=("coeffs", "out"), tight=True)
    b = orc.resolve(9, 8, 3, f.pixel, dep2, f.alpha, f.rgb, bg=f.bg, want=("coeffs", "out"), tight=True)
    np.testing.assert_array_equal(a["coeffs"], b["coeffs"])
    np.testing.assert_array_equal(a["out"], b["out"])
    pa = orc.resolve(9, 8, 3, f.pixel, dep, f.alpha, f.rgb, bg=f.bg, want=("out",))
    pb = orc.resolve(9, 8, 3, f.pixel, dep2, f.alpha, f.rgb, bg=f.bg, want=("out",))
    assert np.abs(pa["out"] - pb["out"]).max() > 1e-4
    del rng


def test_tight_depth_full_range_is_plain(orc):
    """A pixel whose fragments already span [0, 1] is unchanged by the bounds (x' = x), bit for bit."""
    f = synth.frame_c1(seed=45, width=6, height=6, mean=5.0)
    P = f.pixels
    pix = np.concatenate([f.pixel, np.arange(P, dtype=np.uint32), np.arange(P, dtype=np.uint32)])
    dep = np.concatenate([f.depth, np.zeros(P, np.float32), np.ones(P, np.float32)])
    al = np.concatenate([f.alpha, np.full(P, 0.3, np.float32), np.full(P, 0.4, np.float32)])
    rgb = np.concatenate([f.rgb, np.full((P, 3), 0.5, np.float32), np.full((P, 3), 0.25, np.float32)])
    a = orc.resolve(6, 6, 3, pix, dep, al, rgb, bg=f.bg, want=("coeffs", "out"), tight=True)
    b = orc.resolve(6, 6, 3, pix, dep, al, rgb, bg=f.bg, want=("coeffs", "out"))
    np.testing.assert_array_equal(a["coeffs"], b["coeffs"])
    np.testing.assert_array_equal(a["out"], b["out"])


def test_tight_depth_single_fragment(orc):
    """One fragment per pixel maps to depth 0: nothing is in front of it, out = alpha c + bg (1 - alpha)."""
    rng = np.random.default_rng(46)
    P = 20
    pix = np.arange(P, dtype=np.uint32)
    dep = rng.uniform(0.1, 0.9, P).astype(np.float32)
    al = rng.uniform(0.1, 0.9, P).astype(np.float32)
    rgb = rng.random((P, 3), dtype=np.float32)
    bg = (0.3, 0.6, 0.9)
    t = orc.resolve(5, 4, 3, pix, dep, al, rgb, bg=bg, want=("out",), tight=True)
    ref = al[:, None].astype(np.float64) * rgb + np.array(bg)[None, :] * (1.0 - al[:, None].astype(np.float64))
    np.testing.assert_allclose(t["out"], ref, rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------------------------------------- one pass, previous frame
def _layer_frame(rng, P, M, channels, on_grid):
    """One fragment per pixel: depth on the cell grid (j0/M) or at an exact offset inside a cell ((j + t)/M)."""
    j = rng.integers(0, M, P)
    if on_grid:
        t = np.zeros(P)
    else:
        t = rng.choice([0.0, 0.25, 0.5, 0.75], P)
    dep = ((j + t) / M).astype(np.float32)
    alpha = rng.uniform(0.1, 0.8, (P, channels) if channels == 3 else P).astype(np.float32)
    rgb = rng.random((P, 3), dtype=np.float32)
    return np.arange(P, dtype=np.uint32), dep, alpha, rgb, j, t


@pytest.mark.parametrize("channels", [1, 3])
def test_shade_prev_single_previous_layer_closed_form(orc, channels):
    """The previous frame holds one layer of absorbance a0 on the grid at z0 = j0/M. Its Haar expansion is exact,
    so the cell averages are a0 from cell j0 on and 0 before it, and the interpolation of section 2.3.2 gives
    A~(x) = 0 before cell j0, t a0 inside it (x = (j0 + t)/M) and a0 beyond it. Checked for the identity map and
    for a shifted map with pixels that have no history."""
    rng = np.random.default_rng(60 + channels)
    W, H, rank = 6, 5, 3
    P, M = W * H, 16
    bg = (0.3, 0.5, 0.7)
    pp, dp, ap, rp, j0, _ = _layer_frame(rng, P, M, channels, True)
    prev = orc.resolve(W, H, rank, pp, dp, ap, rp, channels=channels, want=("coeffs",))["coeffs"]
    pc, dc, ac, rc, jc, tc = _layer_frame(rng, P, M, channels, False)
    a0 = -np.log1p(-ap.astype(np.float64)).reshape(P, channels)
    acur = ac.astype(np.float64).reshape(P, channels)
    shift = (np.arange(P) + 7) % P
    nohist = np.zeros(P, bool)
    nohist[[3, 11, 29]] = True
    maps = [(None, np.arange(P), np.zeros(P, bool)),
            (np.where(nohist, P + 5, shift).astype(np.uint32), shift, nohist)]
    for pmap, src, none in maps:
        At = np.where((jc < j0[src])[:, None], 0.0,
                      np.where((jc == j0[src])[:, None], tc[:, None] * a0[src], a0[src]))
        At[none] = 0.0
        v = np.exp(-At)
        if channels == 1:
            ref = acur * rc * v + np.array(bg)[None, :] * np.exp(np.log1p(-acur))
        else:
            ref = acur * rc * v + np.array(bg)[None, :] * (1.0 - acur)
        got = orc.shade_prev(W, H, rank, pc, dc, ac, rc, prev=prev, prev_pixel=pmap, bg=bg, channels=channels)
        np.testing.assert_allclose(got["vis"], v, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(got["out"], ref, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("channels,storage", [(1, "exact"), (1, "f16"), (3, "bf16"), (3, "e5b9g9r9")])
def test_shade_prev_static_scene_is_the_two_pass_result(orc, channels, storage):
    """A scene that does not change between frames: shading against the previous frame's (stored) coefficients
    is the two-pass resolve with coefficients at that storage precision."""
    f = synth.frame_c1(seed=61, width=11, height=7, mean=9.0) if channels == 1 else \
        synth.frame_c3(seed=61, width=11, height=7, particles=6.0)
    r = orc.resolve(f.width, f.height, 3, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg, channels=channels,
                    want=("coeffs", "out", "vis", "suma"), storage=storage)
    s = orc.shade_prev(f.width, f.height, 3, f.pixel, f.depth, f.alpha, f.rgb, prev=r["coeffs"], bg=f.bg,
                       channels=channels)
    np.testing.assert_allclose(s["vis"], r["vis"], rtol=1e-14, atol=0)
    np.testing.assert_allclose(s["suma"], r["suma"], rtol=1e-14, atol=0)
    np.testing.assert_allclose(s["out"], r["out"], rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("channels", [1, 3])
def test_shade_prev_without_history_sees_nothing_in_front(orc, channels):
    """No previous buffer (or every pixel mapped outside it): v = 1, out = sum alpha c + bg prod(1 - alpha)."""
    f = synth.frame_c1(seed=62, width=9, height=6, mean=6.0) if channels == 1 else \
        synth.frame_c3(seed=62, width=9, height=6, particles=4.0)
    P = f.pixels
    al = np.clip(f.alpha.astype(np.float64).reshape(f.count, channels), 0.0, 1.0 - 2.0 ** -24)
    S = np.zeros((P, 3))
    T = np.ones((P, channels))
    for i in range(f.count):
        p = f.pixel[i]
        for q in range(3):
            S[p, q] += al[i, q if channels == 3 else 0] * f.rgb[i, q]
        T[p] *= 1.0 - al[i]
    ref = S + np.array(f.bg)[None, :] * (T if channels == 3 else T[:, [0, 0, 0]])
    prev = np.full((P, channels, 16), -0.5)
    for kw in ({}, {"prev": prev, "prev_pixel": np.full(P, P, np.uint32)}):
        got = orc.shade_prev(f.width, f.height, 3, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg, channels=channels, **kw)
        assert (got["vis"] == 1.0).all()
        np.testing.assert_allclose(got["out"], ref, rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------------------------------------- chromatic composite
def test_spectral_weights_golden(orc):
    """Section 3 spectral weights, hand-computed (tests/golden/spectral_weights.txt), and their invariants: each
    tap's weights are non-negative and sum to one, red only below t = 1/2, blue only above it."""
    rows = np.loadtxt(os.path.join(GOLDEN, "spectral_weights.txt"))
    for k, i, r, g, b in rows:
        np.testing.assert_allclose(orc.spectral_weight(int(i), int(k)), [r, g, b], rtol=0, atol=1e-15)
    for k in (3, 5, 7, 9, 11, 17):
        for i in range(k):
            w = orc.spectral_weight(i, k)
            t = i / (k - 1)
            assert (w >= -1e-15).all() and abs(w.sum() - 1.0) < 1e-15
            assert (w[0] == 0.0) if t >= 0.5 else True
            assert (w[2] == 0.0) if t <= 0.5 else True


def _chromatic_inputs(rng, W, H, channels, max_off):
    P = W * H
    S = rng.random((P, 3))
    suma = rng.uniform(0.0, 3.0, (P, channels))
    bg = rng.random((P, 3), dtype=np.float32)
    off = rng.uniform(-max_off, max_off, (P, 2)).astype(np.float32)
    return S, suma, bg, off


@pytest.mark.parametrize("channels", [1, 3])
def test_chromatic_zero_offset_reads_the_pixel(orc, channels):
    """No refraction: every tap lands on the pixel centre, where the bilinear sample is the texel itself."""
    rng = np.random.default_rng(70 + channels)
    W, H = 13, 9
    S, suma, bg, off = _chromatic_inputs(rng, W, H, channels, 0.0)
    T = np.exp(-suma)[:, [0, 0, 0] if channels == 1 else [0, 1, 2]]
    for disp in (0.0, 0.5, 2.0):
        out = orc.resolve_chromatic(W, H, S, suma, bg, np.zeros_like(off), dispersion=disp, taps=5, channels=channels)
        np.testing.assert_allclose(out, S + T * bg, rtol=1e-15, atol=1e-15)


def test_chromatic_uniform_background_is_the_plain_composite(orc):
    """A uniform background is unchanged by any gather (weights normalised per channel): the chromatic composite of
    a frame equals the two-pass resolve over that constant colour."""
    f = synth.frame_c3(seed=71, width=10, height=8, particles=5.0)
    r = orc.resolve(f.width, f.height, 3, f.pixel, f.depth, f.alpha, f.rgb, bg=(0.3, 0.6, 0.1), channels=3,
                    want=("accum", "suma", "out"))
    rng = np.random.default_rng(71)
    off = rng.uniform(-30, 30, (f.pixels, 2)).astype(np.float32)
    bg = np.tile(np.array([0.3, 0.6, 0.1], np.float32), (f.pixels, 1))
    out = orc.resolve_chromatic(f.width, f.height, r["accum"], r["suma"], bg, off, dispersion=0.7, taps=7, channels=3)
    np.testing.assert_allclose(out, r["out"], rtol=1e-7, atol=1e-8)  # background stored as float32


@pytest.mark.parametrize("taps,disp", [(5, 0.5), (3, 1.0), (9, 0.25)])
def test_chromatic_linear_background_closed_form(orc, taps, disp):
    """Bilinear interpolation reproduces a linear image exactly, so away from the edges channel q of the gathered
    background is the image at c + sbar_q delta, sbar_q the spectral-weighted mean of s_i = 1 + disp (t_i - 1/2)."""
    W, H = 40, 30
    P = W * H
    y, x = np.divmod(np.arange(P), W)
    cx, cy = x + 0.5, y + 0.5
    A = np.array([0.1, 0.4, 0.7])
    Bx = np.array([0.01, -0.02, 0.015])
    By = np.array([-0.005, 0.01, 0.02])
    Xg, Yg = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    img = (A[None, None, :] + Bx[None, None, :] * Xg[..., None] + By[None, None, :] * Yg[..., None])
    img = img.reshape(P, 3).astype(np.float64)
    rng = np.random.default_rng(72 + taps)
    off = rng.uniform(-3, 3, (P, 2))
    inner = (x >= 6) & (x < W - 6) & (y >= 6) & (y < H - 6)
    t = np.arange(taps) / (taps - 1)
    w = np.array([orc.spectral_weight(i, taps) for i in range(taps)])
    s = 1.0 + disp * (t - 0.5)
    sbar = (w * s[:, None]).sum(axis=0) / w.sum(axis=0)
    S = np.zeros((P, 3))
    suma = np.zeros((P, 1))
    out = orc.resolve_chromatic(W, H, S, suma, img.astype(np.float32), off.astype(np.float32), dispersion=disp,
                                taps=taps, channels=1)
    offf = off.astype(np.float32).astype(np.float64)
    ref = A[None, :] + Bx[None, :] * (cx[:, None] + sbar[None, :] * offf[:, [0]]) + \
        By[None, :] * (cy[:, None] + sbar[None, :] * offf[:, [1]])
    # the image is stored as float32: compare within its rounding
    np.testing.assert_allclose(out[inner], ref[inner], rtol=0, atol=2e-7)


def test_chromatic_edge_clamp_and_integer_offsets(orc):
    """With no dispersion every tap samples c + delta: an integer offset reads the texel it points at, and an
    offset far off screen reads the edge texel (clamp-to-edge addressing)."""
    rng = np.random.default_rng(73)
    W, H = 17, 11
    P = W * H
    S, suma, bg, _ = _chromatic_inputs(rng, W, H, 1, 0.0)
    S[:] = 0.0
    suma[:] = 0.0
    y, x = np.divmod(np.arange(P), W)
    dx = rng.integers(-4, 5, P)
    dy = rng.integers(-3, 4, P)
    off = np.stack([dx, dy], axis=1).astype(np.float32)
    out = orc.resolve_chromatic(W, H, S, suma, bg, off, dispersion=0.0, taps=5, channels=1)
    tx, ty = np.clip(x + dx, 0, W - 1), np.clip(y + dy, 0, H - 1)
    np.testing.assert_allclose(out, bg[ty * W + tx], rtol=0, atol=1e-15)
    far = np.tile(np.array([[-1000.0, 2000.0]], np.float32), (P, 1))
    out = orc.resolve_chromatic(W, H, S, suma, bg, far, dispersion=0.0, taps=3, channels=1)
    np.testing.assert_allclose(out, bg[(H - 1) * W + np.zeros(P, int)], rtol=0, atol=1e-15)


# ---------------------------------------------------------------------------------------------- generators
def test_generators_are_seeded():
    a = synth.frame_c1(seed=7, width=16, height=16)
    b = synth.frame_c1(seed=7, width=16, height=16)
    c = synth.frame_c1(seed=8, width=16, height=16)
    assert np.array_equal(a.pixel, b.pixel) and np.array_equal(a.depth, b.depth)
    assert not np.array_equal(a.depth, c.depth)
    assert a.depth.min() > 0.05 - 1e-7 and a.depth.max() <= 1.0
    assert 0.05 <= a.alpha.min() and a.alpha.max() <= 0.6


def test_smoke_density_mean_and_clip():
    rng = np.random.default_rng(0)
    g = synth.smoke_density(rng, 192, 108)
    assert g.mean() == pytest.approx(1.0, abs=1e-6)
    assert g.min() >= 0.1 and g.max() <= 2.0


def test_storage_bound_covers_one_step_moves(orc):
    """The composite bound the reduced-storage parity tests use (each stored coefficient one storage step from the
    oracle's, section 2.1 steps 3-4 and the interpolation of section 2.3.2) holds when the oracle's own coefficients
    of random pixels are moved by up to that step: the visibility-weighted sum of the moved expansion stays within
    it."""
    from gpu_helpers import storage_out_bound
    rng = np.random.default_rng(0)
    rel = 2 * 2.0 ** -11
    worst = 0.0
    for _ in range(120):
        rank = int(rng.integers(1, 5))
        M = 1 << (rank + 1)
        k = int(rng.integers(1, 30))
        x = np.sort(rng.random(k))
        a = -np.log1p(-rng.random(k) * 0.9)
        rgb = rng.random(k)
        cf = orc.coeffs_one(rank, x, a)

        def shade(c):
            cells = orc.cells_one(rank, c)
            return sum(-np.expm1(-a[i]) * rgb[i] * np.exp(-orc.reconstruct(rank, cells, x[i])) for i in range(k))

        s0 = shade(cf)
        bound = storage_out_bound(orc, rank, cf, np.full(3, s0), 1, rel, floor=0.0)[0, 0]
        for _ in range(10):
            moved = cf * (1 + rel * rng.choice([-1.0, 1.0], M) * rng.random(M))
            worst = max(worst, abs(shade(moved) - s0) / bound)
    assert worst <= 1.0
    assert worst > 0.3  # the bound is not vacuous
