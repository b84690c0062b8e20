"""Scalar pure-Python twin of the FP64 oracle, for tiny frames.

TEST INFRASTRUCTURE, like the rest of this package: only ``tests/`` use it; the product never calls it.

It computes what the C oracle computes, by another route, so that the two check each other:

* The absorbance of a pixel is the step function A(z) = sum_i a_i [z > x_i] over normalised depth, with
  a_i = -ln(1 - alpha_i) (section 2.2: v = e^-A, each interface a step). Its Haar approximation at rank N
  (section 2.3: the scaling function and levels n = 0..N, M = 2^(N+1) cells) has, on cell j = [j/M, (j+1)/M), the
  cell's mean of A, which a step at x contributes a * clamp(j + 1 - M x, 0, 1) to. The oracle instead adds the
  closed-form coefficients of section 2.3.1 and synthesises the cells from them.
* Coefficients follow from the cell means by the Haar analysis written out: chi_00 = the mean of A over [0, 1];
  with the orthonormal psi_{n,k}(z) = 2^(n/2) psi(2^n z - k) and the stored d_{n,k} = 2^(n/2) X_{n,k}, d_{n,k} is
  2^n / M times (sum of the cell means over the left half of the support - sum over the right half), at m = 2^n + k.
* Visibility at a fragment interpolates linearly between knots (section 2.3.2): knot (j+1)/M carries cell j's mean
  and knot 0 carries 0, so at x in cell j the value is (1 - t) A_{j-1} + t A_j, t = M x - j (x = 1 is t = 1 in the
  last cell). The composite is sum_i alpha_i c_i v_i plus the background times e^(-sum_i a_i) (section 2.1 steps
  3 and 4).
* The exact A-buffer: v_i is the product of (1 - alpha_j) over the fragments strictly in front of fragment i
  (section 1.2's visibility function; equal depths do not occlude each other).

Inputs are clamped as the oracle clamps them (depth to [0, 1]; alpha <= 0 to 0, alpha >= 1 to 1 - 2^-24);
fragments with a pixel id outside the frame or a NaN depth or alpha are dropped and counted. With ``tight``, each
pixel's depths are mapped onto [0, 1] by its own smallest and largest clamped depth (section 2.1, step 1), 0 when
they are equal.
"""
import math

ALPHA_MAX = 1.0 - 2.0 ** -24


def clamp_alpha(a):
    return 0.0 if a <= 0.0 else (ALPHA_MAX if a >= 1.0 else a)


def clamp_depth(x):
    return min(1.0, max(0.0, x))


def absorbance(alpha):
    return -math.log1p(-alpha)


def cell_means(rank, steps):
    """Cell means of A(z) = sum a [z > x] over the M = 2^(rank+1) cells; steps: (x, a) pairs."""
    M = 2 ** (rank + 1)
    return [sum(a * min(1.0, max(0.0, j + 1 - M * x)) for x, a in steps) for j in range(M)]


def coefficients(cells):
    """Stored layout: m = 0 is chi_00, m = 2^n + k is d_{n,k}."""
    M = len(cells)
    out = [0.0] * M
    out[0] = sum(cells) / M
    n = 0
    while 2 ** n < M:
        w = M // 2 ** n
        for k in range(2 ** n):
            lo, mid, hi = k * w, k * w + w // 2, (k + 1) * w
            out[2 ** n + k] = (2 ** n / M) * (sum(cells[lo:mid]) - sum(cells[mid:hi]))
        n += 1
    return out


def interpolate(cells, x):
    M = len(cells)
    j = min(int(math.floor(M * x)), M - 1)
    t = M * x - j
    left = cells[j - 1] if j > 0 else 0.0
    return (1.0 - t) * left + t * cells[j]


def _pixels(width, height, pixel, depth, alpha, rgb, channels):
    """Valid fragments grouped by pixel: {p: [(x, [alpha_c], (r, g, b))]}, and the dropped count."""
    P = width * height
    frags, dropped = {}, 0
    for i in range(len(pixel)):
        p = int(pixel[i])
        x = float(depth[i])
        al = [float(alpha[i])] if channels == 1 else [float(v) for v in alpha[i]]
        if p < 0 or p >= P or math.isnan(x) or any(math.isnan(v) for v in al):
            dropped += 1
            continue
        frags.setdefault(p, []).append((clamp_depth(x), [clamp_alpha(v) for v in al],
                                        tuple(float(v) for v in rgb[i])))
    return frags, dropped


def _tight(fs):
    lo, hi = min(f[0] for f in fs), max(f[0] for f in fs)
    return [((f[0] - lo) / (hi - lo) if hi > lo else 0.0, f[1], f[2]) for f in fs]


def resolve(width, height, rank, pixel, depth, alpha, rgb, bg=(0.0, 0.0, 0.0), channels=1, tight=False):
    """Per pixel: coefficients [C][M] (lists), composite (r, g, b); returns (coeffs {p: ...}, out {p: ...},
    dropped). Pixels without fragments have zero coefficients and the background as composite."""
    frags, dropped = _pixels(width, height, pixel, depth, alpha, rgb, channels)
    M = 2 ** (rank + 1)
    coeffs, out = {}, {}
    for p in range(width * height):
        fs = frags.get(p, [])
        if tight and fs:
            fs = _tight(fs)
        cf, cells = [], []
        for c in range(channels):
            cm = cell_means(rank, [(x, absorbance(al[c])) for x, al, _ in fs])
            cells.append(cm)
            cf.append(coefficients(cm))
        coeffs[p] = cf
        col = []
        for q in range(3):
            c = 0 if channels == 1 else q
            s = sum(al[c] * rgb_[q] * math.exp(-interpolate(cells[c], x)) for x, al, rgb_ in fs)
            col.append(s + bg[q] * math.exp(-sum(absorbance(al[c]) for _, al, _ in fs)))
        out[p] = tuple(col)
    return coeffs, out, dropped


def abuffer(width, height, pixel, depth, alpha, rgb, bg=(0.0, 0.0, 0.0), channels=1):
    """Exact composite per pixel: {p: (r, g, b)}, and the dropped count."""
    frags, dropped = _pixels(width, height, pixel, depth, alpha, rgb, channels)
    out = {}
    for p in range(width * height):
        fs = frags.get(p, [])
        col = []
        for q in range(3):
            c = 0 if channels == 1 else q
            s = 0.0
            for x, al, rgb_ in fs:
                v = 1.0
                for y, bl, _ in fs:
                    if y < x:
                        v *= 1.0 - bl[c]
                s += al[c] * rgb_[q] * v
            t = 1.0
            for _, bl, _ in fs:
                t *= 1.0 - bl[c]
            col.append(s + bg[q] * t)
        out[p] = tuple(col)
    return out, dropped
