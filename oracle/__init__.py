"""FP64 CPU oracle for the wavelet-transparency resolve (Wavelet Transparency, Aizenshtein, Smal, McGuire 2021).

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package. It shares no code with the HIP path; the product never calls it.

The arithmetic lives in ``wt_oracle.c`` (plain C, FP64, built with gcc into ``liboracle.so``); this module only
marshals NumPy arrays through ctypes. What each function computes, and the passage of the paper it follows, is
documented at the C definitions:

* :func:`resolve`  -- build (section 2.3.1), cell averages (2.3), interpolation (2.3.2), visibility-weighted
  shading (2.1 step 3, the compositing sum of 2.2) and the composite over a constant background (2.1 step 4).
* :func:`shade_prev` -- the one-pass variant: shading against the previous frame's coefficients (the
  future-work proposal of the paper's closing section).
* :func:`resolve_chromatic`, :func:`spectral_weight` -- the composite over a background image gathered along the
  refraction offset with per-channel spectral weights (the chromatic-aberration approximation of section 3).
* :func:`abuffer`  -- the exact sorted A-buffer the method approximates (visibility function of 1.2).
* :func:`backward` -- gradient of the resolve with respect to alpha and colour (chain rule through the steps).
* :func:`coeffs_one`, :func:`cells_one`, :func:`reconstruct`, :func:`Psi`, :func:`psi` -- the per-pixel pieces.

``ref_tiny`` is a scalar pure-Python twin for tiny frames that reaches the same quantities by another route
(cell means of the absorbance step function, then the Haar analysis); the tests compare the two.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile ``wt_oracle.c`` with gcc (OpenMP over pixels). Returns the library path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-fopenmp", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = C.CDLL(_LIB)
    vp = C.c_void_p
    lib.orc_resolve.restype = C.c_int
    lib.orc_resolve.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64, vp, vp, vp, vp, vp, vp,
                                C.c_int, C.c_int, vp, vp, vp, vp, vp, vp, vp, C.c_int]
    lib.orc_shade_prev.restype = C.c_int
    lib.orc_shade_prev.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64, vp, vp, vp, vp, vp, vp,
                                   vp, vp, C.c_uint64, vp, vp, vp, vp, vp, C.c_int]
    lib.orc_spectral_weight.restype = None
    lib.orc_spectral_weight.argtypes = [C.c_int, C.c_int, _f64p]
    lib.orc_resolve_chromatic.restype = C.c_int
    lib.orc_resolve_chromatic.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, vp, vp, vp, vp, C.c_double, C.c_int, vp]
    lib.orc_abuffer.restype = C.c_int
    lib.orc_abuffer.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64, vp, vp, vp, vp, vp, vp, C.c_int, vp, vp,
                                vp, C.c_int]
    lib.orc_backward.restype = C.c_int
    lib.orc_backward.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64, vp, vp, vp, vp, vp, vp, vp,
                                 C.c_int, vp, vp, C.c_int]
    lib.orc_coeffs_one.restype = None
    lib.orc_coeffs_one.argtypes = [C.c_int, C.c_int, _f64p, _f64p, _f64p]
    lib.orc_cells_one.restype = None
    lib.orc_cells_one.argtypes = [C.c_int, _f64p, _f64p]
    lib.orc_reconstruct.restype = C.c_double
    lib.orc_reconstruct.argtypes = [C.c_int, _f64p, C.c_double]
    lib.orc_Psi.restype = C.c_double
    lib.orc_Psi.argtypes = [C.c_int, C.c_int, C.c_double]
    lib.orc_psi.restype = C.c_double
    lib.orc_psi.argtypes = [C.c_int, C.c_int, C.c_double]
    lib.orc_absorbance.restype = C.c_double
    lib.orc_absorbance.argtypes = [C.c_double]
    lib.orc_alpha_used.restype = C.c_double
    lib.orc_alpha_used.argtypes = [C.c_double]
    lib.orc_round_storage.restype = C.c_double
    lib.orc_round_storage.argtypes = [C.c_double, C.c_int]
    lib.orc_pack_e5b9g9r9.restype = C.c_uint32
    lib.orc_pack_e5b9g9r9.argtypes = [C.c_float, C.c_float, C.c_float]
    lib.orc_unpack_e5b9g9r9.restype = None
    lib.orc_unpack_e5b9g9r9.argtypes = [C.c_uint32, _f64p]
    lib.orc_num_threads.restype = C.c_int
    lib.orc_num_threads.argtypes = []
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _stream(pixel, depth, alpha, rgb, channels):
    pixel = np.ascontiguousarray(pixel, dtype=np.uint32)
    depth = np.ascontiguousarray(depth, dtype=np.float32)
    alpha = np.ascontiguousarray(alpha, dtype=np.float32).reshape(-1)
    rgb = np.ascontiguousarray(rgb, dtype=np.float32).reshape(-1)
    F = pixel.shape[0]
    if depth.shape[0] != F or alpha.shape[0] != F * channels or rgb.shape[0] != F * 3:
        raise ValueError("fragment arrays disagree in length")
    return pixel, depth, alpha, rgb, F


def num_threads() -> int:
    return int(_load().orc_num_threads())


STORAGE = {"exact": 0, "f32": 0, "f16": 1, "bf16": 2, "e5b9g9r9": 3}


def resolve(width, height, rank, pixel, depth, alpha, rgb, bg=(0.0, 0.0, 0.0), channels=1, mask=None,
            want=("coeffs", "cells", "accum", "suma", "out", "vis"), threads=0, storage="exact", tight=False):
    """FP64 wavelet resolve of one frame. ``storage`` ("exact", "f16", "bf16", or "e5b9g9r9" for three channels)
    rounds the coefficients to that format before they are used; ``tight`` maps each pixel's depths onto its own
    [zmin, zmax] (section 2.1, step 1). Returns a dict with the requested arrays:

    ``coeffs``/``cells`` [P, C, M]; ``accum`` [P, 3]; ``suma`` [P, C]; ``out`` [P, 3]; ``vis`` [F, C]; and
    ``dropped`` (int). ``mask`` (bool [P]) restricts the computed pixels; the rest read as zeros (NaN in vis).
    """
    lib = _load()
    pixel, depth, alpha, rgb, F = _stream(pixel, depth, alpha, rgb, channels)
    P = int(width) * int(height)
    M = 1 << (int(rank) + 1)
    res = {}
    res["coeffs"] = np.zeros((P, channels, M)) if "coeffs" in want else None
    res["cells"] = np.zeros((P, channels, M)) if "cells" in want else None
    res["accum"] = np.zeros((P, 3)) if "accum" in want else None
    res["suma"] = np.zeros((P, channels)) if "suma" in want else None
    res["out"] = np.zeros((P, 3)) if "out" in want else None
    res["vis"] = np.full((F, channels), np.nan) if "vis" in want else None
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    bgv = np.ascontiguousarray(bg, dtype=np.float64)
    dropped = C.c_uint64(0)
    rc = lib.orc_resolve(width, height, rank, channels, F, _ptr(pixel), _ptr(depth), _ptr(alpha), _ptr(rgb), _ptr(bgv),
                         _ptr(m), STORAGE[storage], int(bool(tight)), _ptr(res["coeffs"]), _ptr(res["cells"]),
                         _ptr(res["accum"]),
                         _ptr(res["suma"]), _ptr(res["out"]), _ptr(res["vis"]), C.byref(dropped), int(threads))
    if rc != 0:
        raise RuntimeError("orc_resolve failed with %d" % rc)
    out = {k: v for k, v in res.items() if v is not None}
    out["dropped"] = int(dropped.value)
    return out


def shade_prev(width, height, rank, pixel, depth, alpha, rgb, prev=None, prev_pixel=None, bg=(0.0, 0.0, 0.0),
               channels=1, mask=None, want=("accum", "suma", "out", "vis"), threads=0):
    """One-pass shading against the previous frame's coefficients (the single-pass variant the paper proposes
    as future work): each pixel's fragments see the visibility reconstructed from ``prev`` [Pp, C, M] (stored
    values, FP64) at the pixel ``prev_pixel[p]`` (identity when None; entries >= Pp, or ``prev`` None, mean no
    history: visibility 1). The background weight is exp(-sum a) of this frame's fragments. Returns the arrays of
    :func:`resolve` named in ``want`` (accum, suma, out, vis) and ``dropped``."""
    lib = _load()
    pixel, depth, alpha, rgb, F = _stream(pixel, depth, alpha, rgb, channels)
    P = int(width) * int(height)
    M = 1 << (int(rank) + 1)
    pv, pp, npp = None, None, 0
    if prev is not None:
        pv = np.ascontiguousarray(prev, dtype=np.float64).reshape(-1, channels, M)
        npp = pv.shape[0]
    if prev_pixel is not None:
        pp = np.ascontiguousarray(prev_pixel, dtype=np.uint32).reshape(-1)
        if pp.shape[0] != P:
            raise ValueError("prev_pixel must hold one entry per pixel")
    res = {}
    res["accum"] = np.zeros((P, 3)) if "accum" in want else None
    res["suma"] = np.zeros((P, channels)) if "suma" in want else None
    res["out"] = np.zeros((P, 3)) if "out" in want else None
    res["vis"] = np.full((F, channels), np.nan) if "vis" in want else None
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    bgv = np.ascontiguousarray(bg, dtype=np.float64)
    dropped = C.c_uint64(0)
    rc = lib.orc_shade_prev(width, height, rank, channels, F, _ptr(pixel), _ptr(depth), _ptr(alpha), _ptr(rgb),
                            _ptr(bgv), _ptr(m), _ptr(pv), _ptr(pp), npp, _ptr(res["accum"]), _ptr(res["suma"]),
                            _ptr(res["out"]), _ptr(res["vis"]), C.byref(dropped), int(threads))
    if rc != 0:
        raise RuntimeError("orc_shade_prev failed with %d" % rc)
    out = {k: v for k, v in res.items() if v is not None}
    out["dropped"] = int(dropped.value)
    return out


def spectral_weight(i, k):
    """(red, green, blue) weight of gather tap i of k in the chromatic-aberration composite (section 3)."""
    w = np.zeros(3)
    _load().orc_spectral_weight(int(i), int(k), w)
    return w


def resolve_chromatic(width, height, S, suma, background, offset, dispersion=0.5, taps=5, channels=1):
    """Composite over a background image gathered with k taps along each pixel's refraction offset, weighted per
    channel (section 3). ``S`` [P, 3] and ``suma`` [P, C] are the accumulated colour and absorbance (e.g. from
    :func:`resolve`), ``background`` [P, 3] and ``offset`` [P, 2] (pixels) float32. Returns out [P, 3]."""
    P = int(width) * int(height)
    S = np.ascontiguousarray(S, dtype=np.float64).reshape(P, 3)
    suma = np.ascontiguousarray(suma, dtype=np.float64).reshape(P, channels)
    bg = np.ascontiguousarray(background, dtype=np.float32).reshape(P, 3)
    off = np.ascontiguousarray(offset, dtype=np.float32).reshape(P, 2)
    out = np.zeros((P, 3))
    rc = _load().orc_resolve_chromatic(width, height, channels, _ptr(S), _ptr(suma), _ptr(bg), _ptr(off),
                                       float(dispersion), int(taps), _ptr(out))
    if rc != 0:
        raise RuntimeError("orc_resolve_chromatic failed with %d" % rc)
    return out


def abuffer(width, height, pixel, depth, alpha, rgb, bg=(0.0, 0.0, 0.0), channels=1, mask=None, brute=False,
            want_vis=False, threads=0):
    """Exact A-buffer composite. Returns dict ``out`` [P, 3], optionally ``vis`` [F, C], and ``dropped``."""
    lib = _load()
    pixel, depth, alpha, rgb, F = _stream(pixel, depth, alpha, rgb, channels)
    P = int(width) * int(height)
    out = np.zeros((P, 3))
    vis = np.full((F, channels), np.nan) if want_vis else None
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    bgv = np.ascontiguousarray(bg, dtype=np.float64)
    dropped = C.c_uint64(0)
    rc = lib.orc_abuffer(width, height, channels, F, _ptr(pixel), _ptr(depth), _ptr(alpha), _ptr(rgb), _ptr(bgv),
                         _ptr(m), 1 if brute else 0, _ptr(out), _ptr(vis), C.byref(dropped), int(threads))
    if rc != 0:
        raise RuntimeError("orc_abuffer failed with %d" % rc)
    res = {"out": out, "dropped": int(dropped.value)}
    if want_vis:
        res["vis"] = vis
    return res


def backward(width, height, rank, pixel, depth, alpha, rgb, grad_out, bg=(0.0, 0.0, 0.0), channels=1, mask=None,
             threads=0, tight=False):
    """Gradient of sum(grad_out * out) w.r.t. alpha [F, C] and rgb [F, 3], FP64."""
    lib = _load()
    pixel, depth, alpha, rgb, F = _stream(pixel, depth, alpha, rgb, channels)
    P = int(width) * int(height)
    g = np.ascontiguousarray(grad_out, dtype=np.float64).reshape(-1)
    if g.shape[0] != P * 3:
        raise ValueError("grad_out must hold P*3 values")
    ga = np.zeros((F, channels))
    gr = np.zeros((F, 3))
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    bgv = np.ascontiguousarray(bg, dtype=np.float64)
    rc = lib.orc_backward(width, height, rank, channels, F, _ptr(pixel), _ptr(depth), _ptr(alpha), _ptr(rgb),
                          _ptr(bgv), _ptr(g), _ptr(m), int(bool(tight)), _ptr(ga), _ptr(gr), int(threads))
    if rc != 0:
        raise RuntimeError("orc_backward failed with %d" % rc)
    return ga, gr


def coeffs_one(rank, x, a):
    """Stored coefficients of one pixel/channel from clamped depths ``x`` and absorbance steps ``a``."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    a = np.ascontiguousarray(a, dtype=np.float64)
    out = np.zeros(1 << (rank + 1))
    _load().orc_coeffs_one(int(rank), int(x.shape[0]), x, a, out)
    return out


def cells_one(rank, coef):
    """Cell averages Abar_j of the Haar expansion held in ``coef``."""
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    out = np.zeros_like(coef)
    _load().orc_cells_one(int(rank), coef, out)
    return out


def reconstruct(rank, cells, z):
    """Interpolated absorbance A~(z) from cell averages."""
    cells = np.ascontiguousarray(cells, dtype=np.float64)
    return float(_load().orc_reconstruct(int(rank), cells, float(z)))


def Psi(n, k, x):
    return float(_load().orc_Psi(int(n), int(k), float(x)))


def psi(n, k, z):
    return float(_load().orc_psi(int(n), int(k), float(z)))


def absorbance(alpha):
    return float(_load().orc_absorbance(float(alpha)))


def pack_e5b9g9r9(r, g, b):
    """E5B9G9R9 word of three FP32 magnitudes (section 2.1 storage; the shared-exponent format)."""
    return int(_load().orc_pack_e5b9g9r9(float(r), float(g), float(b)))


def unpack_e5b9g9r9(word):
    out = np.zeros(3)
    _load().orc_unpack_e5b9g9r9(int(word), out)
    return tuple(float(v) for v in out)


def round_storage(v, storage):
    return float(_load().orc_round_storage(float(v), STORAGE[storage]))


def alpha_used(alpha):
    return float(_load().orc_alpha_used(float(alpha)))


def level_scale(n):
    """2^(n/2): stored coefficient d_{n,k} = level_scale(n) * X_{n,k}."""
    return 2.0 ** (0.5 * n)
