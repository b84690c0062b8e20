"""PyTorch-facing wrappers of libwt. PyTorch supplies device memory and the current HIP stream; every step of the
path runs in the library's HIP kernels.

Fragments are device tensors: ``pixel`` int32/uint32 [F] (y * width + x), ``depth`` float32 [F], ``alpha``
float32 [F] or [F, 3], ``rgb`` float32 [F, 3].
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib

DTYPES = {"f32": _lib.WT_F32, "f16": _lib.WT_F16, "bf16": _lib.WT_BF16, "e5b9g9r9": _lib.WT_E5B9G9R9}
# e5b9g9r9 (three channels): one 32-bit word per coefficient index, held in an int32 tensor [P, M]
TORCH_DTYPES = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16, "e5b9g9r9": torch.int32}


@dataclass
class FrameSpec:
    width: int
    height: int
    rank: int
    channels: int = 1
    dtype: str = "f32"
    tight: bool = False   # per-pixel depth bounds (WT_TIGHT_DEPTH): pass each frame's stream whole
    temporal: bool = False  # one-pass render against the previous frame (WT_TEMPORAL): tiles sized for it
    deterministic: bool = False  # WT_DETERMINISTIC debug mode: bit-identical results run to run (slow)

    @property
    def pixels(self) -> int:
        return self.width * self.height

    @property
    def M(self) -> int:
        return 1 << (self.rank + 1)

    @property
    def accum_width(self) -> int:
        return 8 if self.channels == 3 else 4

    def c_desc(self) -> _lib.FrameDesc:
        if self.dtype not in DTYPES:
            raise ValueError("unknown coefficient storage %r" % self.dtype)
        flags = (_lib.WT_TIGHT_DEPTH if self.tight else 0) | (_lib.WT_TEMPORAL if self.temporal else 0) | \
            (_lib.WT_DETERMINISTIC if self.deterministic else 0)
        return _lib.desc(self.width, self.height, self.rank, self.channels, DTYPES[self.dtype], flags)

    def coeff_shape(self):
        if self.dtype == "e5b9g9r9":
            return (self.pixels, self.M)
        return (self.pixels, self.channels, self.M)

    def new_coeffs(self, device="cuda"):
        return torch.zeros(self.coeff_shape(), dtype=TORCH_DTYPES[self.dtype], device=device)

    def new_accum(self, device="cuda"):
        return torch.zeros((self.pixels, self.accum_width), dtype=torch.float32, device=device)


@dataclass
class Fragments:
    pixel: torch.Tensor
    depth: torch.Tensor
    alpha: torch.Tensor
    rgb: torch.Tensor

    @property
    def count(self) -> int:
        return int(self.pixel.shape[0])

    @staticmethod
    def from_numpy(pixel, depth, alpha, rgb, device="cuda") -> "Fragments":
        import numpy as np
        return Fragments(torch.from_numpy(np.ascontiguousarray(pixel).view(np.int32)).to(device),
                         torch.from_numpy(np.ascontiguousarray(depth, dtype=np.float32)).to(device),
                         torch.from_numpy(np.ascontiguousarray(alpha, dtype=np.float32)).to(device),
                         torch.from_numpy(np.ascontiguousarray(rgb, dtype=np.float32)).to(device))

    def c_struct(self, channels: int) -> _lib.Fragments:
        F = self.count
        _check(self.pixel, (torch.int32, getattr(torch, "uint32", torch.int32)), (F,), "pixel")
        _check(self.depth, (torch.float32,), (F,), "depth")
        _check(self.alpha, (torch.float32,), (F,) if channels == 1 else (F, 3), "alpha")
        _check(self.rgb, (torch.float32,), (F, 3), "rgb")
        return _lib.Fragments(F, self.pixel.data_ptr(), self.depth.data_ptr(), self.alpha.data_ptr(),
                              self.rgb.data_ptr())


def _check(t: torch.Tensor, dtypes, shape, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype not in dtypes:
        raise TypeError("%s has dtype %s" % (name, t.dtype))
    if tuple(t.shape) != tuple(shape) and not (t.numel() == 0 and shape[0] == 0):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def workspace_bytes(spec: FrameSpec, max_fragments: int) -> int:
    n = _lib.load().wt_workspace_bytes(C.byref(spec.c_desc()), int(max_fragments))
    if n == 0:
        raise ValueError("invalid frame description %r" % (spec,))
    return int(n)


class Workspace:
    """Device scratch for one frame description and fragment budget (a torch uint8 tensor)."""

    def __init__(self, spec: FrameSpec, max_fragments: int, device="cuda"):
        self.spec = spec
        self.nbytes = workspace_bytes(spec, max_fragments)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)

    @property
    def ptr(self):
        return C.c_void_p(self.buf.data_ptr())


# The tile kernels read a binned workspace under the tile geometry of the description they are given, so a call
# over an already binned stream must use the description it was binned with. The binding records that description
# on the workspace object (``binned_spec``: set by a binning, cleared when the workspace is reused otherwise) and
# refuses a mismatch before anything reaches the library. A scatter must follow the count of the same stream: the
# count records the stream's size and array addresses (``counted_stream``) beside its description. (The library
# checks the same on the device, from stamps the count leaves in the workspace; this refuses it earlier, with a
# clearer message.)
def _binned_as(ws, spec, counted=None, stream=None):
    ws.binned_spec = spec
    ws.counted_spec = counted
    ws.counted_stream = stream


def _stream_id(frags: "Fragments"):
    return (frags.count, frags.pixel.data_ptr(), frags.depth.data_ptr(), frags.alpha.data_ptr(),
            frags.rgb.data_ptr())


def _require_binned(ws, spec, name, attr="binned_spec"):
    got = getattr(ws, attr, None)
    if got is None:
        raise ValueError("%s: the workspace holds no stream %s" % (
            name, "counted by bin_count()" if attr == "counted_spec" else "binned by bin() or bin_count() + bin_scatter()"))
    if got != spec:
        raise ValueError("%s: the workspace was binned for %r, not for %r" % (name, got, spec))


def bin(spec: FrameSpec, frags: Fragments, ws: Workspace, stream=None):
    lib = _lib.load()
    _binned_as(ws, None)
    _lib.check(lib.wt_bin(C.byref(spec.c_desc()), C.byref(frags.c_struct(spec.channels)), ws.ptr, ws.nbytes,
                          _stream(stream)), "wt_bin")
    _binned_as(ws, spec)


def bin_count(spec: FrameSpec, frags: Fragments, ws: Workspace, stream=None):
    """First half of :func:`bin`: per-tile counts and segment layout."""
    _binned_as(ws, None)
    _lib.check(_lib.load().wt_bin_count(C.byref(spec.c_desc()), C.byref(frags.c_struct(spec.channels)), ws.ptr,
                                        ws.nbytes, _stream(stream)), "wt_bin_count")
    _binned_as(ws, None, counted=spec, stream=_stream_id(frags))


def bin_scatter(spec: FrameSpec, frags: Fragments, ws: Workspace, stream=None):
    """Second half of :func:`bin`: copy the stream into its tile segments (after :func:`bin_count` with the same
    arguments)."""
    _require_binned(ws, spec, "bin_scatter", attr="counted_spec")
    if getattr(ws, "counted_stream", None) != _stream_id(frags):
        raise ValueError("bin_scatter: the workspace was counted for another fragment stream (size or arrays differ)")
    _lib.check(_lib.load().wt_bin_scatter(C.byref(spec.c_desc()), C.byref(frags.c_struct(spec.channels)), ws.ptr,
                                          ws.nbytes, _stream(stream)), "wt_bin_scatter")
    _binned_as(ws, spec)


def build_binned(spec: FrameSpec, coeffs: torch.Tensor, ws: Workspace, stream=None):
    _require_binned(ws, spec, "build_binned")
    _check(coeffs, (TORCH_DTYPES[spec.dtype],), spec.coeff_shape(), "coeffs")
    _lib.check(_lib.load().wt_build_binned(C.byref(spec.c_desc()), _ptr(coeffs), ws.ptr, ws.nbytes, _stream(stream)),
               "wt_build_binned")


def evaluate_binned(spec: FrameSpec, coeffs: torch.Tensor, accum: torch.Tensor, ws: Workspace, stream=None):
    _require_binned(ws, spec, "evaluate_binned")
    _check(coeffs, (TORCH_DTYPES[spec.dtype],), spec.coeff_shape(), "coeffs")
    _check(accum, (torch.float32,), (spec.pixels, spec.accum_width), "accum")
    _lib.check(_lib.load().wt_evaluate_binned(C.byref(spec.c_desc()), _ptr(coeffs), _ptr(accum), ws.ptr, ws.nbytes,
                                              _stream(stream)), "wt_evaluate_binned")


def build(spec: FrameSpec, frags: Fragments, coeffs: torch.Tensor, ws: Workspace, stream=None):
    """coeffs += coefficients of ``frags`` (build pass)."""
    _check(coeffs, (TORCH_DTYPES[spec.dtype],), spec.coeff_shape(), "coeffs")
    _binned_as(ws, None)
    _lib.check(_lib.load().wt_build(C.byref(spec.c_desc()), C.byref(frags.c_struct(spec.channels)), _ptr(coeffs),
                                    ws.ptr, ws.nbytes, _stream(stream)), "wt_build")
    _binned_as(ws, spec)


def evaluate(spec: FrameSpec, frags: Fragments, coeffs: torch.Tensor, accum: torch.Tensor, ws: Workspace,
             stream=None):
    """accum += visibility-weighted colour and absorbance of ``frags`` (evaluate pass)."""
    _check(coeffs, (TORCH_DTYPES[spec.dtype],), spec.coeff_shape(), "coeffs")
    _check(accum, (torch.float32,), (spec.pixels, spec.accum_width), "accum")
    _binned_as(ws, None)
    _lib.check(_lib.load().wt_evaluate(C.byref(spec.c_desc()), C.byref(frags.c_struct(spec.channels)), _ptr(coeffs),
                                       _ptr(accum), ws.ptr, ws.nbytes, _stream(stream)), "wt_evaluate")
    _binned_as(ws, spec)


def resolve(spec: FrameSpec, accum: torch.Tensor, bg, out: torch.Tensor = None, stream=None) -> torch.Tensor:
    _check(accum, (torch.float32,), (spec.pixels, spec.accum_width), "accum")
    if out is None:
        out = torch.empty((spec.pixels, 3), dtype=torch.float32, device=accum.device)
    _check(out, (torch.float32,), (spec.pixels, 3), "out")
    _lib.check(_lib.load().wt_resolve(C.byref(spec.c_desc()), _ptr(accum), _lib.bg3(bg), _ptr(out), _stream(stream)),
               "wt_resolve")
    return out


def resolve_chromatic(spec: FrameSpec, accum: torch.Tensor, background: torch.Tensor, offset: torch.Tensor,
                      dispersion: float = 0.5, taps: int = 5, out: torch.Tensor = None, stream=None) -> torch.Tensor:
    """Composite over a background image [P, 3] gathered along each pixel's refraction offset [P, 2] (pixels) with
    the per-channel spectral weights of the chromatic-aberration approximation (``taps`` odd, >= 3)."""
    _check(accum, (torch.float32,), (spec.pixels, spec.accum_width), "accum")
    _check(background, (torch.float32,), (spec.pixels, 3), "background")
    _check(offset, (torch.float32,), (spec.pixels, 2), "offset")
    if out is None:
        out = torch.empty((spec.pixels, 3), dtype=torch.float32, device=accum.device)
    _check(out, (torch.float32,), (spec.pixels, 3), "out")
    _lib.check(_lib.load().wt_resolve_chromatic(C.byref(spec.c_desc()), _ptr(accum), _ptr(background), _ptr(offset),
                                                float(dispersion), int(taps), _ptr(out), _stream(stream)),
               "wt_resolve_chromatic")
    return out


def render(spec: FrameSpec, frags: Fragments, bg, ws: Workspace, out: torch.Tensor = None,
           coeffs: torch.Tensor = None, stream=None) -> torch.Tensor:
    """Whole path for one frame (bin, build, evaluate, resolve); writes ``out`` and, if given, ``coeffs``."""
    dev = frags.pixel.device
    if out is None:
        out = torch.empty((spec.pixels, 3), dtype=torch.float32, device=dev)
    _check(out, (torch.float32,), (spec.pixels, 3), "out")
    if coeffs is not None:
        _check(coeffs, (TORCH_DTYPES[spec.dtype],), spec.coeff_shape(), "coeffs")
    _binned_as(ws, None)
    _lib.check(_lib.load().wt_render(C.byref(spec.c_desc()), C.byref(frags.c_struct(spec.channels)), _lib.bg3(bg),
                                     _ptr(coeffs), _ptr(out), ws.ptr, ws.nbytes, _stream(stream)), "wt_render")
    _binned_as(ws, spec)
    return out


def render_noalloc(spec: FrameSpec, frags: Fragments, bg, out: torch.Tensor, coeffs: torch.Tensor = None,
                   stream=None) -> torch.Tensor:
    """:func:`render` without a workspace: the library bins into its own static per-GPU array (for callers that
    cannot allocate, e.g. under graph capture). ``out`` is required, so the call allocates nothing."""
    _check(out, (torch.float32,), (spec.pixels, 3), "out")
    if coeffs is not None:
        _check(coeffs, (TORCH_DTYPES[spec.dtype],), spec.coeff_shape(), "coeffs")
    _lib.check(_lib.load().wt_render_noalloc(C.byref(spec.c_desc()), C.byref(frags.c_struct(spec.channels)),
                                             _lib.bg3(bg), _ptr(coeffs), _ptr(out), _stream(stream)),
               "wt_render_noalloc")
    return out


def render_binned(spec: FrameSpec, ws: Workspace, bg, out: torch.Tensor, coeffs: torch.Tensor = None, stream=None):
    """Build, evaluate and resolve of a stream already binned into ``ws`` by :func:`bin`."""
    _require_binned(ws, spec, "render_binned")
    _check(out, (torch.float32,), (spec.pixels, 3), "out")
    if coeffs is not None:
        _check(coeffs, (TORCH_DTYPES[spec.dtype],), spec.coeff_shape(), "coeffs")
    _lib.check(_lib.load().wt_render_binned(C.byref(spec.c_desc()), ws.ptr, ws.nbytes, _lib.bg3(bg), _ptr(coeffs),
                                            _ptr(out), _stream(stream)), "wt_render_binned")
    return out


def _temporal_args(spec, prev, coeffs, prev_pixel, out):
    if prev is not None:
        _check(prev, (TORCH_DTYPES[spec.dtype],), spec.coeff_shape(), "prev")
    if coeffs is not None:
        _check(coeffs, (TORCH_DTYPES[spec.dtype],), spec.coeff_shape(), "coeffs")
    if prev_pixel is not None:
        _check(prev_pixel, (torch.int32, getattr(torch, "uint32", torch.int32)), (spec.pixels,), "prev_pixel")
    _check(out, (torch.float32,), (spec.pixels, 3), "out")


def render_temporal(spec: FrameSpec, frags: Fragments, bg, ws: Workspace, prev: torch.Tensor = None,
                    coeffs: torch.Tensor = None, prev_pixel: torch.Tensor = None, out: torch.Tensor = None,
                    stream=None) -> torch.Tensor:
    """One pass against the previous frame: shades ``frags`` with the visibility of ``prev`` (the previous frame's
    coefficients, read at ``prev_pixel[p]``, or at p when None; None for no history) while building this frame's
    coefficients into ``coeffs`` (may be ``prev`` itself when ``prev_pixel`` is None). ``spec.temporal`` must be
    set."""
    if out is None:
        out = torch.empty((spec.pixels, 3), dtype=torch.float32, device=frags.pixel.device)
    _temporal_args(spec, prev, coeffs, prev_pixel, out)
    _binned_as(ws, None)
    _lib.check(_lib.load().wt_render_temporal(C.byref(spec.c_desc()), C.byref(frags.c_struct(spec.channels)),
                                              _lib.bg3(bg), _ptr(prev), _ptr(prev_pixel), _ptr(coeffs), _ptr(out),
                                              ws.ptr, ws.nbytes, _stream(stream)), "wt_render_temporal")
    _binned_as(ws, spec)
    return out


def render_temporal_binned(spec: FrameSpec, ws: Workspace, bg, out: torch.Tensor, prev: torch.Tensor = None,
                           coeffs: torch.Tensor = None, prev_pixel: torch.Tensor = None, stream=None):
    """:func:`render_temporal` over a stream already binned into ``ws`` by :func:`bin`."""
    _require_binned(ws, spec, "render_temporal_binned")
    _temporal_args(spec, prev, coeffs, prev_pixel, out)
    _lib.check(_lib.load().wt_render_temporal_binned(C.byref(spec.c_desc()), ws.ptr, ws.nbytes, _lib.bg3(bg),
                                                     _ptr(prev), _ptr(prev_pixel), _ptr(coeffs), _ptr(out),
                                                     _stream(stream)), "wt_render_temporal_binned")
    return out


def backward(spec: FrameSpec, frags: Fragments, coeffs: torch.Tensor, accum: torch.Tensor, bg, grad_out: torch.Tensor,
             ws: Workspace, grad_alpha: torch.Tensor = None, grad_rgb: torch.Tensor = None, stream=None):
    dev = frags.pixel.device
    F = frags.count
    if grad_alpha is None:
        grad_alpha = torch.empty((F,) if spec.channels == 1 else (F, 3), dtype=torch.float32, device=dev)
    if grad_rgb is None:
        grad_rgb = torch.empty((F, 3), dtype=torch.float32, device=dev)
    _check(coeffs, (TORCH_DTYPES[spec.dtype],), spec.coeff_shape(), "coeffs")
    _check(accum, (torch.float32,), (spec.pixels, spec.accum_width), "accum")
    _check(grad_out, (torch.float32,), (spec.pixels, 3), "grad_out")
    _binned_as(ws, None)  # the gradient bins its own layout (smaller tiles, records that keep alpha)
    _lib.check(_lib.load().wt_backward(C.byref(spec.c_desc()), C.byref(frags.c_struct(spec.channels)), _ptr(coeffs),
                                       _ptr(accum), _lib.bg3(bg), _ptr(grad_out), _ptr(grad_alpha), _ptr(grad_rgb),
                                       ws.ptr, ws.nbytes, _stream(stream)), "wt_backward")
    return grad_alpha, grad_rgb


def dropped_count(ws: Workspace, stream=None) -> int:
    n = C.c_uint64(0)
    _lib.check(_lib.load().wt_dropped_count(ws.ptr, ws.nbytes, C.byref(n), _stream(stream)), "wt_dropped_count")
    return int(n.value)
