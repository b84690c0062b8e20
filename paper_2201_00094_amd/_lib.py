"""ctypes view of libwt.so (declarations in include/wt.h). Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwt.so")

WT_OK, WT_ERR_INVALID, WT_ERR_RANGE, WT_ERR_NOMEM, WT_ERR_HIP, WT_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "WT_OK", -1: "WT_ERR_INVALID", -2: "WT_ERR_RANGE", -3: "WT_ERR_NOMEM", -4: "WT_ERR_HIP",
                -5: "WT_ERR_UNSUPPORTED"}
WT_F32, WT_F16, WT_BF16, WT_E5B9G9R9 = 0, 1, 2, 3
WT_TIGHT_DEPTH = 1
WT_TEMPORAL = 2
WT_DETERMINISTIC = 4
WT_SCRATCH_BYTES = 256 << 20  # the static device array behind wt_render_noalloc
WT_MAX_FRAGMENTS = (1 << 32) - (1 << 20)  # the largest fragment count a call takes


class FrameDesc(C.Structure):
    _fields_ = [("width", C.c_uint32), ("height", C.c_uint32), ("rank", C.c_uint32), ("channels", C.c_uint32),
                ("coeff_dtype", C.c_uint32), ("flags", C.c_uint32)]


class Fragments(C.Structure):
    _fields_ = [("count", C.c_uint64), ("pixel", C.c_void_p), ("depth", C.c_void_p), ("alpha", C.c_void_p),
                ("rgb", C.c_void_p)]


_D = C.POINTER(FrameDesc)
_F = C.POINTER(Fragments)
_vp, _sz, _st = C.c_void_p, C.c_size_t, C.c_void_p

# name -> (restype, argtypes), in the order of include/wt.h
SIGNATURES = {
    "wt_workspace_bytes": (C.c_size_t, [_D, C.c_uint64]),
    "wt_bin": (C.c_int, [_D, _F, _vp, _sz, _st]),
    "wt_bin_count": (C.c_int, [_D, _F, _vp, _sz, _st]),
    "wt_bin_scatter": (C.c_int, [_D, _F, _vp, _sz, _st]),
    "wt_build_binned": (C.c_int, [_D, _vp, _vp, _sz, _st]),
    "wt_evaluate_binned": (C.c_int, [_D, _vp, _vp, _vp, _sz, _st]),
    "wt_build": (C.c_int, [_D, _F, _vp, _vp, _sz, _st]),
    "wt_evaluate": (C.c_int, [_D, _F, _vp, _vp, _vp, _sz, _st]),
    "wt_resolve": (C.c_int, [_D, _vp, C.POINTER(C.c_float), _vp, _st]),
    "wt_resolve_chromatic": (C.c_int, [_D, _vp, _vp, _vp, C.c_float, C.c_uint32, _vp, _st]),
    "wt_render": (C.c_int, [_D, _F, C.POINTER(C.c_float), _vp, _vp, _vp, _sz, _st]),
    "wt_render_noalloc": (C.c_int, [_D, _F, C.POINTER(C.c_float), _vp, _vp, _st]),
    "wt_render_binned": (C.c_int, [_D, _vp, _sz, C.POINTER(C.c_float), _vp, _vp, _st]),
    "wt_render_temporal": (C.c_int, [_D, _F, C.POINTER(C.c_float), _vp, _vp, _vp, _vp, _vp, _sz, _st]),
    "wt_render_temporal_binned": (C.c_int, [_D, _vp, _sz, C.POINTER(C.c_float), _vp, _vp, _vp, _vp, _st]),
    "wt_backward": (C.c_int, [_D, _F, _vp, _vp, C.POINTER(C.c_float), _vp, _vp, _vp, _vp, _sz, _st]),
    "wt_dropped_count": (C.c_int, [_vp, _sz, C.POINTER(C.c_uint64), _st]),
    "wt_last_error": (C.c_char_p, []),
    "wt_abi_version": (C.c_int, []),
}

_lib = None


class WTError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__("%s failed: %s (%s)" % (where, STATUS_NAMES.get(status, status), message))


def load():
    """Load libwt.so (built in-tree by ``__graft_entry__.build()``). There is no fallback: a missing library is
    an error."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libwt.so is not built (%s); run `python -m paper_2201_00094_amd._build`" % LIB_PATH)
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, where: str):
    if status != WT_OK:
        raise WTError(status, where, load().wt_last_error().decode(errors="replace"))


def desc(width, height, rank, channels=1, dtype=WT_F32, flags=0) -> FrameDesc:
    return FrameDesc(int(width), int(height), int(rank), int(channels), int(dtype), int(flags))


def bg3(bg):
    vals = [float(v) for v in bg]
    if len(vals) != 3:
        raise ValueError("background must have 3 components")
    return (C.c_float * 3)(*vals)
