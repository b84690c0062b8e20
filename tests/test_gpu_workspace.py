"""Workspace misuse through the C ABI is refused on the device and reported, never read past the layout: a binned
call under another description than the stream was binned with, and a scatter that does not belong to the count
before it (another stream, or the same arrays whose contents changed in between). Each case leaves the outputs
untouched, reports the misuse once through wt_dropped_count, and a correct call afterwards gives the right result.
The conditions are made on the host side (arguments and array contents); every kernel exits normally."""
import ctypes as C

import numpy as np
import pytest

import synth
from gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_00094_amd import _lib
    return torch, _lib, _lib.load()


def _frags(torch, _lib, f):
    t = [torch.from_numpy(a).cuda() for a in (f.pixel.view(np.int32), f.depth, f.alpha, f.rgb)]
    return t, _lib.Fragments(f.count, *(x.data_ptr() for x in t))


def _status(lib, ws, nb, stream):
    n = C.c_uint64(0)
    st = lib.wt_dropped_count(C.c_void_p(ws.data_ptr()), nb, C.byref(n), stream)
    return st, lib.wt_last_error().decode()


def _render_binned(lib, _lib, d, ws, nb, f, out, stream):
    st = lib.wt_render_binned(C.byref(d), C.c_void_p(ws.data_ptr()), nb, _lib.bg3(f.bg), None,
                              C.c_void_p(out.data_ptr()), stream)
    assert st == _lib.WT_OK  # the host cannot see the mismatch: the device refuses


def test_binned_call_under_another_description(env, orc):
    torch, _lib, lib = env
    f = synth.frame_c1(seed=3, width=96, height=64)
    say("case workspace: render_binned under another description")
    d3, d4 = _lib.desc(96, 64, 3), _lib.desc(96, 64, 4)
    nb = max(lib.wt_workspace_bytes(C.byref(d3), f.count), lib.wt_workspace_bytes(C.byref(d4), f.count))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    keep, fr = _frags(torch, _lib, f)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.wt_bin(C.byref(d3), C.byref(fr), C.c_void_p(ws.data_ptr()), nb, stream) == _lib.WT_OK
    out = torch.full((96 * 64, 3), float("nan"), device="cuda")
    _render_binned(lib, _lib, d4, ws, nb, f, out, stream)  # rank 4 over a rank-3 binning
    torch.cuda.synchronize()
    assert bool(torch.isnan(out).all()), "a refused call wrote outputs"
    st, msg = _status(lib, ws, nb, stream)
    assert st == _lib.WT_ERR_INVALID and "no complete binning" in msg
    assert _status(lib, ws, nb, stream)[0] == _lib.WT_OK  # reported once
    # the same binned stream under its own description
    _render_binned(lib, _lib, d3, ws, nb, f, out, stream)
    torch.cuda.synchronize()
    o = orc.resolve(f.width, f.height, 3, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg, want=("out",))["out"]
    assert np.abs(out.cpu().double().numpy() - o).max() <= 1e-4
    assert _status(lib, ws, nb, stream)[0] == _lib.WT_OK


def test_scatter_that_does_not_follow_its_count(env, orc):
    torch, _lib, lib = env
    f = synth.frame_c1(seed=4, width=80, height=48)
    g = synth.frame_c1(seed=5, width=80, height=48)
    say("case workspace: scatter of another stream, and of a stream changed after its count")
    d = _lib.desc(80, 48, 3)
    nb = lib.wt_workspace_bytes(C.byref(d), max(f.count, g.count))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    wsp = C.c_void_p(ws.data_ptr())
    kf, ff = _frags(torch, _lib, f)
    kg, fg = _frags(torch, _lib, g)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = torch.full((80 * 48, 3), float("nan"), device="cuda")
    # count f, scatter g
    assert lib.wt_bin_count(C.byref(d), C.byref(ff), wsp, nb, stream) == _lib.WT_OK
    assert lib.wt_bin_scatter(C.byref(d), C.byref(fg), wsp, nb, stream) == _lib.WT_OK
    _render_binned(lib, _lib, d, ws, nb, f, out, stream)
    torch.cuda.synchronize()
    assert bool(torch.isnan(out).all())
    st, msg = _status(lib, ws, nb, stream)
    assert st == _lib.WT_ERR_INVALID and "scatter" in msg and "no complete binning" in msg
    # count f, then move every fragment of f into pixel 0 (one tile gets far more than counted), scatter f
    assert lib.wt_bin_count(C.byref(d), C.byref(ff), wsp, nb, stream) == _lib.WT_OK
    kf[0].zero_()
    assert lib.wt_bin_scatter(C.byref(d), C.byref(ff), wsp, nb, stream) == _lib.WT_OK
    _render_binned(lib, _lib, d, ws, nb, f, out, stream)
    torch.cuda.synchronize()
    assert bool(torch.isnan(out).all())
    st, msg = _status(lib, ws, nb, stream)
    assert st == _lib.WT_ERR_INVALID and "more fragments for a tile" in msg
    # a scatter run twice after one count
    kf[0].copy_(torch.from_numpy(f.pixel.view(np.int32)).cuda())
    assert lib.wt_bin_count(C.byref(d), C.byref(ff), wsp, nb, stream) == _lib.WT_OK
    assert lib.wt_bin_scatter(C.byref(d), C.byref(ff), wsp, nb, stream) == _lib.WT_OK
    assert lib.wt_bin_scatter(C.byref(d), C.byref(ff), wsp, nb, stream) == _lib.WT_OK
    _render_binned(lib, _lib, d, ws, nb, f, out, stream)
    torch.cuda.synchronize()
    assert bool(torch.isnan(out).all())
    assert _status(lib, ws, nb, stream)[0] == _lib.WT_ERR_INVALID
    # and the proper sequence still works
    assert lib.wt_bin_count(C.byref(d), C.byref(ff), wsp, nb, stream) == _lib.WT_OK
    assert lib.wt_bin_scatter(C.byref(d), C.byref(ff), wsp, nb, stream) == _lib.WT_OK
    _render_binned(lib, _lib, d, ws, nb, f, out, stream)
    torch.cuda.synchronize()
    o = orc.resolve(f.width, f.height, 3, f.pixel, f.depth, f.alpha, f.rgb, bg=f.bg, want=("out",))["out"]
    assert np.abs(out.cpu().double().numpy() - o).max() <= 1e-4
    assert _status(lib, ws, nb, stream)[0] == _lib.WT_OK
