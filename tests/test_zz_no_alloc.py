"""wt_render_noalloc (the entry point that allocates nothing: its workspace is the library's static per-GPU array)
through the C ABI, against wt_render with a caller workspace on the same inputs, on two calls in a row, the second
with a smaller frame of another rank. Contract of the parity tests: coefficients within 1e-5 relative per element
(exact zeros stay zero), composite rgb within 1e-4 absolute."""
import ctypes as C

import numpy as np
import pytest

import synth
from gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(torch, f, noalloc):
    import paper_2201_00094_amd as wt
    from paper_2201_00094_amd import _lib
    lib = _lib.load()
    spec = wt.FrameSpec(f.width, f.height, f.rank, f.channels)
    fr = wt.Fragments.from_numpy(f.pixel, f.depth, f.alpha, f.rgb)
    out = torch.full((spec.pixels, 3), float("nan"), dtype=torch.float32, device="cuda")
    coeffs = torch.full(spec.coeff_shape(), float("nan"), dtype=torch.float32, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    d = spec.c_desc()
    frags = fr.c_struct(spec.channels)
    if noalloc:
        st = lib.wt_render_noalloc(C.byref(d), C.byref(frags), _lib.bg3(f.bg), C.c_void_p(coeffs.data_ptr()),
                                   C.c_void_p(out.data_ptr()), stream)
        _lib.check(st, "wt_render_noalloc")
    else:
        ws = wt.Workspace(spec, f.count)
        st = lib.wt_render(C.byref(d), C.byref(frags), _lib.bg3(f.bg), C.c_void_p(coeffs.data_ptr()),
                           C.c_void_p(out.data_ptr()), ws.ptr, ws.nbytes, stream)
        _lib.check(st, "wt_render")
    torch.cuda.synchronize()
    return coeffs.cpu().double().numpy(), out.cpu().double().numpy()


def _assert_same(a, b):
    (ca, oa), (cb, ob) = a, b
    zero = cb == 0
    assert (ca[zero] == 0).all(), "a coefficient that is exactly zero through wt_render is not zero"
    assert (np.abs(ca - cb) <= 1e-5 * np.abs(cb)).all(), float(np.nanmax(np.abs(ca - cb) / np.maximum(np.abs(cb), 1e-30)))
    assert np.isfinite(oa).all()
    assert np.abs(oa - ob).max() <= 1e-4


def test_noalloc_matches_render_twice(torch_dev):
    big = synth.frame_c1(seed=11, width=640, height=360, rank=3, mean=12.0)
    small = synth.frame_c1(seed=12, width=157, height=93, rank=4, mean=6.0)
    from paper_2201_00094_amd import _lib
    for name, f in (("first, 640x360 rank 3", big), ("second, 157x93 rank 4", small)):
        say("case wt_render_noalloc", name, "fragments", f.count)
        got = _run(torch_dev, f, noalloc=True)
        ref = _run(torch_dev, f, noalloc=False)
        _assert_same(got, ref)
    assert small.count < big.count
    # the static array's limit: refused before anything is enqueued
    lib = _lib.load()
    d = _lib.desc(1920, 1080, 3)
    too_many = _lib.Fragments(_lib.WT_SCRATCH_BYTES // 28 + 1, 8, 8, 8, 8)
    assert lib.wt_render_noalloc(C.byref(d), C.byref(too_many), _lib.bg3((0, 0, 0)), None, C.c_void_p(8),
                                 None) == _lib.WT_ERR_RANGE
    assert "scratch" in lib.wt_last_error().decode()
