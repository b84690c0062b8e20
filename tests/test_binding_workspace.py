"""The binding's record of what a workspace holds: calls over an already binned stream must use the description it
was binned with (the tile kernels read the workspace under that description's tile geometry). Driven on the CPU
with a stand-in for the library that returns a chosen status, so only the binding's own bookkeeping runs."""
import ctypes as C

import pytest
import torch

import paper_2201_00094_amd._lib as _lib
import paper_2201_00094_amd.wt as wt


class FakeLib:
    def __init__(self):
        self.fail = set()
        self.calls = []

    def __getattr__(self, name):
        if not name.startswith("wt_"):
            raise AttributeError(name)
        if name == "wt_last_error":
            return lambda: b"failed on purpose"

        def call(*args):
            self.calls.append(name)
            return _lib.WT_ERR_INVALID if name in self.fail else _lib.WT_OK
        return call


class FakeWs:
    ptr = C.c_void_p(0)
    nbytes = 1 << 20


@pytest.fixture
def fake(monkeypatch):
    lib = FakeLib()
    monkeypatch.setattr(_lib, "load", lambda: lib)
    monkeypatch.setattr(wt, "_check", lambda *a, **k: None)
    monkeypatch.setattr(wt, "_stream", lambda stream=None: C.c_void_p(0))
    return lib


def _frags(n=4):
    return wt.Fragments(torch.zeros(n, dtype=torch.int32), torch.zeros(n), torch.zeros(n), torch.zeros(n, 3))


A = wt.FrameSpec(64, 48, 3, 1, "f32")
B = wt.FrameSpec(64, 48, 4, 1, "f32")
T = wt.FrameSpec(64, 48, 3, 1, "f32", False, True)
OUT = torch.zeros(1)


def test_count_scatter_render_with_one_description(fake):
    ws, fr = FakeWs(), _frags()
    wt.bin_count(A, fr, ws)
    wt.bin_scatter(A, fr, ws)
    wt.render_binned(A, ws, (0, 0, 0), OUT)
    wt.render_binned(A, ws, (0, 0, 0), OUT)  # the binned stream serves any number of calls
    with pytest.raises(ValueError, match="binned for"):
        wt.render_binned(B, ws, (0, 0, 0), OUT)
    with pytest.raises(ValueError, match="binned for"):
        wt.render_temporal_binned(T, ws, (0, 0, 0), OUT)
    assert fake.calls == ["wt_bin_count", "wt_bin_scatter", "wt_render_binned", "wt_render_binned"]


def test_scatter_needs_a_count_with_the_same_description(fake):
    ws, fr = FakeWs(), _frags()
    with pytest.raises(ValueError, match="counted"):
        wt.bin_scatter(A, fr, ws)
    wt.bin_count(A, fr, ws)
    with pytest.raises(ValueError, match="binned for"):
        wt.bin_scatter(B, fr, ws)
    with pytest.raises(ValueError, match="no stream"):
        wt.render_binned(A, ws, (0, 0, 0), OUT)  # counted, not yet scattered
    assert fake.calls == ["wt_bin_count"]


def test_scatter_needs_a_count_of_the_same_stream(fake):
    """A count records the stream it counted (size and array addresses); a scatter of another stream under the same
    description is refused before the library is called, and the counted stream still scatters afterwards."""
    ws, fr, other, longer = FakeWs(), _frags(), _frags(), _frags(5)
    wt.bin_count(A, fr, ws)
    with pytest.raises(ValueError, match="another fragment stream"):
        wt.bin_scatter(A, other, ws)
    with pytest.raises(ValueError, match="another fragment stream"):
        wt.bin_scatter(A, longer, ws)
    wt.bin_scatter(A, fr, ws)
    wt.render_binned(A, ws, (0, 0, 0), OUT)
    assert fake.calls == ["wt_bin_count", "wt_bin_scatter", "wt_render_binned"]
    # the same arrays under a new count: the identity follows the latest count
    wt.bin_count(A, other, ws)
    with pytest.raises(ValueError, match="another fragment stream"):
        wt.bin_scatter(A, fr, ws)
    wt.bin_scatter(A, other, ws)


def test_temporal_binning_serves_only_the_temporal_description(fake):
    ws, fr = FakeWs(), _frags()
    wt.bin(T, fr, ws)
    wt.render_temporal_binned(T, ws, (0, 0, 0), OUT)
    with pytest.raises(ValueError, match="binned for"):
        wt.render_binned(A, ws, (0, 0, 0), OUT)


def test_whole_path_calls_bin_and_the_gradient_clears(fake):
    ws, fr = FakeWs(), _frags()
    wt.bin(A, fr, ws)
    wt.build_binned(A, OUT, ws)
    wt.evaluate_binned(A, OUT, OUT, ws)
    wt.backward(A, fr, OUT, OUT, (0, 0, 0), OUT, ws, grad_alpha=OUT, grad_rgb=OUT)
    with pytest.raises(ValueError, match="no stream"):
        wt.build_binned(A, OUT, ws)  # the gradient's own layout is in the workspace now
    wt.render(A, fr, (0, 0, 0), ws, out=OUT)
    wt.render_binned(A, ws, (0, 0, 0), OUT)
    wt.render_temporal(T, fr, (0, 0, 0), ws, out=OUT)
    wt.render_temporal_binned(T, ws, (0, 0, 0), OUT)
    wt.build(B, fr, OUT, ws)
    wt.evaluate_binned(B, OUT, OUT, ws)
    with pytest.raises(ValueError):
        wt.evaluate_binned(A, OUT, OUT, ws)


def test_a_failed_binning_leaves_no_usable_stream(fake):
    ws, fr = FakeWs(), _frags()
    wt.bin(A, fr, ws)
    fake.fail.add("wt_bin")
    with pytest.raises(_lib.WTError):
        wt.bin(A, fr, ws)
    with pytest.raises(ValueError, match="no stream"):
        wt.render_binned(A, ws, (0, 0, 0), OUT)
