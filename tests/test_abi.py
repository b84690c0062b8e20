"""Host-side checks of the C ABI (no GPU): every symbol of include/wt.h is exported, and argument validation
fails before anything is enqueued."""
import ctypes as C
import os
import re

import pytest

from paper_2201_00094_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wt.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(wt_[a-z_0-9]+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_header_declares_the_path():
    names = header_functions()
    for n in ("wt_build", "wt_evaluate", "wt_resolve", "wt_render", "wt_backward", "wt_bin", "wt_workspace_bytes",
              "wt_last_error", "wt_dropped_count"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in header_functions():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, name


def test_abi_version(lib):
    assert lib.wt_abi_version() == 2


def test_workspace_bytes(lib):
    d = _lib.desc(1920, 1080, 3)
    a = lib.wt_workspace_bytes(C.byref(d), 0)
    b = lib.wt_workspace_bytes(C.byref(d), 1000)
    c = lib.wt_workspace_bytes(C.byref(d), 132_710_400)
    assert 0 < a < b < c
    assert c >= 132_710_400 * 28  # binned copy: pixel, depth, alpha, rgb, stream index
    assert lib.wt_workspace_bytes(C.byref(_lib.desc(16, 16, 11)), 10) == 0  # rank > 10
    assert lib.wt_workspace_bytes(C.byref(_lib.desc(16, 16, 3, channels=2)), 10) == 0
    assert lib.wt_workspace_bytes(None, 10) == 0
    assert lib.wt_workspace_bytes(C.byref(_lib.desc(16, 16, 3)), 1 << 32) == 0
    # the fragment limit: 2^32 - 2^20 fragments are sized, one more is not
    assert lib.wt_workspace_bytes(C.byref(_lib.desc(16, 16, 3)), _lib.WT_MAX_FRAGMENTS) >= _lib.WT_MAX_FRAGMENTS * 28
    assert lib.wt_workspace_bytes(C.byref(_lib.desc(16, 16, 3)), _lib.WT_MAX_FRAGMENTS + 1) == 0


def _err(lib):
    return lib.wt_last_error().decode()


def test_validation_errors_before_any_launch(lib):
    d = _lib.desc(64, 64, 3)
    f = _lib.Fragments(10, None, None, None, None)
    ws = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.wt_bin(None, C.byref(f), ws, 1 << 20, None) == _lib.WT_ERR_INVALID
    assert "desc" in _err(lib)
    assert lib.wt_bin(C.byref(d), C.byref(f), ws, 1 << 20, None) == _lib.WT_ERR_INVALID
    assert "NULL" in _err(lib)
    big = _lib.Fragments(1 << 32, 1, 1, 1, 1)
    assert lib.wt_bin(C.byref(d), C.byref(big), ws, 1 << 20, None) == _lib.WT_ERR_RANGE
    over = _lib.Fragments(_lib.WT_MAX_FRAGMENTS + 1, 1, 1, 1, 1)
    assert lib.wt_bin(C.byref(d), C.byref(over), ws, 1 << 20, None) == _lib.WT_ERR_RANGE
    assert "WT_MAX_FRAGMENTS" in _err(lib)
    at_limit = _lib.Fragments(_lib.WT_MAX_FRAGMENTS, 1, 1, 1, 1)
    assert lib.wt_bin(C.byref(d), C.byref(at_limit), ws, 1 << 20, None) == _lib.WT_ERR_RANGE
    assert "workspace" in _err(lib)  # the count passes; the 1 MiB workspace does not
    ok = _lib.Fragments(10, 8, 8, 8, 8)
    assert lib.wt_bin(C.byref(d), C.byref(ok), ws, 16, None) == _lib.WT_ERR_RANGE
    assert "workspace" in _err(lib)
    assert lib.wt_bin(C.byref(d), C.byref(ok), None, 1 << 30, None) == _lib.WT_ERR_INVALID
    assert lib.wt_bin(C.byref(_lib.desc(0, 5, 3)), C.byref(ok), ws, 1 << 30, None) == _lib.WT_ERR_INVALID
    assert lib.wt_bin(C.byref(_lib.desc(65536, 65536, 3)), C.byref(ok), ws, 1 << 30, None) == _lib.WT_ERR_RANGE
    assert lib.wt_bin(C.byref(_lib.desc(8, 8, 3, 1, 7)), C.byref(ok), ws, 1 << 30, None) == _lib.WT_ERR_INVALID
    # packed E5B9G9R9 storage: three channels only, rank <= 4
    e5 = _lib.WT_E5B9G9R9
    assert lib.wt_bin(C.byref(_lib.desc(8, 8, 3, 1, e5)), C.byref(ok), ws, 1 << 30, None) == _lib.WT_ERR_INVALID
    assert lib.wt_bin(C.byref(_lib.desc(8, 8, 5, 3, e5)), C.byref(ok), ws, 1 << 30, None) == _lib.WT_ERR_UNSUPPORTED
    assert lib.wt_workspace_bytes(C.byref(_lib.desc(8, 8, 4, 3, e5)), 10) > 0
    # flags: WT_TIGHT_DEPTH and WT_TEMPORAL are defined, and exclude each other
    assert lib.wt_bin(C.byref(_lib.desc(8, 8, 3, 1, 0, 8)), C.byref(ok), ws, 1 << 30, None) == _lib.WT_ERR_INVALID
    assert lib.wt_workspace_bytes(C.byref(_lib.desc(8, 8, 3, 1, 0, _lib.WT_TIGHT_DEPTH)), 10) > 0
    assert lib.wt_workspace_bytes(C.byref(_lib.desc(8, 8, 3, 1, 0, _lib.WT_TEMPORAL)), 10) > 0
    both = _lib.WT_TIGHT_DEPTH | _lib.WT_TEMPORAL
    assert lib.wt_bin(C.byref(_lib.desc(8, 8, 3, 1, 0, both)), C.byref(ok), ws, 1 << 30, None) == \
        _lib.WT_ERR_UNSUPPORTED
    assert lib.wt_bin(C.byref(_lib.desc(8, 8, 5, 1, 0, _lib.WT_TEMPORAL)), C.byref(ok), ws, 1 << 30, None) == \
        _lib.WT_ERR_UNSUPPORTED
    bg = _lib.bg3((0, 0, 0))
    assert lib.wt_resolve(C.byref(d), None, bg, ws, None) == _lib.WT_ERR_INVALID
    assert lib.wt_render(C.byref(d), C.byref(ok), None, None, ws, ws, 1 << 30, None) == _lib.WT_ERR_INVALID
    assert lib.wt_build_binned(C.byref(d), None, ws, 1 << 30, None) == _lib.WT_ERR_INVALID
    assert lib.wt_evaluate_binned(C.byref(d), ws, None, ws, 1 << 30, None) == _lib.WT_ERR_INVALID
    assert lib.wt_backward(C.byref(d), C.byref(ok), ws, ws, bg, None, ws, ws, ws, 1 << 30, None) == \
        _lib.WT_ERR_INVALID
    # the one-pass render: a WT_TEMPORAL description, and no in-place update through a reprojection map
    assert lib.wt_render_temporal(C.byref(d), C.byref(ok), bg, None, None, ws, ws, ws, 1 << 30, None) == \
        _lib.WT_ERR_INVALID
    assert "WT_TEMPORAL" in _err(lib)
    dt = _lib.desc(64, 64, 3, 1, 0, _lib.WT_TEMPORAL)
    assert lib.wt_render_temporal_binned(C.byref(dt), ws, 1 << 30, bg, ws, ws, ws, ws, None) == _lib.WT_ERR_INVALID
    assert "prev_pixel" in _err(lib)
    assert lib.wt_render_temporal_binned(C.byref(dt), ws, 1 << 30, None, None, None, None, ws, None) == \
        _lib.WT_ERR_INVALID
    assert lib.wt_render_temporal_binned(C.byref(dt), ws, 16, bg, None, None, None, ws, None) == _lib.WT_ERR_RANGE
    # chromatic composite: odd taps in 3..63, finite dispersion, no NULL arrays
    for taps in (1, 2, 4, 65):
        assert lib.wt_resolve_chromatic(C.byref(d), ws, ws, ws, 0.5, taps, ws, None) == _lib.WT_ERR_INVALID
    assert "taps" in _err(lib)
    assert lib.wt_resolve_chromatic(C.byref(d), ws, ws, ws, float("nan"), 5, ws, None) == _lib.WT_ERR_INVALID
    assert lib.wt_resolve_chromatic(C.byref(d), ws, None, ws, 0.5, 5, ws, None) == _lib.WT_ERR_INVALID
    assert lib.wt_resolve_chromatic(C.byref(d), C.c_void_p(0x1004), ws, ws, 0.5, 5, ws, None) == _lib.WT_ERR_INVALID
    assert "aligned" in _err(lib)
    n = C.c_uint64(0)
    assert lib.wt_dropped_count(None, 1 << 20, C.byref(n), None) == _lib.WT_ERR_INVALID
    assert lib.wt_dropped_count(ws, 8, C.byref(n), None) == _lib.WT_ERR_RANGE


def test_python_binding_rejects_host_tensors():
    import torch
    import paper_2201_00094_amd as wt
    spec = wt.FrameSpec(8, 8, 3)
    fr = wt.Fragments(torch.zeros(4, dtype=torch.int32), torch.zeros(4), torch.zeros(4), torch.zeros(4, 3))
    with pytest.raises(TypeError):
        fr.c_struct(1)
    with pytest.raises(ValueError):
        wt.FrameSpec(8, 8, 3, dtype="f64").c_desc()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No fallback: without libwt.so every entry point raises instead of computing anything elsewhere."""
    import paper_2201_00094_amd as wt
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libwt.so"))
    with pytest.raises(RuntimeError, match="not built"):
        _lib.load()
    with pytest.raises(RuntimeError, match="not built"):
        wt.workspace_bytes(wt.FrameSpec(8, 8, 3), 10)


def test_product_never_touches_the_oracle():
    """The product package and its C sources neither import, load nor name the oracle (test infrastructure)."""
    pkg = os.path.join(ROOT, "paper_2201_00094_amd")
    for base, _, files in os.walk(pkg):
        for name in files:
            if name.endswith((".py", ".hip", ".h", ".cpp")):
                with open(os.path.join(base, name), encoding="utf-8") as fh:
                    assert "oracle" not in fh.read().lower(), os.path.join(base, name)
    with open(HEADER, encoding="utf-8") as fh:
        assert "oracle" not in fh.read().lower()


def test_every_description_sizes_and_validates(lib):
    """Every rank, channel count, storage type and flag combination over frame sizes up to the 2^32-pixel limit:
    the workspace size is 0 exactly for descriptions the validation rejects, grows with the fragment count and
    holds the binned copy, and each binning or one-pass call with a 16-byte workspace stops at validation (range or
    unsupported, never a launch)."""
    sizes = [(1, 1), (7, 5), (1920, 1080), (3840, 2160), (65535, 65537)]
    counts = [0, 1, 1_000_000, _lib.WT_MAX_FRAGMENTS]
    ok = _lib.Fragments(10, 8, 8, 8, 8)
    ws = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    bg = _lib.bg3((0, 0, 0))
    errs = (_lib.WT_ERR_RANGE, _lib.WT_ERR_UNSUPPORTED)
    n_valid = 0
    for rank in range(11):
        for ch in (1, 3):
            for dt in (_lib.WT_F32, _lib.WT_F16, _lib.WT_BF16, _lib.WT_E5B9G9R9):
                for fl in (0, _lib.WT_TIGHT_DEPTH, _lib.WT_TEMPORAL):
                    for w, h in sizes:
                        d = _lib.desc(w, h, rank, ch, dt, fl)
                        got = [lib.wt_workspace_bytes(C.byref(d), n) for n in counts]
                        st = lib.wt_bin(C.byref(d), C.byref(ok), ws, 16, None)
                        if got[0] == 0:
                            assert all(g == 0 for g in got)
                            assert st in (_lib.WT_ERR_INVALID, _lib.WT_ERR_UNSUPPORTED), (rank, ch, dt, fl, w, h)
                            continue
                        n_valid += 1
                        assert got == sorted(got) and got[0] < got[2], (rank, ch, dt, fl, w, h, got)
                        assert got[2] >= 1_000_000 * 28 and got[3] >= _lib.WT_MAX_FRAGMENTS * 28
                        assert st in errs, (rank, ch, dt, fl, w, h, st, _err(lib))
                        if fl == _lib.WT_TEMPORAL:
                            st = lib.wt_render_temporal_binned(C.byref(d), ws, 16, bg, None, None, None, ws, None)
                            assert st in errs, (rank, ch, dt, w, h, st, _err(lib))
    assert n_valid > 500


def test_noalloc_refuses_frames_beyond_its_array(lib):
    # validation and the size limit come before the library looks up its static array (no GPU needed)
    d = _lib.desc(1920, 1080, 3)
    ok_ptr = C.c_void_p(8)
    too_many = _lib.Fragments(_lib.WT_SCRATCH_BYTES // 28 + 1, 8, 8, 8, 8)
    assert lib.wt_render_noalloc(C.byref(d), C.byref(too_many), _lib.bg3((0, 0, 0)), None, ok_ptr,
                                 None) == _lib.WT_ERR_RANGE
    assert "scratch" in _err(lib)
    assert lib.wt_render_noalloc(None, C.byref(too_many), _lib.bg3((0, 0, 0)), None, ok_ptr,
                                 None) == _lib.WT_ERR_INVALID
    assert lib.wt_render_noalloc(C.byref(d), C.byref(too_many), None, None, ok_ptr, None) == _lib.WT_ERR_INVALID
    assert lib.wt_render_noalloc(C.byref(d), C.byref(too_many), _lib.bg3((0, 0, 0)), None, None,
                                 None) == _lib.WT_ERR_INVALID
    # three channels at 4K bin in two levels (two record copies): about a quarter of the one-channel limit
    d3 = _lib.desc(3840, 2160, 3, channels=3)
    n3 = _lib.Fragments(_lib.WT_SCRATCH_BYTES // 72 + 1, 8, 8, 8, 8)
    assert lib.wt_render_noalloc(C.byref(d3), C.byref(n3), _lib.bg3((0, 0, 0)), None, ok_ptr,
                                 None) == _lib.WT_ERR_RANGE


def test_binding_constants_match_the_header():
    """The numeric #defines of wt.h (fragment limit, scratch size, flags) are the binding's constants."""
    with open(os.path.join(ROOT, "include", "wt.h")) as fh:
        text = fh.read()
    defs = dict(re.findall(r"^#define (WT_[A-Z_0-9]+) (.+)$", text, flags=re.M))
    val = {"WT_MAX_FRAGMENTS": int(defs["WT_MAX_FRAGMENTS"].rstrip("ul")),
           "WT_SCRATCH_BYTES": (lambda m: int(m[0]) << int(m[1]))(
               re.fullmatch(r"\(\(size_t\)(\d+) << (\d+)\)", defs["WT_SCRATCH_BYTES"]).groups()),
           "WT_TIGHT_DEPTH": int(defs["WT_TIGHT_DEPTH"].rstrip("u")),
           "WT_TEMPORAL": int(defs["WT_TEMPORAL"].rstrip("u")),
           "WT_DETERMINISTIC": int(defs["WT_DETERMINISTIC"].rstrip("u"))}
    for name, v in val.items():
        assert getattr(_lib, name) == v, name
    assert _lib.WT_MAX_FRAGMENTS == (1 << 32) - (1 << 20)

