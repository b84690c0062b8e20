"""Shared helpers for the GPU parity tests: move a synthetic frame to the device, run the library, compare with
the oracle under the parity contract."""
import sys

import numpy as np


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def device_frags(f, device="cuda"):
    import paper_2201_00094_amd as wt
    return wt.Fragments.from_numpy(f.pixel, f.depth, f.alpha, f.rgb, device=device)


def spec_of(f, dtype="f32", rank=None, tight=False):
    import paper_2201_00094_amd as wt
    return wt.FrameSpec(f.width, f.height, f.rank if rank is None else rank, f.channels, dtype, tight)


def gpu_render(f, dtype="f32", rank=None, want_coeffs=True, tight=False):
    import torch
    import paper_2201_00094_amd as wt
    spec = spec_of(f, dtype, rank, tight)
    fr = device_frags(f)
    ws = wt.Workspace(spec, f.count)
    coeffs = spec.new_coeffs() if want_coeffs else None
    out = wt.render(spec, fr, f.bg, ws, coeffs=coeffs)
    torch.cuda.synchronize()
    res = {"out": out.cpu().double().numpy(), "dropped": wt.dropped_count(ws)}
    if want_coeffs:
        res.update(_coeffs_out(coeffs, dtype))
    return res


def _coeffs_out(coeffs, dtype):
    if dtype == "e5b9g9r9":
        return {"words": coeffs.cpu().numpy().view(np.uint32)}
    return {"coeffs": coeffs.float().cpu().double().numpy()}


def e5_decode(orc, words):
    """Signed coefficients [P, 3, M] of E5B9G9R9 words [P, M], decoded with the oracle's unpacking (coefficient 0
    is >= 0, the others <= 0)."""
    P, M = words.shape
    out = np.zeros((P, 3, M))
    for p in range(P):
        for m in range(M):
            v = orc.unpack_e5b9g9r9(int(words[p, m]))
            out[p, :, m] = v if m == 0 else tuple(-x for x in v)
    return out


def gpu_passes(f, dtype="f32", rank=None, chunks=1, tight=False):
    """Separate build / evaluate / resolve calls, each taking the raw stream (optionally in chunks)."""
    import torch
    import paper_2201_00094_amd as wt
    spec = spec_of(f, dtype, rank, tight)
    coeffs = spec.new_coeffs()
    accum = spec.new_accum()
    bounds = np.linspace(0, f.count, chunks + 1).astype(np.int64)
    ws = wt.Workspace(spec, max(1, int(np.diff(bounds).max())))
    parts = [device_frags(f.subset(np.arange(bounds[i], bounds[i + 1]))) for i in range(chunks)]
    for p in parts:
        wt.build(spec, p, coeffs, ws)
    for p in parts:
        wt.evaluate(spec, p, coeffs, accum, ws)
    out = wt.resolve(spec, accum, f.bg)
    torch.cuda.synchronize()
    res = {"accum": accum.cpu().double().numpy(), "out": out.cpu().double().numpy()}
    res.update(_coeffs_out(coeffs, dtype))
    return res


def oracle_frame(orc, f, rank=None, storage="exact", mask=None, want=("coeffs", "accum", "suma", "out"), tight=False):
    return orc.resolve(f.width, f.height, f.rank if rank is None else rank, f.pixel, f.depth, f.alpha, f.rgb,
                       bg=f.bg, channels=f.channels, mask=mask, want=want, storage=storage, tight=tight)


def assert_coeffs(g, o, rel=1e-5, sel=None, what="coeffs", atol=0.0):
    """Every element within rel * |oracle| + atol; exact zeros stay zero. atol is the storage format's smallest
    step (its subnormal spacing) where a reduced storage is compared: below the smallest normal value one step is
    that absolute spacing, not a fixed fraction of the value."""
    g = g.reshape(o.shape)
    if sel is not None:
        g, o = g[sel], o[sel]
    zero = o == 0
    assert (g[zero] == 0).all(), "%s: %d oracle zeros are non-zero on the GPU" % (what, int((g[zero] != 0).sum()))
    err = np.abs(g - o)
    bad = err > rel * np.abs(o) + atol
    if bad.any():
        i = np.unravel_index(np.argmax(err / np.maximum(np.abs(o), 1e-300)), o.shape)
        raise AssertionError("%s: %d elements beyond %.1e relative; worst at %s: gpu %r oracle %r" %
                             (what, int(bad.sum()), rel, i, g[i], o[i]))


def assert_close_abs(g, o, atol, sel=None, what="out"):
    g = g.reshape(o.shape)
    if sel is not None:
        g, o = g[sel], o[sel]
    err = np.abs(g - o)
    if not (err <= atol).all():
        i = np.unravel_index(np.argmax(err), o.shape)
        raise AssertionError("%s: max abs error %.3e > %.1e at %s: gpu %r oracle %r" % (what, err.max(), atol, i, g[i],
                                                                                       o[i]))
    return float(err.max()) if err.size else 0.0


def accum_to_oracle_layout(acc, channels):
    """GPU accum [P][4] or [P][8] -> (S [P][3], suma [P][C])."""
    if channels == 1:
        return acc[:, :3], acc[:, 3:4]
    return acc[:, :3], acc[:, 4:7]


def storage_out_bound(orc, rank, coeffs, accum, channels, rel, floor=1e-4, atol=0.0):
    """Per-pixel bound on |composite(GPU) - composite(oracle)| when both store coefficients at reduced precision
    and may round one coefficient to neighbouring storage values (FP32 accumulation on one side, FP64 on the other,
    straddling a rounding midpoint). The composite is S + bg exp(-sum a) (section 2.1, steps 3-4); the sum of
    absorbances is exact on both sides, so storage reaches it only through each fragment's visibility
    V = exp(-A~(z)). A~ interpolates between 0 and the cell averages (section 2.3.2), so |dA~| is at most
    E = max_j sum_m |dAbar_j/dc_m| |dc_m| with |dc_m| <= rel |c_m| + atol, and every V, hence S, moves by a factor within
    exp(+-E): |d out_q| <= (exp(E) - 1) S_q. ``floor`` covers FP32 arithmetic. coeffs [P][C*M] or [P][C][M]
    (oracle, at the reduced storage), accum [P][3] (oracle); returns [P][3]."""
    M = 1 << (rank + 1)
    jac = np.abs(np.stack([orc.cells_one(rank, np.eye(M)[m]) for m in range(M)], axis=1))  # [j][m]
    c = np.abs(np.asarray(coeffs, dtype=np.float64).reshape(-1, channels, M))
    E = ((c * rel + atol) @ jac.T).max(axis=2)  # [P][C]
    if channels == 1:
        E = np.repeat(E, 3, axis=1)
    return np.expm1(E) * np.abs(np.asarray(accum, dtype=np.float64).reshape(-1, 3)) + floor


# smallest step of each reduced storage format (its subnormal spacing)
STORAGE_ATOL = {"f32": 0.0, "f16": 2.0 ** -24, "bf16": 2.0 ** -133}


def assert_within(g, o, tol, sel=None, what="out"):
    """|g - o| <= tol elementwise (tol broadcast to o's shape); returns the largest error and the largest ratio of
    error to bound."""
    g = g.reshape(o.shape)
    tol = np.broadcast_to(tol, o.shape)
    if sel is not None:
        g, o, tol = g[sel], o[sel], tol[sel]
    err = np.abs(g - o)
    if not (err <= tol).all():
        i = np.unravel_index(np.argmax(err / tol), o.shape)
        raise AssertionError("%s: error %.3e > bound %.3e at %s: gpu %r oracle %r" % (what, err[i], tol[i], i, g[i],
                                                                                       o[i]))
    return (float(err.max()) if err.size else 0.0), (float((err / tol).max()) if err.size else 0.0)
