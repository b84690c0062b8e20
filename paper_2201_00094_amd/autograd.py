"""torch.autograd.Function over the resolve: forward runs the build, evaluate and resolve kernels; backward runs
the gradient kernel (wt_backward) for alpha and rgb. Depth receives no gradient."""
from __future__ import annotations

import torch

from . import wt as _wt


class WaveletComposite(torch.autograd.Function):
    """out = WaveletComposite.apply(pixel, depth, alpha, rgb, spec, bg[, workspace])."""

    @staticmethod
    def forward(ctx, pixel, depth, alpha, rgb, spec: _wt.FrameSpec, bg, ws: _wt.Workspace = None):
        frags = _wt.Fragments(pixel, depth.detach(), alpha.detach().contiguous(), rgb.detach().contiguous())
        if ws is None:
            ws = _wt.Workspace(spec, frags.count, device=pixel.device)
        coeffs = spec.new_coeffs(device=pixel.device)
        accum = spec.new_accum(device=pixel.device)
        _wt.bin(spec, frags, ws)
        _wt.build_binned(spec, coeffs, ws)
        _wt.evaluate_binned(spec, coeffs, accum, ws)
        out = _wt.resolve(spec, accum, bg)
        ctx.save_for_backward(pixel, frags.depth, frags.alpha, frags.rgb, coeffs, accum)
        ctx.spec, ctx.bg, ctx.ws = spec, tuple(float(b) for b in bg), ws
        return out

    @staticmethod
    def backward(ctx, grad_out):
        pixel, depth, alpha, rgb, coeffs, accum = ctx.saved_tensors
        frags = _wt.Fragments(pixel, depth, alpha, rgb)
        ga, gr = _wt.backward(ctx.spec, frags, coeffs, accum, ctx.bg, grad_out.contiguous().float(), ctx.ws)
        need = ctx.needs_input_grad
        return None, None, (ga if need[2] else None), (gr if need[3] else None), None, None, None


def composite(pixel, depth, alpha, rgb, spec, bg, ws=None):
    return WaveletComposite.apply(pixel, depth, alpha, rgb, spec, bg, ws)
