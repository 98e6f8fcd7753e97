"""torch.autograd wrapper of the forward (hk_opacity) and adjoint (hk_opacity_backward) calls.

The differentiable inputs are T, ln P and the per-line S_ref, gamma_ref and n (float64 tensors
in the caller's line order, passed to the library as per-line overrides). Strengths and widths
are recomputed by the adjoint kernel, nothing but the inputs is saved between the passes."""
import math

import torch

from . import _lib


class HkOpacityFn(torch.autograd.Function):
    """k = HkOpacityFn.apply(T, lnP, S_ref, gamma_ref, n_exp, lines, grid, cutoff).

    T, lnP: 0-d float64 tensors; S_ref, gamma_ref, n_exp: float64 device tensors of n_lines
    (or None: the values held by ``lines`` are used and get no gradient); returns float32 k."""

    @staticmethod
    def forward(ctx, T, lnP, S_ref, gamma_ref, n_exp, lines, grd, cutoff):
        Tv, Pv = float(T), math.exp(float(lnP))
        ovr = None
        if S_ref is not None or gamma_ref is not None or n_exp is not None:
            ovr = tuple(None if t is None else t.detach().contiguous() for t in (S_ref, gamma_ref, n_exp))
        k = _lib.hk_opacity(lines, Tv, Pv, grd, cutoff, ovr=ovr)
        ctx.lines, ctx.grd, ctx.cutoff, ctx.Tv, ctx.Pv, ctx.ovr = lines, grd, cutoff, Tv, Pv, ovr
        ctx.shapes = (T, lnP)
        return k

    @staticmethod
    def backward(ctx, gk):
        T, lnP = ctx.shapes
        out2, dS, dg, dn = _lib.hk_opacity_backward(ctx.lines, ctx.Tv, ctx.Pv, ctx.grd, ctx.cutoff,
                                                    gk.detach().to(torch.float32).contiguous(), ovr=ctx.ovr)
        dT = out2[0].to(device=T.device, dtype=T.dtype) if ctx.needs_input_grad[0] else None
        dlnP = out2[1].to(device=lnP.device, dtype=lnP.dtype) if ctx.needs_input_grad[1] else None
        gS = dS if ctx.needs_input_grad[2] else None
        gg = dg.to(torch.float64) if ctx.needs_input_grad[3] else None
        gn = dn.to(torch.float64) if ctx.needs_input_grad[4] else None
        return dT, dlnP, gS, gg, gn, None, None, None


def opacity(lines, T, lnP, grd, cutoff, S_ref=None, gamma_ref=None, n_exp=None):
    """Differentiable k(nu) on ``grd`` (see HkOpacityFn)."""
    return HkOpacityFn.apply(T, lnP, S_ref, gamma_ref, n_exp, lines, grd, cutoff)
