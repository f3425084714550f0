"""torch.autograd wrapper of the chi0 application.

Forward runs lgw_chi0_apply; backward runs lgw_chi0_apply_vjp (adjoint
Sternheimer solves at the conjugate frequency plus the orbital response), so
both the perturbing potential and the local potential get gradients.
"""
from __future__ import annotations

import torch


class Chi0Apply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V_loc, dV, lg, z):
        ctx.lg = lg
        ctx.z = z
        ctx.save_for_backward(dV)
        return lg.chi0_apply(dV, z)

    @staticmethod
    def backward(ctx, g):
        (dV,) = ctx.saved_tensors
        need_V, need_dV = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gdV, gV = ctx.lg.chi0_apply_vjp(dV, ctx.z, g.contiguous(), want_dV=need_dV,
                                        want_V=need_V)
        if gV is not None:
            gV = gV.reshape(ctx.lg.N, ctx.lg.N, ctx.lg.N)
        if gdV is not None:
            gdV = gdV.reshape(dV.shape)
        return gV, gdV, None, None


def chi0_apply(lg, V_loc: torch.Tensor, dV: torch.Tensor, z) -> torch.Tensor:
    """dn = chi0(z) dV with gradients to V_loc (the potential `lg` was set up
    with, [N, N, N] float64) and to dV."""
    return Chi0Apply.apply(V_loc, dV, lg, z)
