"""torch.autograd wrappers of the chi0 application and of the Lanczos loss.

Chi0Apply: forward runs lgw_chi0_apply; backward runs lgw_chi0_apply_vjp
(adjoint Sternheimer solves at the conjugate frequency plus the orbital
response), so both the perturbing potential and the local potential get
gradients.

LanczosLoss: sum_z log det(I + E(z)) over the Lanczos-projected dielectric
matrix; lgw_lanczos_loss_vjp returns the loss and its gradient together, so
forward keeps the gradient for backward.
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


class LanczosLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, V_loc, lg, q0, k, z):
        loss, gV, _ = lg.lanczos_loss_vjp(q0, k, z, want_V=ctx.needs_input_grad[0])
        ctx.save_for_backward(gV.reshape(V_loc.shape) if gV is not None else None)
        return torch.tensor(loss, dtype=torch.float64, device=V_loc.device)

    @staticmethod
    def backward(ctx, g):
        (gV,) = ctx.saved_tensors
        return (g * gV if gV is not None else None), None, None, None, None


def lanczos_loss(lg, V_loc: torch.Tensor, q0: torch.Tensor, k: int, z) -> torch.Tensor:
    """sum_z log det(I + Q^H (eps(z)-1) Q), Q from k Lanczos steps on eps(0)-1,
    differentiable with respect to V_loc (the potential `lg` was set up with)."""
    return LanczosLoss.apply(V_loc, lg, q0, k, z)
