"""Differentiable inviscid flux: forward = fdbb_flux, backward = the
hand-written adjoint kernel fdbb_flux_adjoint (Ubar = sum_d A_d(U)^T Fbar_d,
or A_dir(U)^T Fbar_dir for one direction), never forming A_d."""
from __future__ import annotations

import torch

from . import fdbb as F


def _as_fields(g: torch.Tensor) -> torch.Tensor:
    """Cotangents from autograd may be expanded or strided; the kernels need
    a field set with unit point stride."""
    if g.dim() == 2 and (g.shape[1] <= 1 or g.stride(1) == 1) and g.stride(0) >= g.shape[1]:
        return g
    return F.to_fields(g.contiguous())


class EulerFlux(torch.autograd.Function):
    """F = flux(U) with F of shape (K*D, n) (field r*D + d is row r of F_d),
    or F_dir of shape (K, n) when ``direction`` is given."""

    @staticmethod
    def forward(ctx, U, gamma=1.4, direction=None):
        # one direction evaluates and stores only F_direction (K fields)
        ctx.save_for_backward(U)
        ctx.gamma = gamma
        ctx.direction = direction
        return F.flux(U, gamma, direction=direction)

    @staticmethod
    def backward(ctx, gF):
        (U,) = ctx.saved_tensors
        d = -1 if ctx.direction is None else ctx.direction
        Ub = F.flux_adjoint(U, _as_fields(gF), ctx.gamma, d)
        return Ub, None, None


def euler_flux(U: torch.Tensor, gamma: float = 1.4, direction: int | None = None) -> torch.Tensor:
    return EulerFlux.apply(U, gamma, direction)
