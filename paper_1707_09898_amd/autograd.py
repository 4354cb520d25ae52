"""Differentiation form: the stray field as a torch.autograd.Function.

forward:  H = -N (*) (chi rho^p M0)              (tof_field, three components)
backward: dL/drho = chi p rho^(p-1) M0 . (-N (*) dL/dH)   (tof_adjoint)

The backward is the hand-written adjoint convolution: the stray-field
operator is self-adjoint (Sec. Methodology: the adjoint problem has the form
of the forward one), so the vector-Jacobian product is one more convolution
with the same tensor spectra followed by the penalization derivative.  Any
differentiable torch expression of H then gets dJ/drho through PyTorch's
tape, e.g. J = mean over a sensor box of |H - H*|^2.
"""
from __future__ import annotations

import torch


class StrayField(torch.autograd.Function):
    """H = field(rho) with a hand-written backward through the adjoint."""

    @staticmethod
    def forward(ctx, rho: torch.Tensor, engine) -> torch.Tensor:
        H = engine.field(rho.contiguous(), comps=7)
        ctx.save_for_backward(rho)
        ctx.engine = engine
        return H

    @staticmethod
    def backward(ctx, gH: torch.Tensor):
        (rho,) = ctx.saved_tensors
        grad = ctx.engine.adjoint(rho.contiguous(), gH.contiguous())
        return grad, None


def stray_field(rho: torch.Tensor, engine) -> torch.Tensor:
    """Differentiable H [3][nz][ny][nx] of the density rho [nz][ny][nx]."""
    return StrayField.apply(rho, engine)
