"""Differentiable forward operator: E as a torch.autograd.Function.

forward(x) = E x runs the library's forward kernels (coil product, centred
transform, mask); backward(g) = E^H g runs the adjoint kernels.  For a
C-linear map PyTorch's complex convention hands backward the conjugate
Wirtinger derivative dL/dy*, and the vector-Jacobian product is E^H of it,
so for L = ||E x - y||^2 autograd yields x.grad = 2 E^H (E x - y).
"""
from __future__ import annotations

import torch

from .sense import Plan, SenseError


class SenseE(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, plan: Plan) -> torch.Tensor:
        if plan.kspace_storage != "c64":
            raise SenseError(1, "autograd needs complex64 k-space storage")
        ctx.plan = plan
        return plan.E(x.contiguous())

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        return ctx.plan.EH(g.contiguous()), None


def sense_E(x: torch.Tensor, plan: Plan) -> torch.Tensor:
    """y = E x with gradient E^H (the library's adjoint kernels)."""
    return SenseE.apply(x, plan)
