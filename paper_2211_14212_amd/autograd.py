"""torch.autograd wrappers of the cone-beam projector pair.

``project(vol, plan)`` applies A (the HIP forward projector); its backward is
the hand-written matched back projector A^T, which is the exact adjoint of A
up to FP32 rounding.  ``backproject(proj, plan)`` is the transpose pair.
Both run on the plan's GPU and the caller's current stream.
"""
from __future__ import annotations

import torch


class ConeProject(torch.autograd.Function):
    """y = A x; dL/dx = A^T dL/dy."""

    @staticmethod
    def forward(ctx, vol: torch.Tensor, plan):
        ctx.plan = plan
        return plan.forward(vol.contiguous())

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        g = grad_out.contiguous()
        return ctx.plan.backproject(g, out_dtype=g.dtype), None


class ConeBackproject(torch.autograd.Function):
    """x = A^T y; dL/dy = A dL/dx."""

    @staticmethod
    def forward(ctx, proj: torch.Tensor, plan):
        ctx.plan = plan
        return plan.backproject(proj.contiguous())

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        g = grad_out.contiguous()
        return ctx.plan.forward(g, out_dtype=g.dtype), None


def project(vol: torch.Tensor, plan) -> torch.Tensor:
    return ConeProject.apply(vol, plan)


def backproject(proj: torch.Tensor, plan) -> torch.Tensor:
    return ConeBackproject.apply(proj, plan)
