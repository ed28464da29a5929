"""torch.autograd binding of the relaxed renderer and its adjoint kernel.

Gradients of a rendered-view loss with respect to the dequantised residual
planes and the per-block shifts, for encoder-side refinement.  Both
directions run in the library's HIP kernels; the backward recomputes the
forward's ray geometry instead of storing it.
"""

from __future__ import annotations

import torch

from .lf import LightField


class RelaxedRender(torch.autograd.Function):
    @staticmethod
    def forward(ctx, residual, shift, field: LightField, cams, width: int, height: int):
        ctx.field, ctx.width, ctx.height = field, width, height
        ctx.save_for_backward(residual, shift, cams)
        return field.render_relaxed(residual, shift, cams, width, height)

    @staticmethod
    def backward(ctx, grad_out):
        residual, shift, cams = ctx.saved_tensors
        g_res, g_sh = ctx.field.render_backward(residual, shift, cams, ctx.width, ctx.height,
                                                grad_out.contiguous().float())
        return g_res, g_sh, None, None, None, None


def render_relaxed(field: LightField, residual: torch.Tensor, shift: torch.Tensor, cams: torch.Tensor,
                   width: int, height: int) -> torch.Tensor:
    """Differentiable render: float32 [V, 3, height, width]."""
    return RelaxedRender.apply(residual, shift, field, cams, width, height)
