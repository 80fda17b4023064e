"""Differentiable inpainting: u = B g with the hand-written adjoint as backward.

Section 4 writes the inpainting result as u = B g, with B the product of the
interpolation matrix and the inverse of the FEM matrix, and optimises g by
least squares. ``InpaintFn`` exposes that map to torch.autograd: the forward
pass runs the library's inpainting (solve + interpolation) and the backward
pass runs its adjoint, B^T grad_u (transposed interpolation + the same
symmetric solve + coupling tail). For MSE(g) = ||B g - f||^2 / P the gradient
is (2 / P) B^T (B g - f).
"""
from __future__ import annotations

import torch

from . import Mesh, SolveOpts


class InpaintFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, g: torch.Tensor, mesh: Mesh, opts: SolveOpts | None = None):
        g = g.detach().contiguous()
        u, _ = mesh.inpaint(g=g, opts=opts)
        ctx.mesh = mesh
        ctx.opts = opts
        return u

    @staticmethod
    def backward(ctx, grad_u: torch.Tensor):
        s, _ = ctx.mesh.adjoint(grad_u.detach().contiguous().to(torch.float64), opts=ctx.opts)
        return s, None, None


def inpaint(g: torch.Tensor, mesh: Mesh, opts: SolveOpts | None = None) -> torch.Tensor:
    """u = B g, differentiable in g."""
    return InpaintFn.apply(g, mesh, opts)


def mse_loss(g: torch.Tensor, f: torch.Tensor, mesh: Mesh,
             opts: SolveOpts | None = None) -> torch.Tensor:
    """MSE(g) = mean((B g - f)^2) with f the uint8 image (flattened)."""
    u = inpaint(g, mesh, opts)
    return torch.mean((u - f.reshape(-1).to(torch.float64)) ** 2)
