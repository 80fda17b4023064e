"""Differentiable inpainting and MSE, with the hand-written adjoint as backward.

Section 4 writes the inpainting result as u = B g, with B the product of the
interpolation matrix and the inverse of the FEM matrix, and optimises g by
least squares. Two torch.autograd.Functions expose that map; every step of
their forward and backward passes runs in the library, this module only
passes tensors through:

- ``InpaintFn``: u = B g (solve + interpolation); backward B^T grad_u
  (transposed interpolation + the same symmetric solve + coupling tail).
- ``MseFn``: MSE(g) = ||B g - f||^2 / P (inpainting, then the error sum
  divided by P on the device); backward s (2 / P) B^T (B g - f) for the
  incoming d loss / d MSE = s, from the library's MSE backward.
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


class MseFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, g: torch.Tensor, f: torch.Tensor, mesh: Mesh,
                opts: SolveOpts | None = None):
        g = g.detach().contiguous()
        u, _ = mesh.inpaint(g=g, opts=opts)
        mse = mesh.mse_dev(u, f)
        ctx.mesh = mesh
        ctx.opts = opts
        ctx.u = u
        ctx.f = f
        return mse.reshape(())

    @staticmethod
    def backward(ctx, grad_mse: torch.Tensor):
        scale = grad_mse.detach().to(torch.float64).reshape(1).contiguous()
        grad, _ = ctx.mesh.mse_backward(ctx.u, ctx.f, scale=scale, opts=ctx.opts)
        return grad, None, None, None


def inpaint(g: torch.Tensor, mesh: Mesh, opts: SolveOpts | None = None) -> torch.Tensor:
    """u = B g, differentiable in g."""
    return InpaintFn.apply(g, mesh, opts)


def mse_loss(g: torch.Tensor, f: torch.Tensor, mesh: Mesh,
             opts: SolveOpts | None = None) -> torch.Tensor:
    """MSE(g) = mean((B g - f)^2) over all P pixels, f the uint8 image
    (flattened), differentiable in g."""
    return MseFn.apply(g, f.reshape(-1).contiguous(), mesh, opts)
