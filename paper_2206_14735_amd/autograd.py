"""torch.autograd.Function over the library's forward and backward.

``gosurf_loss(grid, mlp, model, batch, loss_cfg, workspace)`` returns the
weighted total loss of a sampled batch (a 0-dim tensor on the device).
Calling ``backward()`` on it (or on anything computed from it) makes
gosurf_backward write the exact gradients of that total into ``grid.grad``
and ``mlp.grad``: the grid scatter, the decoder weight gradients and the
double backward of the Eikonal and smoothness terms, all in the library's
kernels.  The incoming gradient (any sign) is passed to the library as its loss scale.
The per-ray and per-sample forward results stay available in
``last_forward`` of the returned tensor's grad_fn context.

The function is once differentiable: the gradient it returns is not itself
differentiable through torch.
"""
from __future__ import annotations

import torch
from torch.autograd.function import once_differentiable

from . import gosurf as G


class GoSurfLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, grid, mlp, model, batch, loss_cfg, workspace, grid_bf16=None):
        out = G.gosurf_forward(model, grid.detach(), mlp.detach(), batch, loss_cfg, workspace, grid_bf16=grid_bf16)
        ctx.save_for_backward(grid, mlp)
        ctx.state = (model, batch, loss_cfg, workspace, out, grid_bf16)
        ctx.last_forward = out
        return out.losses[6].clone()

    @staticmethod
    @once_differentiable
    def backward(ctx, g):
        grid, mlp = ctx.saved_tensors
        model, batch, loss_cfg, workspace, out, grid_bf16 = ctx.state
        scale = float(g)
        gg, gm = torch.zeros_like(grid), torch.zeros_like(mlp)
        if scale != 0.0:
            G.gosurf_backward(model, grid.detach(), mlp.detach(), batch, loss_cfg, out, scale, gg, gm, workspace,
                              grid_bf16=grid_bf16)
        return gg, gm, None, None, None, None, None


def gosurf_loss(grid, mlp, model, batch, loss_cfg, workspace, grid_bf16=None):
    """Weighted total loss of `batch` with gradients through the library."""
    return GoSurfLoss.apply(grid, mlp, model, batch, loss_cfg, workspace, grid_bf16)
