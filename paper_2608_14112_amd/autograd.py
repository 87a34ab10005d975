"""torch.autograd bridge: the truncated Gaussian field as a differentiable op.

    field = GaussianField(n, Grid(nx, ny, nz), k=3.0)
    V = field(theta)            # theta: float32 cuda [11, n], requires_grad
    (V * W).sum().backward()    # theta.grad via the library's VJP kernel

Forward is gve_evaluate, backward gve_vjp (sum_p u(p) dV(p)/dtheta with the
truncation indicator held fixed), both on the library's stream.
"""
from __future__ import annotations

import torch

from . import NPARAM, Context, Grid, Params, evaluate, vjp


class _FieldFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, theta, gctx, grid, params):
        th = theta.detach().contiguous()
        params.upload_device(th)
        out = torch.empty(grid.shape, device=theta.device, dtype=torch.float32)
        evaluate(gctx, params, grid, out)
        fctx.save_for_backward(th)
        fctx.gctx, fctx.grid, fctx.params = gctx, grid, params
        return out

    @staticmethod
    def backward(fctx, gout):
        (th,) = fctx.saved_tensors
        fctx.params.upload_device(th)     # the module may have been called again since
        grad = vjp(fctx.gctx, fctx.params, gout.contiguous(), fctx.grid)
        return grad, None, None, None


class GaussianField(torch.nn.Module):
    """V = sum_i c_i G_i [m_i^2 < k^2] on `grid` as a function of theta [11, n]."""

    def __init__(self, n: int, grid: Grid, k: float = 3.0, brick: int = 8, brick_z=None):
        super().__init__()
        self.gctx = Context(k=k, brick=brick, brick_z=brick_z)
        self.params = Params(self.gctx, n)
        self.grid = grid
        self.n = n

    def forward(self, theta):
        if theta.shape != (NPARAM, self.n) or theta.dtype != torch.float32 or not theta.is_cuda:
            raise ValueError(f"theta must be a float32 cuda tensor of shape ({NPARAM}, {self.n})")
        return _FieldFn.apply(theta, self.gctx, self.grid, self.params)
