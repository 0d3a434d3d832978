"""torch.autograd.Function over the bbFMM: forward = bbfmm_apply, backward = the adjoint FMM.

With L = sum_i g_i . phi_i and phi = A(x) q, the backward returns
  dL/dq = A^T g                       (bbfmm_apply_adjoint: transposed chain L2P^T, L2L^T,
                                       M2L^T, M2M^T, P2M^T, near field^T)
  dL/dx = bbfmm_eval_grad(q, g)       (target and source roles of every point, tree held fixed).
The tree (leaf membership, cell centres) is piecewise constant in the positions and is held
fixed, so dL/dx is the derivative of the FMM approximation inside the current cells.
"""
from __future__ import annotations

import torch

from .binding import Octree, Plan


class FMMFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, points, q, depth: int, order: int, kernel: str = "inv_r", svd_eps: float = 0.0,
                c: float = 0.0, root_lo=(0.0, 0.0, 0.0), root_width: float = 1.0):
        squeeze = q.dim() == 1
        qq = q.detach().reshape(q.shape[0], -1).contiguous().to(torch.float64)
        tree = Octree(points.detach().contiguous().to(torch.float64), depth, root_lo, root_width)
        plan = Plan(tree, kernel, order, svd_eps, "fp64", c)
        phi = plan.apply(qq)
        ctx.plan = plan
        ctx.squeeze = squeeze
        ctx.save_for_backward(qq)
        return phi.reshape(-1) if squeeze else phi

    @staticmethod
    def backward(ctx, grad_phi):
        (qq,) = ctx.saved_tensors
        plan = ctx.plan
        g = grad_phi.reshape(qq.shape[0], -1).contiguous().to(torch.float64)
        grad_q = plan.apply_adjoint(g)
        grad_points = plan.eval_grad(qq, g, 3) if ctx.needs_input_grad[0] else None
        if ctx.squeeze:
            grad_q = grad_q.reshape(-1)
        return grad_points, (grad_q if ctx.needs_input_grad[1] else None), None, None, None, None, None, None, None
