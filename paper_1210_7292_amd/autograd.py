"""torch.autograd.Function over the bbFMM: forward = bbfmm_apply, backward = the adjoint FMM.

With L = sum_i g_i . phi_i and phi = A(x) q, the backward returns
  dL/dq = A^T g                       (bbfmm_apply_adjoint: transposed chain L2P^T, L2L^T,
                                       M2L^T, M2M^T, P2M^T, near field^T)
  dL/dx = bbfmm_eval_grad(q, g)       (target and source roles of every point, tree held fixed).
The tree (leaf membership, cell centres) is piecewise constant in the positions and is held
fixed, so dL/dx is the derivative of the FMM approximation inside the current cells.

The plan is built once by the caller (operator precompute and tree build are not repeated per
call); each forward moves the plan's tree to the given positions with bbfmm_tree_update_points,
which requires every point to stay in its leaf, and runs the plan's M2L precision.
"""
from __future__ import annotations

import torch

from .binding import BBFMMError, Octree, Plan


class FMMFunction(torch.autograd.Function):
    """FMMFunction.apply(points, q, plan) -> phi.

    points: (n, 3) float64 on the plan's device, each inside the leaf it had when plan.tree was
    built (uniform trees); q: (n,) or (n, nrhs) float64. The plan keeps the forward's locals for the
    backward, so the same plan must not run another apply between this forward and its backward.
    """

    @staticmethod
    def forward(ctx, points, q, plan: Plan):
        if plan.tree.adaptive:
            raise BBFMMError(-4, "FMMFunction needs a uniform tree (gradients on adaptive trees are not supported)")
        squeeze = q.dim() == 1
        qq = q.detach().reshape(q.shape[0], -1).contiguous().to(torch.float64)
        plan.tree.update_points(points.detach().contiguous().to(torch.float64))
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
        return grad_points, (grad_q if ctx.needs_input_grad[1] else None), None


def make_plan(points, depth: int, order: int, kernel: str = "inv_r", svd_eps: float = 0.0, c: float = 0.0,
              m2l_prec: str = "fp64", root_lo=(0.0, 0.0, 0.0), root_width: float = 1.0) -> Plan:
    """Uniform tree of `points` and its plan, for FMMFunction."""
    tree = Octree(points.detach().contiguous().to(torch.float64), depth, root_lo, root_width)
    return Plan(tree, kernel, order, svd_eps, m2l_prec, c)


def fmm(points, q, plan: Plan):
    """Differentiable phi = A(points) q (see FMMFunction)."""
    return FMMFunction.apply(points, q, plan)
