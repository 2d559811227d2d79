"""The weighted residual r_w(theta) as a differentiable PyTorch function backed by the library's kernels.

`residual(theta, prob)` returns r_w = sqrt(w) * residual(theta) (the least-squares residual whose
Gauss-Newton matrix is G = J_w^T J_w, eq. G_matrixfree). Its reverse-mode derivative runs the adjoint
kernel (`ngd_vjp`: J_w^T grad_r, seeds of the reverse sweep scaled by grad_r) and its forward-mode
derivative the forward-tangent kernel (`ngd_jvp`: J_w theta_dot); neither forms J_w, which is the
"Recompute Jacobian" strategy of Section 4.1.2.
"""
from __future__ import annotations

import torch

from .api import Problem


class ResidualFn(torch.autograd.Function):
    """r_w(theta); backward = J_w^T grad_r (adjoint kernel), jvp = J_w theta_dot (tangent kernel)."""

    @staticmethod
    def forward(theta: torch.Tensor, prob: Problem) -> torch.Tensor:
        r, _, _, _ = prob.residual_jacobian(theta.detach().contiguous(), None, want_grad=False, want_loss=False)
        return r

    @staticmethod
    def setup_context(ctx, inputs, output):
        theta, prob = inputs
        ctx.prob = prob
        ctx.save_for_backward(theta)
        ctx.save_for_forward(theta)

    @staticmethod
    def backward(ctx, grad_r):
        (theta,) = ctx.saved_tensors
        g = ctx.prob.vjp(theta.detach().contiguous(), grad_r.to(theta.dtype).contiguous())
        return g.to(theta.dtype), None

    @staticmethod
    def jvp(ctx, theta_dot, _prob_dot):
        (theta,) = ctx.saved_tensors
        return ctx.prob.jvp(theta.detach().contiguous(), theta_dot.to(theta.dtype).contiguous())


def residual(theta: torch.Tensor, prob: Problem) -> torch.Tensor:
    """r_w(theta) with reverse- and forward-mode derivatives from the library's kernels."""
    return ResidualFn.apply(theta, prob)
