"""torch.autograd bridge for the shape sensitivity of u^T K u (Section 4.1.2).

UKU.apply(ctrl, u, plan, E, nu, precision) returns u^T K^pi(ctrl) u for the plan's
topology; its backward returns d(u^T K u)/d ctrl from the library's adjoint
kernels (the displacement u is treated as fixed: with u = K^-1 f and a load that
does not move, the compliance gradient is minus this).  Compliance wraps that
sign convention for a u that already solves K u = f.
"""
from __future__ import annotations

import torch


class UKU(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ctrl, u, plan, E, nu, precision="f64"):
        assert ctrl.is_cuda and ctrl.dtype == torch.float64
        plan.set_macro_ctrl(ctrl.detach().contiguous())
        val, grad = plan.uKu_grad(E, nu, u.detach().contiguous(), precision)
        ctx.save_for_backward(grad)
        return val.reshape(())

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g * grad, None, None, None, None, None


class Compliance(torch.autograd.Function):
    """c = f^T K^-1 f for a u that already solves K u = f (so c = u^T K u); dc/dctrl = -d(u^T K u)/dctrl
    because the load does not depend on the macro control points."""

    @staticmethod
    def forward(ctx, ctrl, u, plan, E, nu, precision="f64"):
        plan.set_macro_ctrl(ctrl.detach().contiguous())
        val, grad = plan.uKu_grad(E, nu, u.detach().contiguous(), precision)
        ctx.save_for_backward(grad)
        return val.reshape(())

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return -g * grad, None, None, None, None, None
