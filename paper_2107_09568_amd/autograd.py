"""torch.autograd bridge for the shape sensitivities of Section 4.1.2.

UKU.apply(ctrl, u, plan, E, nu, precision) returns u^T K^pi(ctrl) u for the plan's
topology; its backward returns d(u^T K u)/d ctrl from the library's adjoint kernels,
u held fixed.  The derivative by u (2 K u) is not provided: u must not require grad.

Compliance.apply(ctrl, u, plan, E, nu, precision, load) is c = f^T K^-1 f for a u that
already solves K u = f (c = u^T K u at the solution).  With u = K^-1 f the solve's
derivative folds into the adjoint (eq. (69)-(73)):
    dc/dm = 2 u . df/dm - u^T (dK/dm) u.
load = None: f is a nodal vector that does not depend on ctrl, so the first term vanishes.
load = (body, traction): f = f^pi(ctrl), the library's load vector (igamt_load_assemble)
for that body force and face tractions; its body term carries |det J| and its face terms
the area element, so it moves with ctrl and the first term comes from igamt_uf_grad (the
plan's load table must be built).
"""
from __future__ import annotations

import torch


def _no_u_grad(u):
    if u.requires_grad:
        raise NotImplementedError("the derivative by u is not provided: pass u.detach()")


class UKU(torch.autograd.Function):
    @staticmethod
    def forward(ctx, ctrl, u, plan, E, nu, precision="f64"):
        assert ctrl.is_cuda and ctrl.dtype == torch.float64
        _no_u_grad(u)
        plan.set_macro_ctrl(ctrl.detach().contiguous())
        val, grad = plan.uKu_grad(E, nu, u.detach().contiguous(), precision)
        ctx.save_for_backward(grad)
        return val.reshape(())

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g * grad, None, None, None, None, None


class Compliance(torch.autograd.Function):
    """c = f^T K^-1 f for a u that already solves K u = f; see the module docstring for `load`."""

    @staticmethod
    def forward(ctx, ctrl, u, plan, E, nu, precision="f64", load=None):
        assert ctrl.is_cuda and ctrl.dtype == torch.float64
        _no_u_grad(u)
        plan.set_macro_ctrl(ctrl.detach().contiguous())
        ud = u.detach().contiguous()
        val, grad = plan.uKu_grad(E, nu, ud, precision)
        grad = -grad
        if load is not None:
            body, traction = load
            _, gf = plan.uf_grad(body, traction, ud)
            grad = grad + 2.0 * gf
        ctx.save_for_backward(grad)
        return val.reshape(())

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return g * grad, None, None, None, None, None, None
