"""torch.autograd wrappers of the butterfly transform.

The transform is linear, f = Phi~ c, so the gradient of a loss with respect to
c is Phi~^T (dL/df) and the backward pass is one transposed apply (the analysis
map, Sec. 1).  Nothing but the plan is kept between forward and backward: the
level vectors of the forward sweep are not stored, the transposed sweep
recomputes its own, so memory does not grow with n.
"""
import torch


class BFApply(torch.autograd.Function):
    """f = Phi~ c with backward grad_c = Phi~^T grad_f."""

    @staticmethod
    def forward(ctx, c, plan):
        ctx.plan = plan
        return plan.apply(c.contiguous())

    @staticmethod
    def backward(ctx, grad_f):
        return ctx.plan.apply_t(grad_f.contiguous()), None


class BFApplyT(torch.autograd.Function):
    """g = Phi~^T f with backward grad_f = Phi~ grad_g."""

    @staticmethod
    def forward(ctx, f, plan):
        ctx.plan = plan
        return plan.apply_t(f.contiguous())

    @staticmethod
    def backward(ctx, grad_g):
        return ctx.plan.apply(grad_g.contiguous()), None


def synthesis(c, plan):
    return BFApply.apply(c, plan)


def analysis(f, plan):
    return BFApplyT.apply(f, plan)


def least_squares_step(plan, c, f, lr):
    """One gradient-descent step on ||Phi~ c - f||^2 through autograd; returns the loss."""
    c = c.detach().requires_grad_(True)
    r = BFApply.apply(c, plan) - f
    loss = (r * r).sum()
    loss.backward()
    with torch.no_grad():
        c_new = c - lr * c.grad
    return c_new.detach(), loss.detach()
