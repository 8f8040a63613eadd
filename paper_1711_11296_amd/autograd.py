"""Reverse-mode differentiation of the transform pair.

SHTForward (grid -> spec) and SHTInverse (spec -> grid) are
torch.autograd.Functions whose backward passes call the library's adjoint
transforms (the exact transposes of the stored-array linear maps), so that a
variational data-assimilation cost can be differentiated through either
direction.  Spectra are real tensors [..., ncoef, 2]; Im of m = 0 is not a
degree of freedom (its gradient is 0).
"""

import torch


class SHTForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, grid, plan):
        ctx.plan = plan
        return plan.forward(grid.contiguous())

    @staticmethod
    def backward(ctx, grad_spec):
        return ctx.plan.forward_adjoint(grad_spec.contiguous()), None


class SHTInverse(torch.autograd.Function):
    @staticmethod
    def forward(ctx, spec, plan):
        ctx.plan = plan
        return plan.inverse(spec.contiguous())

    @staticmethod
    def backward(ctx, grad_grid):
        return ctx.plan.inverse_adjoint(grad_grid.contiguous()), None


def sht_forward(grid, plan):
    """Differentiable analysis grid -> spec."""
    return SHTForward.apply(grid, plan)


def sht_inverse(spec, plan):
    """Differentiable synthesis spec -> grid."""
    return SHTInverse.apply(spec, plan)
