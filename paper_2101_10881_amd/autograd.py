"""torch.autograd.Function over the multiple-double evaluation.

Forward: eval_and_diff with a plan that keeps the monomial products
(MDPE_KEEP_MONOMIAL_VALUES), on a fresh workspace saved for the backward.
Backward: the hand-written reverse pass eval_adjoint (correlations of the
upstream adjoint with the gradient series and with the monomial products).

Tensors hold m-doubles limb-planar: coeff [m][N+1][d+1], z [m][n][d+1],
value [m][d+1].  The gradient returned for an m-double tensor is the
m-double adjoint in the same layout: limb 0 is the double-precision value
of dL/dx and the lower limbs extend its precision; the upstream gradient
of the value is read the same way.
"""
from __future__ import annotations

import torch

from . import mdpe


class PolyEvalFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coeff, z, poly):
        if not isinstance(poly, mdpe.Polynomial) or not (poly.plan.info["flags"] & mdpe.MDPE_KEEP_MONOMIAL_VALUES):
            raise ValueError("poly must be a Polynomial built with keep_monomials=True")
        coeff = coeff.contiguous()
        z = z.contiguous()
        ws = poly.new_workspace()
        value, grad = poly.eval_and_diff(coeff, z, workspace=ws)
        ctx.poly = poly
        ctx.ws = ws
        ctx.mark_non_differentiable(grad)
        ctx.save_for_backward(grad)
        return value, grad

    @staticmethod
    def backward(ctx, ybar, _grad_bar):
        if ybar is None:
            return None, None, None
        (grad,) = ctx.saved_tensors
        cbar, zbar = ctx.poly.adjoint(ybar.contiguous(), grad, workspace=ctx.ws)
        return cbar, zbar, None


def poly_eval(coeff, z, poly):
    """value, gradient = p(z), dp/dz; differentiable in coeff and z through value."""
    return PolyEvalFunction.apply(coeff, z, poly)
