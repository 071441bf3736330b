"""Dose + cost as differentiable torch functions.

The forward pass runs the dose product and the eq. 1 penalty (plus the eq. 2
smoothing in the aperture form) in the HIP library; the backward pass runs
the library's hand-written adjoint (transpose) product on the saved dose
derivative F'(z).  Gradients are FP64; the dose derivative handed to the
adjoint is FP32, as in the optimiser itself.
"""
from __future__ import annotations

import torch


class _ApertureCost(torch.autograd.Function):
    """cost(y) = F(z(y)) + gamma G(y) for fixed apertures (eq. 3)."""

    @staticmethod
    def forward(ctx, y, prob, l, r, occ):
        yc = y.detach().contiguous()
        out = prob.grad(yc, l, r, occ, want=("dF",))
        ctx.prob, ctx.plan = prob, (l, r, occ)
        ctx.save_for_backward(yc, out["dF"])
        return out["cost"].sum()

    @staticmethod
    def backward(ctx, grad_out):
        y, dF = ctx.saved_tensors
        l, r, occ = ctx.plan
        dfdy, _ = ctx.prob.grad_apertures(y, l, r, occ, dF)
        return grad_out * dfdy, None, None, None, None


class _FluenceCost(torch.autograd.Function):
    """cost(x) = F(D^T x) for beamlet intensities x (eq. 1 on the dose of x)."""

    @staticmethod
    def forward(ctx, x, prob):
        xc = x.detach().contiguous()
        out = prob.grad_fluence(xc, want=("dF",))
        ctx.prob = prob
        ctx.save_for_backward(out["dF"])
        return out["cost"][0]

    @staticmethod
    def backward(ctx, grad_out):
        (dF,) = ctx.saved_tensors
        g = ctx.prob.adjoint(dF)
        return grad_out * g, None


def aperture_cost(prob, y, l, r, occ):
    """Differentiable F(z(y)) + gamma G(y); y: CUDA float64 [N]."""
    return _ApertureCost.apply(y, prob, l, r, occ)


def fluence_cost(prob, x):
    """Differentiable F(D^T x); x: CUDA float64 [nb]."""
    return _FluenceCost.apply(x, prob)
