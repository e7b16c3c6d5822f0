"""Differentiable synthesis and analysis (torch.autograd.Function).

The backward passes call the hand-written adjoint kernels of libshtn:
SynthFn.backward(g) = S^T g (shtn_synth_adj) and AnalysFn.backward(h) = A^T h
(shtn_analys_adj).  Gradients of complex spectra follow PyTorch's convention
dL/dRe Q + i dL/dIm Q, which is exactly what the adjoint entry points return.
Both maps are linear, so their backward passes are themselves differentiable
through the opposite Function (double backward).
"""
from __future__ import annotations

import torch


class SynthFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Q, plan):
        ctx.plan = plan
        return plan.synth(Q)

    @staticmethod
    def backward(ctx, g):
        return SynthAdjFn.apply(g.contiguous(), ctx.plan), None


class SynthAdjFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, g, plan):
        ctx.plan = plan
        return plan.synth_adj(g)

    @staticmethod
    def backward(ctx, h):
        return SynthFn.apply(h.contiguous(), ctx.plan), None


class AnalysFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, g, plan):
        ctx.plan = plan
        return plan.analys(g)

    @staticmethod
    def backward(ctx, h):
        return AnalysAdjFn.apply(h.contiguous(), ctx.plan), None


class AnalysAdjFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, h, plan):
        ctx.plan = plan
        return plan.analys_adj(h)

    @staticmethod
    def backward(ctx, g):
        return AnalysFn.apply(g.contiguous(), ctx.plan), None


def synth(Q, plan):
    """Differentiable synthesis: [..., nlm] complex128 -> [..., nlat, nphi]."""
    return SynthFn.apply(Q, plan)


def analys(g, plan):
    """Differentiable analysis: [..., nlat, nphi] float64 -> [..., nlm] complex128."""
    return AnalysFn.apply(g, plan)
