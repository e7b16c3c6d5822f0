"""Differentiable synthesis and analysis (torch.autograd.Function).

The backward passes call the hand-written adjoint kernels of libshtn:
SynthFn.backward(g) = S^T g (shtn_synth_adj) and AnalysFn.backward(h) = A^T h
(shtn_analys_adj).  Gradients of complex spectra follow PyTorch's convention
dL/dRe Q + i dL/dIm Q, which is exactly what the adjoint entry points return.
Both maps are linear, so their backward passes are themselves differentiable
through the opposite Function (double backward).  The vector transforms
(spheroidal / toroidal) follow the same pattern with shtn_vec_synth_adj and
shtn_vec_analys_adj.
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


class VecSynthFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, S, T, plan):
        ctx.plan = plan
        return plan.vec_synth(S, T)

    @staticmethod
    def backward(ctx, gt, gp):
        gS, gT = VecSynthAdjFn.apply(gt.contiguous(), gp.contiguous(), ctx.plan)
        return gS, gT, None


class VecSynthAdjFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gt, gp, plan):
        ctx.plan = plan
        return plan.vec_synth_adj(gt, gp)

    @staticmethod
    def backward(ctx, hS, hT):
        gt, gp = VecSynthFn.apply(hS.contiguous(), hT.contiguous(), ctx.plan)
        return gt, gp, None


class VecAnalysFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vt, vp, plan):
        ctx.plan = plan
        return plan.vec_analys(vt, vp)

    @staticmethod
    def backward(ctx, hS, hT):
        gt, gp = VecAnalysAdjFn.apply(hS.contiguous(), hT.contiguous(), ctx.plan)
        return gt, gp, None


class VecAnalysAdjFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, hS, hT, plan):
        ctx.plan = plan
        return plan.vec_analys_adj(hS, hT)

    @staticmethod
    def backward(ctx, gt, gp):
        hS, hT = VecAnalysFn.apply(gt.contiguous(), gp.contiguous(), ctx.plan)
        return hS, hT, None


def vec_synth(S, T, plan):
    """Differentiable vector synthesis: spheroidal and toroidal spectra -> (V_theta, V_phi)."""
    return VecSynthFn.apply(S, T, plan)


def vec_analys(vt, vp, plan):
    """Differentiable vector analysis: (V_theta, V_phi) -> spheroidal and toroidal spectra."""
    return VecAnalysFn.apply(vt, vp, plan)


def synth(Q, plan):
    """Differentiable synthesis: [..., nlm] complex128 -> [..., nlat, nphi]."""
    return SynthFn.apply(Q, plan)


def analys(g, plan):
    """Differentiable analysis: [..., nlat, nphi] float64 -> [..., nlm] complex128."""
    return AnalysFn.apply(g, plan)
