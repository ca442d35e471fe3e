"""Differentiable treecode: a torch.autograd.Function over the C-ABI.

forward  : stk_evaluate with the plan kept (interaction lists, centres, scales).
backward : stk_evaluate_adjoint on that plan, i.e. the exact gradient of the discrete
           operator the forward pass applied (lists and cluster geometry held fixed).
Gradients flow to targets, sources, f and h; nu is treated as a constant.  If the same
tensor is passed as targets and sources, autograd adds the two position gradients.
"""
from __future__ import annotations

import torch

from . import _native as native


class StokesTreecode(torch.autograd.Function):
    @staticmethod
    def forward(ctx, targets, sources, f, h, nu, p: int, theta: float, n0: int, precision: str = "mixed"):
        # the adjoint applies the transpose of a one-right-hand-side operator: a batch of K
        # (f, h) sets can be evaluated, but not differentiated, through this function
        if f.dim() == 3 and f.shape[0] > 1 and any(ctx.needs_input_grad[:4]):
            raise ValueError("stokes_treecode: gradients need one right-hand side (f, h of shape (N, 3)); "
                             f"got K = {f.shape[0]}")
        args = [t.detach().contiguous() for t in (targets, sources, f, h, nu)]
        u, plan = native.evaluate(*args, p, theta, n0, precision, keep_plan=True)
        ctx.plan = plan
        ctx.n_sources = sources.shape[0]
        return u

    @staticmethod
    def backward(ctx, gu):
        want = []
        if ctx.needs_input_grad[2]:
            want.append("f")
        if ctx.needs_input_grad[3]:
            want.append("h")
        if ctx.needs_input_grad[0]:
            want.append("targets")
        if ctx.needs_input_grad[1]:
            want.append("sources")
        g = native.evaluate_adjoint(ctx.plan, gu.contiguous().to(torch.float64), ctx.n_sources, tuple(want))
        return (g.get("targets"), g.get("sources"), g.get("f"), g.get("h"), None, None, None, None, None)


def stokes_treecode(targets, sources, f, h, nu, p: int = 8, theta: float = 0.5, n0: int = 1000,
                    precision: str = "mixed"):
    """u_i(x^m) of eq. StoStre by the treecode, differentiable in targets, sources, f, h."""
    return StokesTreecode.apply(targets, sources, f, h, nu, p, theta, n0, precision)
