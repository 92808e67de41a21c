"""The objective J(I+, I-, b) of the distortion-correction problem (Eq. 2-6) as a
torch.autograd.Function with a hand-written backward.

forward: J, D, S, P from rgp_loss_grad (no gradient, no Hessian: nothing is kept but the inputs).
backward: recomputes on the device what it needs (checkpointing: no intermediate is stored between
the passes) - dJ/db from rgp_loss_grad, dJ/dI+- from rgp_loss_grad_images (the adjoint of the
interpolation and modulation) - and scales by the incoming gradient.  Gradients with respect to
the images are returned in the images' dtype (e.g. BF16 storage), computed in the field type.
"""
from __future__ import annotations

import torch

from . import rgp


class Objective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, I_plus, I_minus, b, pe, h, alpha, beta):
        jdsp, _, _, _ = rgp.loss_grad(I_plus, I_minus, b, pe, h, alpha, beta, want_grad=False,
                                      want_hess=False)
        ctx.save_for_backward(I_plus, I_minus, b)
        ctx.cfg = (pe, tuple(h), alpha, beta)
        return jdsp[0]

    @staticmethod
    def backward(ctx, gJ):
        I_plus, I_minus, b = ctx.saved_tensors
        pe, h, alpha, beta = ctx.cfg
        need_p, need_m, need_b = ctx.needs_input_grad[:3]
        g_p = g_m = g_b = None
        if need_b:
            _, g, _, _ = rgp.loss_grad(I_plus, I_minus, b, pe, h, alpha, beta, want_grad=True,
                                       want_hess=False)
            g_b = g * gJ.to(g.dtype)
        if need_p or need_m:
            gp, gm = rgp.loss_grad_images(I_plus, I_minus, b, pe, h)
            s = gJ.to(gp.dtype)
            g_p = (gp * s).to(I_plus.dtype) if need_p else None
            g_m = (gm * s).to(I_minus.dtype) if need_m else None
        return g_p, g_m, g_b, None, None, None, None


def objective(I_plus, I_minus, b, pe, h=(1.0, 1.0, 1.0), alpha=300.0, beta=1e-4):
    """J (0-dim FP64 device tensor) with gradients to I_plus, I_minus and b."""
    return Objective.apply(I_plus, I_minus, b, pe, tuple(h), float(alpha), float(beta))
