"""The objective J(I+, I-, b) of the distortion-correction problem (Eq. 2-6) as a
torch.autograd.Function with a hand-written backward, on one grid or summed over the levels of the
multilevel pyramid.

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


class PyramidObjective(torch.autograd.Function):
    """sum_l w_l J_l(R^l I+, R^l I-, b_l, 2^l h): the objective on every level of the pyramid that
    the coarse-to-fine scheme solves on (Sec. 3.4; R = 2x2x2 block means, spacing doubled per
    level), with the field of each level an input of its own.  Checkpointed per level: the forward
    keeps only the finest images and the fields; the backward rebuilds each level's images by
    restriction, takes dJ_l/db_l and dJ_l/dI_l on that level, and carries the image gradients to
    the finest level with the adjoint restriction, coarsest first: g = g_0 + R^T (g_1 + R^T (...))."""

    @staticmethod
    def forward(ctx, I_plus, I_minus, pe, h, alpha, beta, weights, *fields):
        J = None
        P, M, hl = I_plus, I_minus, tuple(h)
        for l, b in enumerate(fields):
            if l > 0:
                P, M = rgp.restrict_image(P, b.dtype), rgp.restrict_image(M, b.dtype)
                hl = tuple(2.0 * x for x in hl)
            jdsp, _, _, _ = rgp.loss_grad(P, M, b, pe, hl, alpha, beta, want_grad=False,
                                          want_hess=False)
            Jl = jdsp[0] * weights[l]
            J = Jl if J is None else J + Jl
        ctx.save_for_backward(I_plus, I_minus, *fields)
        ctx.cfg = (pe, tuple(h), alpha, beta, tuple(weights))
        return J

    @staticmethod
    def backward(ctx, gJ):
        I_plus, I_minus, *fields = ctx.saved_tensors
        pe, h, alpha, beta, weights = ctx.cfg
        need_p, need_m = ctx.needs_input_grad[:2]
        need_b = ctx.needs_input_grad[7:]
        levels = []
        P, M, hl = I_plus, I_minus, h
        for l, b in enumerate(fields):
            if l > 0:
                P, M = rgp.restrict_image(P, b.dtype), rgp.restrict_image(M, b.dtype)
                hl = tuple(2.0 * x for x in hl)
            levels.append((P, M, hl))
        g_fields = []
        for l, (b, (P, M, hl)) in enumerate(zip(fields, levels)):
            if need_b[l]:
                _, g, _, _ = rgp.loss_grad(P, M, b, pe, hl, alpha, beta, want_grad=True,
                                           want_hess=False)
                g_fields.append(g * (gJ.to(g.dtype) * weights[l]))
            else:
                g_fields.append(None)
        g_p = g_m = None
        if need_p or need_m:
            acc_p = acc_m = None
            for l in range(len(fields) - 1, -1, -1):
                P, M, hl = levels[l]
                gp, gm = rgp.loss_grad_images(P, M, fields[l], pe, hl)
                if weights[l] != 1.0:
                    gp.mul_(weights[l])
                    gm.mul_(weights[l])
                if acc_p is not None:
                    rgp.restrict_image_adjoint(acc_p, tuple(P.shape), out=gp, accumulate=True)
                    rgp.restrict_image_adjoint(acc_m, tuple(M.shape), out=gm, accumulate=True)
                acc_p, acc_m = gp, gm
            s = gJ.to(acc_p.dtype)
            g_p = (acc_p * s).to(I_plus.dtype) if need_p else None
            g_m = (acc_m * s).to(I_minus.dtype) if need_m else None
        return (g_p, g_m, None, None, None, None, None, *g_fields)


def pyramid_objective(I_plus, I_minus, fields, pe, h=(1.0, 1.0, 1.0), alpha=300.0, beta=1e-4,
                      weights=None):
    """sum over levels of w_l J_l (0-dim FP64 device tensor), with gradients to I_plus, I_minus
    and every field.  fields[l] is the field of level l (finest first): cells ceil(m / 2^l) per
    axis, one node more along pe.  weights default to 1 per level."""
    fields = list(fields)
    if not fields:
        raise ValueError("at least one level")
    weights = [1.0] * len(fields) if weights is None else [float(w) for w in weights]
    if len(weights) != len(fields):
        raise ValueError("one weight per level")
    if any(b.dtype != fields[0].dtype for b in fields):
        raise ValueError("every level's field has the same dtype")
    shape = tuple(int(m) for m in I_plus.shape)
    for l, b in enumerate(fields):
        if l > 0:
            shape = rgp.coarse_shape(shape)
        if tuple(b.shape) != rgp.field_shape(shape, pe):
            raise ValueError(f"level {l}: field shape {tuple(b.shape)}, expected "
                             f"{rgp.field_shape(shape, pe)}")
    return PyramidObjective.apply(I_plus, I_minus, int(pe), tuple(float(x) for x in h),
                                  float(alpha), float(beta), tuple(weights), *fields)
