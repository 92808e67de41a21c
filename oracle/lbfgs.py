"""FP64 NumPy oracle of the L-BFGS solver (Sec. 2.3.3): a quasi-Newton method on the explicit
gradient of the discretised objective, with the inverse Hessian estimated from the last few
steps.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never imports this.

The paper hands the explicit gradient to an external L-BFGS solver and fixes none of its
settings.  The readings used here (and identically by the HIP path):

* R28 direction d = -H g by the two-loop recursion over the last ``memory`` pairs
  (s_i = b_{i+1} - b_i, y_i = grad_{i+1} - grad_i), oldest pair dropped first, with the initial
  inverse Hessian H0 = (s^T y / y^T y) I of the newest pair (Nocedal and Wright, Algorithm 7.4 and
  Eq. 7.20).  A pair enters the memory only when s^T y > 1e-10 |s| |y| (it keeps H positive
  definite; otherwise it is dropped).  With no pair in memory (the first step of a level) the
  direction is the steepest descent scaled to a largest entry of 1: d = -g / max|g|.
* R29 step size: the Armijo backtracking of the Gauss-Newton solver (gamma = 1, 1/2, ...; at most
  ``ls_max_trials`` trials; J = +inf rejects a trial); when no trial is accepted the level stops
  with b unchanged.  The history starts empty on every pyramid level.
"""
from __future__ import annotations

import math
from typing import Callable, List, Tuple

import numpy as np

from . import rgp as _r

PAIR_CURVATURE = 1e-10   # s^T y > PAIR_CURVATURE |s| |y| for a pair to be kept


def two_loop(g: np.ndarray, pairs: List[Tuple[np.ndarray, np.ndarray, float]]) -> np.ndarray:
    """H g for the L-BFGS inverse Hessian H of ``pairs`` (oldest first; each (s, y, 1/s^T y)),
    with H0 = (s^T y / y^T y) I of the newest pair: the two-loop recursion."""
    q = g.copy()
    alphas = []
    for s, y, rho in reversed(pairs):
        a = rho * float(np.sum(s * q))
        alphas.append(a)
        q = q - a * y
    s, y, _ = pairs[-1]
    r = (float(np.sum(s * y)) / float(np.sum(y * y))) * q
    for (s, y, rho), a in zip(pairs, reversed(alphas)):
        bt = rho * float(np.sum(y * r))
        r = r + (a - bt) * s
    return r


def lbfgs(fun: Callable, x0: np.ndarray, *, iters: int, memory: int = 10, armijo_c: float = 1e-4,
          ls_max_trials: int = 10):
    """``iters`` L-BFGS steps from x0 on fun(x) -> (J, gradient or None when J = +inf).

    Returns (x, list of GNStep records: J, D, S, P as fun's extra values when it returns an
    object with them, |g|, g.d, the number of pairs used, the H0 scale (or 1/max|g| without
    pairs), gamma, trials, accepted)."""
    x = np.array(x0, dtype=np.float64)
    obj, g = fun(x)
    pairs: List[Tuple[np.ndarray, np.ndarray, float]] = []
    hist = []
    parts = lambda o: (o.J, o.D, o.S, o.P) if hasattr(o, "D") else (float(o), math.nan,
                                                                      math.nan, math.nan)
    for _ in range(iters):
        J, D, S, P = parts(obj)
        if g is None:   # outside the barrier: nothing to do on this level
            hist.append(_r.GNStep(J, D, S, P, math.nan, math.nan, 0, math.nan, 0.0, 0, False))
            break
        if pairs:
            d = -two_loop(g, pairs)
            sy, yy = float(np.sum(pairs[-1][0] * pairs[-1][1])), float(np.sum(pairs[-1][1] ** 2))
            h0 = sy / yy
        else:
            gmax = float(np.max(np.abs(g)))
            h0 = 1.0 / gmax if gmax > 0.0 else 0.0
            d = -h0 * g
        gq = float(np.sum(g * d))
        gamma, accepted, trials = 1.0, False, 0
        for t in range(ls_max_trials):
            trials = t + 1
            ot, _ = fun(x + gamma * d, want_grad=False)
            Jt = ot.J if hasattr(ot, "J") else float(ot)
            if Jt <= J + armijo_c * gamma * gq:
                accepted = True
                break
            gamma *= 0.5
        hist.append(_r.GNStep(J, D, S, P, float(np.sqrt(np.sum(g * g))), gq, len(pairs), h0,
                              gamma if accepted else 0.0, trials, accepted))
        if not accepted:
            break
        s = gamma * d
        x = x + s
        obj, g_new = fun(x)
        if g_new is not None:
            y = g_new - g
            sy = float(np.sum(s * y))
            if sy > PAIR_CURVATURE * float(np.linalg.norm(s)) * float(np.linalg.norm(y)):
                pairs.append((s, y, 1.0 / sy))
                if len(pairs) > memory:
                    pairs.pop(0)
        g = g_new
    return x, hist


def lbfgs_cols(Ip, Im, b, hc, *, alpha=_r.ALPHA, beta=_r.BETA, iters=5, memory=10,
               armijo_c=1e-4, ls_max_trials=10):
    """L-BFGS on the objective of Eq. (6) in column form (PE axis last)."""
    def fun(x, want_grad=True):
        if not want_grad:
            return _r.objective_cols(Ip, Im, x, hc, alpha, beta), None
        obj, g, _ = _r.objective_gradient_cols(Ip, Im, x, hc, alpha, beta)
        return obj, g
    return lbfgs(fun, b, iters=iters, memory=memory, armijo_c=armijo_c,
                 ls_max_trials=ls_max_trials)


def lbfgs_level(Ip, Im, b, pe, h, **kw):
    """L-BFGS on one level in the caller's layout."""
    hc = _r.col_spacing(h, pe)
    bcol, hist = lbfgs_cols(_r.to_cols(Ip, pe), _r.to_cols(Im, pe), _r.to_cols(b, pe), hc, **kw)
    return _r.from_cols(bcol, pe), hist
