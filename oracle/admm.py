"""FP64 NumPy oracle of the ADMM solver (Sec. 2.3.2, Eq. 8-11).

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never imports this.

The objective is split into F(b) = D(b) + alpha S3(b) + beta P(b), where S3 is the part of the
smoothness term along the phase-encoding (PE) axis, and G(z) = alpha (S1(z) + S2(z)), the parts
along the two other axes.  With the scaled multiplier u, one iteration is
    b <- argmin F(b) + (rho vol / 2) |b - z + u|^2          (Eq. 9: separable by column)
    z <- argmin G(z) + (rho vol / 2) |b - z + u|^2          (Eq. 10: a shifted 2D Laplacian per
                                                              PE index, inverted by FFT)
    u <- u + b - z                                          (Eq. 11)
and rho is adapted so that the primal and dual residuals stay close.

Readings of what the paper leaves open (used identically by the HIP path):

* R30 S3 keeps the Neumann differences along the PE axis; G uses periodic differences across the
  PE axis (S_d = (vol/2) sum over all n positions of (z_{i+1} - z_i)^2 / h_d^2, index i + 1 taken
  modulo n), which is what makes the z-update's blocks circulant and lets the FFT invert them
  exactly (the paper assumes periodic boundaries there).  ADMM therefore minimises
  D + alpha (S3 + S1 + S2 with periodic cross-axis differences) + beta P.
* R31 the b-update is one Gauss-Newton step on F_rho(b) = F(b) + (rho vol / 2)|b - c|^2,
  c = z - u, from the current b: the search direction solves the Gauss-Newton system of
  F_rho, which is block diagonal with one tridiagonal block per PE column, by Jacobi-
  preconditioned CG run independently on every column ("BlockPCG": per-column step sizes, a
  column stops after ``pcg_iters`` iterations, when its residual falls below ``pcg_rtol`` times
  its right-hand side, or when p^T H p <= 0); the step size is the Armijo search of the
  Gauss-Newton solver on F_rho.  A step that no trial accepts stops the level (b unchanged).
* R34 z and u start as z = b, u = 0 on every pyramid level; rho starts at ``rho0`` (default
  alpha) on every level.  After each iteration, with primal residual r = |b - z| and dual
  residual s = rho |z - z_prev|: rho <- 2 rho, u <- u / 2 if r > 10 s; rho <- rho / 2,
  u <- 2 u if s > 10 r (Boyd et al., Sec. 3.4.1, mu = 10, tau = 2).  The field returned is b.
* Every iteration is recorded as a GNStep: J = F_rho(b) before the step, D, S' = S3 + (rho /
  alpha)(1/2) vol |b - c|^2 (so that J = D + alpha S' + beta P), P, |grad|, grad.q, the largest
  column iteration count, the largest column relative residual, gamma, trials, accepted; plus
  the rho the iteration used.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import rgp as _r

MU, TAU = 10.0, 2.0


@dataclasses.dataclass
class ADMMStep(_r.GNStep):
    rho: float = math.nan


def pe_diff_sq(b, hp):
    """sum |Delta_PE b|^2 / h_pe^2 (Neumann, the PE part of S)."""
    d = np.diff(b, axis=-1)
    return float(np.sum(d * d)) / (hp * hp)


def pe_laplacian(b, hp):
    """L3 b = Delta_PE^T Delta_PE b / h_pe^2."""
    return _r.dif_T(_r.dif(b, hp), hp)


def cross_laplacian_periodic(z, hc):
    """L12 z with periodic differences along the two cross axes (axes 0 and 1 of column form)."""
    out = np.zeros_like(z)
    for ax in (0, 1):
        d = (np.roll(z, -1, axis=ax) - z) / (hc[ax] ** 2)   # forward differences, wrapped
        out -= d
        out += np.roll(d, 1, axis=ax)
    return out


def g_value(z, hc, alpha):
    """G(z) = alpha (S1 + S2) with periodic cross-axis differences."""
    vol = hc[0] * hc[1] * hc[2]
    tot = 0.0
    for ax in (0, 1):
        d = np.roll(z, -1, axis=ax) - z
        tot += float(np.sum(d * d)) / (hc[ax] ** 2)
    return 0.5 * vol * alpha * tot


def z_update(v, rho, alpha, hc):
    """argmin_z G(z) + (rho vol / 2)|v - z|^2: (alpha L12 + rho I) z = rho v, solved per PE index
    by a 2D FFT over the cross axes (eigenvalues (2 - 2 cos(2 pi k / n)) / h^2 per axis)."""
    na, nb = v.shape[0], v.shape[1]
    la = (2.0 - 2.0 * np.cos(2.0 * np.pi * np.arange(na) / na)) / hc[0] ** 2
    lb = (2.0 - 2.0 * np.cos(2.0 * np.pi * np.arange(nb) / nb)) / hc[1] ** 2
    lam = la[:, None, None] + lb[None, :, None]
    vh = np.fft.fft2(rho * v, axes=(0, 1))
    return np.real(np.fft.ifft2(vh / (alpha * lam + rho), axes=(0, 1)))


def f_rho(Ip, Im, b, hc, c, rho, alpha, beta):
    """F_rho at b: (J, D, S', P) as recorded (R34), or J = inf outside the barrier."""
    hp = hc[2]
    vol = hc[0] * hc[1] * hc[2]
    Tp, _, _, Db = _r.transform_cols(Ip, b, hp, +1.0)
    Tm, _, _, _ = _r.transform_cols(Im, b, hp, -1.0)
    r = Tp - Tm
    D = 0.5 * vol * float(np.sum(r * r))
    e = b - c
    Sp = 0.5 * vol * (pe_diff_sq(b, hp) + (rho / alpha) * float(np.sum(e * e)))
    if np.any(np.abs(Db) >= 1.0):
        return math.inf, D, Sp, math.inf
    P = 0.5 * vol * float(np.sum(_r.phi(Db)))
    return D + alpha * Sp + beta * P, D, Sp, P


def f_rho_gradient(Ip, Im, b, hc, c, rho, alpha, beta):
    """Gradient of F_rho and its Gauss-Newton bands per column: (grad, diag, off) with off[k]
    the coupling of PE nodes k and k+1 (0 at the last node); None when outside the barrier."""
    hp = hc[2]
    vol = hc[0] * hc[1] * hc[2]
    obj, g, lin = _r.objective_gradient_cols(Ip, Im, b, hc, alpha, beta)
    if g is None:
        return None
    # drop the cross-axis (Neumann) smoothness of J, add the PE part and the proximal term
    g = g - alpha * vol * _r.laplacian(b, hc) + alpha * vol * pe_laplacian(b, hp)
    g = g + rho * vol * (b - c)
    # bands: data + barrier of the GN operator, the PE Laplacian, the proximal identity
    left = 0.5 * lin.c1 + lin.c2 / hp    # d r_j / d b_{j+1}
    right = 0.5 * lin.c1 - lin.c2 / hp   # d r_j / d b_j
    p2 = 0.5 * beta * vol * lin.phi2 / (hp * hp)
    m1 = b.shape[-1]
    diag = np.zeros(b.shape)
    diag[..., 1:] += vol * left * left + p2
    diag[..., :-1] += vol * right * right + p2
    cnt = np.full(m1, 2.0)
    cnt[0] = cnt[-1] = 1.0
    diag += alpha * vol * cnt / (hp * hp) + rho * vol
    off = np.zeros(b.shape)
    off[..., :-1] = vol * right * left - p2 - alpha * vol / (hp * hp)
    return g, diag, off


def tri_matvec(diag, off, v):
    """Per-column tridiagonal product with the bands of f_rho_gradient."""
    out = diag * v
    out[..., :-1] += off[..., :-1] * v[..., 1:]
    out[..., 1:] += off[..., :-1] * v[..., :-1]
    return out


def block_pcg(diag, off, rhs, maxit, rtol):
    """Jacobi-preconditioned CG on every column independently (R31), from x = 0.  Returns
    (x, iterations per column, final relative residual per column)."""
    x = np.zeros_like(rhs)
    r = rhs.copy()
    nb = np.sqrt(np.sum(r * r, axis=-1))
    z = r / diag
    p = z.copy()
    rz = np.sum(r * z, axis=-1)
    active = nb > 0.0
    its = np.zeros(nb.shape, dtype=np.int64)
    relres = np.where(active, 1.0, 0.0)
    for _ in range(maxit):
        if not np.any(active):
            break
        q = tri_matvec(diag, off, p)
        pq = np.sum(p * q, axis=-1)
        active &= pq > 0.0
        a = np.where(active, rz / np.where(pq > 0.0, pq, 1.0), 0.0)[..., None]
        x = x + a * p
        r = r - a * q
        its += active
        rr = np.sqrt(np.sum(r * r, axis=-1))
        relres = np.where(active, rr / np.where(nb > 0.0, nb, 1.0), relres)
        cont = active & ~(relres < rtol)
        z = r / diag
        rzn = np.sum(r * z, axis=-1)
        beta = np.where(cont, rzn / np.where(rz != 0.0, rz, 1.0), 0.0)[..., None]
        p = np.where(cont[..., None], z + beta * p, p)
        rz = np.where(cont, rzn, rz)
        active = cont
    return x, its, relres


def admm_cols(Ip, Im, b, hc, *, alpha=_r.ALPHA, beta=_r.BETA, iters=5, pcg_iters=10,
              pcg_rtol=0.1, rho0=None, armijo_c=1e-4, ls_max_trials=10):
    """``iters`` ADMM iterations (R30, R31, R34) on one level, column form.  Returns (b, list of
    ADMMStep)."""
    vol = hc[0] * hc[1] * hc[2]
    b = np.array(b, dtype=np.float64)
    z = b.copy()
    u = np.zeros_like(b)
    rho = float(alpha if rho0 is None else rho0)
    hist = []
    for _ in range(iters):
        c = z - u
        J, D, Sp, P = f_rho(Ip, Im, b, hc, c, rho, alpha, beta)
        res = f_rho_gradient(Ip, Im, b, hc, c, rho, alpha, beta)
        if res is None:
            hist.append(ADMMStep(J, D, Sp, P, math.nan, math.nan, 0, math.nan, 0.0, 0, False,
                                 rho))
            break
        g, dg, of = res
        q, its, rel = block_pcg(dg, of, -g, pcg_iters, pcg_rtol)
        gq = float(np.sum(g * q))
        gamma, accepted, trials = 1.0, False, 0
        for t in range(ls_max_trials):
            trials = t + 1
            Jt = f_rho(Ip, Im, b + gamma * q, hc, c, rho, alpha, beta)[0]
            if Jt <= J + armijo_c * gamma * gq:
                accepted = True
                break
            gamma *= 0.5
        hist.append(ADMMStep(J, D, Sp, P, float(np.sqrt(np.sum(g * g))), gq, int(its.max()),
                             float(rel.max()), gamma if accepted else 0.0, trials, accepted,
                             rho))
        if not accepted:
            break
        b = b + gamma * q
        z_prev = z
        z = z_update(b + u, rho, alpha, hc)
        u = u + b - z
        rp = math.sqrt(float(np.sum((b - z) ** 2)))
        sd = rho * math.sqrt(float(np.sum((z - z_prev) ** 2)))
        if rp > MU * sd:
            rho *= TAU
            u = u / TAU
        elif sd > MU * rp:
            rho /= TAU
            u = u * TAU
    return b, hist


def admm_level(Ip, Im, b, pe, h, **kw):
    """ADMM on one level in the caller's layout."""
    hc = _r.col_spacing(h, pe)
    bcol, hist = admm_cols(_r.to_cols(Ip, pe), _r.to_cols(Im, pe), _r.to_cols(b, pe), hc, **kw)
    return _r.from_cols(bcol, pe), hist
