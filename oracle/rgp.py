"""FP64 NumPy oracle of the hot path: OT initialisation, objective, gradient, Gauss-Newton
operator, Jacobi-preconditioned CG, Armijo Gauss-Newton, multilevel pyramid and correction.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never imports this.

Everything here follows the paper (Julian and Ruthotto, "PyHySCO: GPU-enabled susceptibility
artifact distortion correction in seconds") step by step, in float64, with no blocking or
fusion.  Conventions:

* Arrays arrive in the caller's layout ``[m0][m1][m2]`` with the phase-encoding (PE) axis ``pe``.
  Internally the PE axis is moved last (Sec. 2.4.1 permutes it last too), giving column form
  ``[na][nb][m]`` for images and ``[na][nb][m+1]`` for the field map.
* The field map lives on the e_pe-staggered grid of Sec. 2.1: cell centres across the PE axis,
  nodes along it (m + 1 of them).  Images are cell-centred.
* ``h = (h0, h1, h2)`` are voxel sizes in caller axis order; ``vol = h0 h1 h2`` is the weight of
  the midpoint quadrature of Sec. 2.1.

Readings of points the paper leaves open (each one is also listed in the design notes):

* R1  the 1D linear image model is zero outside the column;
* R2  at a knot the image slope is the right-sided one, and sample positions are formed in index
  space, xi = j +- (A b)_j / h_pe;
* R3  the "five-point" negative Laplacian of Eq. (5) is the 3D seven-point stencil on the
  staggered field with Neumann boundaries (positive semi-definite, constants in its kernel);
* R4  D, S and P all carry the weight vol / 2;
* R5  phi = +inf outside (-1, 1) makes J = +inf (a value, not an error);
* R7  OT positivity shift s = max(0, -min I) + eps * max |I| over both images;
* R8  nodal CDFs C_k = sum_{j<k} i_j / sum_j i_j, k = 0..m;
* R9  pseudo-inverse = linear spline through (C_k, k h);
* R10 b0 = (1/4) [C+^{-1}(C-) - C-^{-1}(C+)];
* R11 OT guard: columns with |D b0| > 0.99 are clipped and re-integrated from b0_0 = 0;
* R13 PCG relative residual is measured against |grad J|;
* R14 Armijo with c = 1e-4, gamma = 1, halving, at most ``ls_max_trials`` trial steps;
* R16 pyramid: 2x2x2 mean restriction (ceil(m/2) cells), linear prolongation on the staggered grid
  with constant extrapolation at the outer half cells; b keeps physical units;
* R25 optional blur of the OT field: 3x3x3 Gaussian, standard deviation 1 voxel, weights
  normalised to sum 1, periodic over the field's node grid (the paper applies it as an FFT
  convolution, which wraps around);
* R27 failures of a solve are reported, first one wins, by a status code: an image with a
  non-finite value (no Gauss-Newton step is taken, the initial field is zero when OT would
  have made it), a level that starts from a field outside the barrier (J = +inf: the level
  stops with b unchanged), a step that no Armijo trial accepts (the level stops with b
  unchanged).  Later levels still run.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

ALPHA = 300.0  # smoothness weight fixed in Sec. 2.1
BETA = 1e-4    # barrier weight fixed in Sec. 2.1

# Status of a whole solve (R27); 0 when nothing failed.
STATUS_OK = 0
STATUS_NONFINITE = -4    # an input image holds a NaN or an infinity
STATUS_BARRIER = -5      # a level started from a field with |D b| >= 1 somewhere (J = +inf)
STATUS_LINESEARCH = -6   # no Armijo trial was accepted in some Gauss-Newton step


# --------------------------------------------------------------------------------------------
# Layout helpers
# --------------------------------------------------------------------------------------------

def to_cols(x: np.ndarray, pe: int) -> np.ndarray:
    """Caller layout -> column form (PE axis last), as a float64 copy."""
    return np.ascontiguousarray(np.moveaxis(np.asarray(x, dtype=np.float64), pe, -1))


def from_cols(x: np.ndarray, pe: int) -> np.ndarray:
    """Column form -> caller layout."""
    return np.ascontiguousarray(np.moveaxis(x, -1, pe))


def col_spacing(h: Sequence[float], pe: int) -> tuple:
    """Spacings in column-form axis order (the two cross axes, then the PE axis)."""
    cross = [float(h[d]) for d in range(3) if d != pe]
    return (cross[0], cross[1], float(h[pe]))


# --------------------------------------------------------------------------------------------
# Operators along the PE axis (Sec. 2.1 discretisation, Sec. 2.4.2 "averaging" and
# "finite difference" linear operators)
# --------------------------------------------------------------------------------------------

def avg(b: np.ndarray) -> np.ndarray:
    """(A b)_j = (b_j + b_{j+1}) / 2: nodes -> cell centres."""
    return 0.5 * (b[..., :-1] + b[..., 1:])


def dif(b: np.ndarray, hp: float) -> np.ndarray:
    """(D b)_j = (b_{j+1} - b_j) / h: nodes -> cell centres."""
    return (b[..., 1:] - b[..., :-1]) / hp


def avg_T(u: np.ndarray) -> np.ndarray:
    """Adjoint of ``avg``: (A^T u)_k = (u_{k-1} + u_k) / 2 with u_{-1} = u_m = 0."""
    out = np.zeros(u.shape[:-1] + (u.shape[-1] + 1,))
    out[..., :-1] += 0.5 * u
    out[..., 1:] += 0.5 * u
    return out


def dif_T(u: np.ndarray, hp: float) -> np.ndarray:
    """Adjoint of ``dif``: (D^T u)_k = (u_{k-1} - u_k) / h with u_{-1} = u_m = 0."""
    out = np.zeros(u.shape[:-1] + (u.shape[-1] + 1,))
    out[..., :-1] -= u / hp
    out[..., 1:] += u / hp
    return out


# --------------------------------------------------------------------------------------------
# Image model (Sec. 2.4.1: piecewise linear 1D interpolation along the PE axis)
# --------------------------------------------------------------------------------------------

def interp_lin(I: np.ndarray, xi: np.ndarray, hp: float):
    """Linear interpolant of the cell samples I[..., k] at index-space positions xi.

    Returns (value, slope), the slope being d/dx in physical units.  Samples outside 0..m-1 are
    zero (R1).  At a knot the right-sided interval [floor(xi), floor(xi) + 1] is used (R2).
    """
    m = I.shape[-1]
    k0f = np.floor(xi)
    w = xi - k0f
    k0 = k0f.astype(np.int64)
    k1 = k0 + 1

    def sample(k):
        ok = (k >= 0) & (k < m)
        kc = np.clip(k, 0, m - 1)
        return np.where(ok, np.take_along_axis(I, kc, axis=-1), 0.0)

    v0 = sample(k0)
    v1 = sample(k1)
    return (1.0 - w) * v0 + w * v1, (v1 - v0) / hp


# --------------------------------------------------------------------------------------------
# Barrier phi of Eq. (3) and its derivatives
# --------------------------------------------------------------------------------------------

def phi(z):
    """phi(z) = z^4 / (1 - z^2) on (-1, 1), +inf elsewhere (Eq. 3)."""
    z = np.asarray(z, dtype=np.float64)
    inside = np.abs(z) < 1.0
    zz = np.where(inside, z, 0.0)
    return np.where(inside, zz ** 4 / (1.0 - zz * zz), np.inf)


def dphi(z):
    """phi'(z) = 2 z^3 (2 - z^2) / (1 - z^2)^2 (only meaningful on (-1, 1))."""
    z = np.asarray(z, dtype=np.float64)
    q = 1.0 - z * z
    return 2.0 * z ** 3 * (2.0 - z * z) / (q * q)


def d2phi(z):
    """phi''(z) = 2 z^2 (6 - 3 z^2 + z^4) / (1 - z^2)^3 >= 0 on (-1, 1)."""
    z = np.asarray(z, dtype=np.float64)
    q = 1.0 - z * z
    z2 = z * z
    return 2.0 * z2 * (6.0 - 3.0 * z2 + z2 * z2) / (q * q * q)


# --------------------------------------------------------------------------------------------
# Smoothness term (Eq. 5) on the staggered field, Neumann boundaries (R3)
# --------------------------------------------------------------------------------------------

def smooth_sq(b: np.ndarray, hc: Sequence[float]) -> float:
    """sum_d |Delta_d b|^2 / h_d^2 = b^T L b over the three axes of the column-form field."""
    tot = 0.0
    for ax in range(3):
        d = np.diff(b, axis=ax)
        tot += float(np.sum(d * d)) / (hc[ax] ** 2)
    return tot


def laplacian(b: np.ndarray, hc: Sequence[float]) -> np.ndarray:
    """L b = sum_d Delta_d^T Delta_d b / h_d^2 (negative Laplacian, Neumann)."""
    out = np.zeros_like(b)
    for ax in range(3):
        d = np.diff(b, axis=ax) / (hc[ax] ** 2)
        n = b.shape[ax]
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        out[tuple(lo)] -= d
        out[tuple(hi)] += d
    return out


def laplacian_diag(shape: Sequence[int], hc: Sequence[float]) -> np.ndarray:
    """Diagonal of L: sum_d (number of neighbours along d) / h_d^2."""
    out = np.zeros(shape)
    for ax in range(3):
        n = shape[ax]
        cnt = np.full(n, 2.0)
        if n == 1:
            cnt[:] = 0.0
        else:
            cnt[0] = cnt[-1] = 1.0
        sh = [1, 1, 1]
        sh[ax] = n
        out += cnt.reshape(sh) / (hc[ax] ** 2)
    return out


# --------------------------------------------------------------------------------------------
# Mass-preserving transform (Eq. 1), distance (Eq. 2), objective (Eq. 4 / Eq. 6)
# --------------------------------------------------------------------------------------------

def _positions(m: int, Ab: np.ndarray, hp: float, sign: float) -> np.ndarray:
    j = np.arange(m, dtype=np.float64)
    return j + sign * (Ab / hp)


def transform_cols(I: np.ndarray, b: np.ndarray, hp: float, sign: float):
    """T[I, b, sign v] at the cell centres of every column (Eq. 1, Sec. 2.4.2).

    Returns (T, I_at, I_slope, Db): T = I(xi) (1 + sign Db) with xi = j + sign (A b)/h.
    """
    Ab = avg(b)
    Db = dif(b, hp)
    xi = _positions(I.shape[-1], Ab, hp, sign)
    val, slope = interp_lin(I, xi, hp)
    return val * (1.0 + sign * Db), val, slope, Db


@dataclasses.dataclass
class Objective:
    J: float
    D: float
    S: float
    P: float


def objective_cols(Ip, Im, b, hc, alpha=ALPHA, beta=BETA) -> Objective:
    """J = D + alpha S + beta P with weights vol/2 (Eq. 2, 3, 5, 6; R4, R5)."""
    hp = hc[2]
    vol = hc[0] * hc[1] * hc[2]
    Tp, _, _, Db = transform_cols(Ip, b, hp, +1.0)
    Tm, _, _, _ = transform_cols(Im, b, hp, -1.0)
    r = Tp - Tm
    D = 0.5 * vol * float(np.sum(r * r))
    S = 0.5 * vol * smooth_sq(b, hc)
    if np.any(np.abs(Db) >= 1.0):
        P = math.inf
    else:
        P = 0.5 * vol * float(np.sum(phi(Db)))
    return Objective(D + alpha * S + beta * P, D, S, P)


@dataclasses.dataclass
class Linearization:
    """Everything the GN operator needs about the current iterate (Sec. 2.4.4)."""

    c1: np.ndarray      # dr/d(Ab) per cell
    c2: np.ndarray      # dr/d(Db) per cell
    phi2: np.ndarray    # phi''(Db) per cell
    hc: tuple
    alpha: float
    beta: float

    @property
    def vol(self):
        return self.hc[0] * self.hc[1] * self.hc[2]


def objective_gradient_cols(Ip, Im, b, hc, alpha=ALPHA, beta=BETA):
    """Objective, gradient and GN linearisation at b (column form).

    grad J = vol [A^T(c1 r) + D^T(c2 r)] + alpha vol L b + (beta vol / 2) D^T phi'(D b)
    with r = T+ - T-, c1 = I+'(xi+)(1 + Db) + I-'(xi-)(1 - Db), c2 = I+(xi+) + I-(xi-).
    Returns (Objective, grad or None when J = +inf, Linearization or None).
    """
    hp = hc[2]
    vol = hc[0] * hc[1] * hc[2]
    Tp, vp, sp, Db = transform_cols(Ip, b, hp, +1.0)
    Tm, vm, sm, _ = transform_cols(Im, b, hp, -1.0)
    r = Tp - Tm
    D = 0.5 * vol * float(np.sum(r * r))
    S = 0.5 * vol * smooth_sq(b, hc)
    if np.any(np.abs(Db) >= 1.0):
        return Objective(math.inf, D, S, math.inf), None, None
    P = 0.5 * vol * float(np.sum(phi(Db)))
    obj = Objective(D + alpha * S + beta * P, D, S, P)
    c1 = sp * (1.0 + Db) + sm * (1.0 - Db)
    c2 = vp + vm
    g = vol * (avg_T(c1 * r) + dif_T(c2 * r, hp))
    g += alpha * vol * laplacian(b, hc)
    g += 0.5 * beta * vol * dif_T(dphi(Db), hp)
    lin = Linearization(c1, c2, d2phi(Db), tuple(hc), alpha, beta)
    return obj, g, lin


def interp_lin_T(u: np.ndarray, xi: np.ndarray, m: int) -> np.ndarray:
    """Adjoint of the value part of ``interp_lin``: G[..., k] = sum_j u_j ((1 - w_j) [k0_j = k]
    + w_j [k0_j + 1 = k]) over k = 0..m-1, with k0 = floor(xi), w = xi - k0 (R1, R2; samples
    outside 0..m-1 receive nothing)."""
    k0f = np.floor(xi)
    w = xi - k0f
    k0 = k0f.astype(np.int64)
    G = np.zeros(u.shape[:-1] + (m,))
    lead = np.indices(u.shape[:-1])
    for k, wt in ((k0, 1.0 - w), (k0 + 1, w)):
        ok = (k >= 0) & (k < m)
        idx = tuple(np.broadcast_to(ax[..., None], u.shape)[ok] for ax in lead) + (k[ok],)
        np.add.at(G, idx, (u * wt)[ok])
    return G


def image_gradient_cols(Ip, Im, b, hc):
    """Gradient of J with respect to the two images (only D depends on them, Eq. 2):
    dJ/dI+ = vol A+^T (r (1 + Db)), dJ/dI- = -vol A-^T (r (1 - Db)), with A+- the linear
    interpolation at xi+- = j +- (A b)/h and r = T+ - T-."""
    hp = hc[2]
    vol = hc[0] * hc[1] * hc[2]
    m = Ip.shape[-1]
    Tp, _, _, Db = transform_cols(Ip, b, hp, +1.0)
    Tm, _, _, _ = transform_cols(Im, b, hp, -1.0)
    r = Tp - Tm
    Ab = avg(b)
    gp = vol * interp_lin_T(r * (1.0 + Db), _positions(m, Ab, hp, +1.0), m)
    gm = -vol * interp_lin_T(r * (1.0 - Db), _positions(m, Ab, hp, -1.0), m)
    return gp, gm


def gn_matvec_cols(lin: Linearization, v: np.ndarray) -> np.ndarray:
    """H_J v = vol [A^T(c1 w) + D^T(c2 w)] + alpha vol L v + (beta vol/2) D^T(phi'' D v),
    w = c1 A v + c2 D v: the Gauss-Newton approximation of Sec. 2.3.1 (drops sum r nabla^2 r)."""
    hp = lin.hc[2]
    vol = lin.vol
    w = lin.c1 * avg(v) + lin.c2 * dif(v, hp)
    out = vol * (avg_T(lin.c1 * w) + dif_T(lin.c2 * w, hp))
    out += lin.alpha * vol * laplacian(v, lin.hc)
    out += 0.5 * lin.beta * vol * dif_T(lin.phi2 * dif(v, hp), hp)
    return out


def gn_diag_cols(lin: Linearization) -> np.ndarray:
    """Diagonal of H_J, the Jacobi preconditioner of Sec. 2.3.1."""
    hp = lin.hc[2]
    vol = lin.vol
    left = 0.5 * lin.c1 + lin.c2 / hp    # d r_j / d b_{j+1}
    right = 0.5 * lin.c1 - lin.c2 / hp   # d r_j / d b_j
    nshape = lin.c1.shape[:-1] + (lin.c1.shape[-1] + 1,)
    d = np.zeros(nshape)
    d[..., 1:] += left * left
    d[..., :-1] += right * right
    d *= vol
    d += lin.alpha * vol * laplacian_diag(nshape, lin.hc)
    p2 = 0.5 * lin.beta * vol * lin.phi2 / (hp * hp)
    d[..., 1:] += p2
    d[..., :-1] += p2
    return d


# --------------------------------------------------------------------------------------------
# Jacobi-preconditioned CG (Sec. 2.3.1; Hestenes-Stiefel)
# --------------------------------------------------------------------------------------------

@dataclasses.dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    relres: float


def pcg(apply_H, rhs: np.ndarray, diag: np.ndarray, maxit: int, rtol: float,
        record: Optional[list] = None) -> PCGResult:
    """Textbook PCG from x0 = 0 with the Jacobi preconditioner diag^{-1}.

    Stops after ``maxit`` iterations, when p^T H p <= 0 (the step is not taken), or when
    |r| / |rhs| < rtol (R13).  ``record`` (a list) receives every residual r_i.
    """
    x = np.zeros_like(rhs)
    r = rhs.copy()
    nb = float(np.sqrt(np.sum(rhs * rhs)))
    if nb == 0.0:
        return PCGResult(x, 0, 0.0)
    if record is not None:
        record.append(r.copy())
    z = r / diag
    p = z.copy()
    rz = float(np.sum(r * z))
    it = 0
    relres = 1.0
    for i in range(maxit):
        q = apply_H(p)
        pq = float(np.sum(p * q))
        if pq <= 0.0:
            break
        a = rz / pq
        x = x + a * p
        r = r - a * q
        it = i + 1
        if record is not None:
            record.append(r.copy())
        relres = float(np.sqrt(np.sum(r * r))) / nb
        if relres < rtol:
            break
        z = r / diag
        rz_new = float(np.sum(r * z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    return PCGResult(x, it, relres)


# --------------------------------------------------------------------------------------------
# Gauss-Newton with Armijo backtracking (Sec. 2.3.1, Eq. 7)
# --------------------------------------------------------------------------------------------

@dataclasses.dataclass
class GNStep:
    J: float
    D: float
    S: float
    P: float
    gnorm: float
    gq: float
    pcg_iters: int
    pcg_relres: float
    gamma: float
    trials: int
    accepted: bool


def gauss_newton_cols(Ip, Im, b, hc, *, alpha=ALPHA, beta=BETA, gn_iters=5, pcg_iters=10,
                      pcg_rtol=0.0, armijo_c=1e-4, ls_max_trials=10):
    """``gn_iters`` GN steps b <- b + gamma q, H_J q = -grad J solved by PCG.

    gamma = 1, halved until J(b + gamma q) <= J(b) + c gamma grad^T q (J = +inf fails), at most
    ``ls_max_trials`` trials; when no trial succeeds the iteration stops with b unchanged.
    Returns (b, list of GNStep).
    """
    b = np.array(b, dtype=np.float64)
    hist: List[GNStep] = []
    for _ in range(gn_iters):
        obj, g, lin = objective_gradient_cols(Ip, Im, b, hc, alpha, beta)
        if g is None:
            hist.append(GNStep(obj.J, obj.D, obj.S, obj.P, math.nan, math.nan, 0, math.nan, 0.0, 0, False))
            break
        d = gn_diag_cols(lin)
        res = pcg(lambda v: gn_matvec_cols(lin, v), -g, d, pcg_iters, pcg_rtol)
        q = res.x
        gq = float(np.sum(g * q))
        gamma = 1.0
        accepted = False
        trials = 0
        for t in range(ls_max_trials):
            trials = t + 1
            Jt = objective_cols(Ip, Im, b + gamma * q, hc, alpha, beta).J
            if Jt <= obj.J + armijo_c * gamma * gq:
                accepted = True
                break
            gamma *= 0.5
        gn = float(np.sqrt(np.sum(g * g)))
        hist.append(GNStep(obj.J, obj.D, obj.S, obj.P, gn, gq, res.iters, res.relres,
                           gamma if accepted else 0.0, trials, accepted))
        if not accepted:
            break
        b = b + gamma * q
    return b, hist


# --------------------------------------------------------------------------------------------
# Multilevel pyramid transfers (coarse-to-fine schedule; R16)
# --------------------------------------------------------------------------------------------

def restrict_image(I: np.ndarray) -> np.ndarray:
    """Coarse cell = mean of the existing fine cells of its 2x2x2 block; ceil(m/2) cells."""
    I = np.asarray(I, dtype=np.float64)
    m = I.shape
    mc = tuple((s + 1) // 2 for s in m)
    pad = [(0, 2 * c - s) for s, c in zip(m, mc)]
    S = np.pad(I, pad).reshape(mc[0], 2, mc[1], 2, mc[2], 2).sum(axis=(1, 3, 5))
    N = np.pad(np.ones(m), pad).reshape(mc[0], 2, mc[1], 2, mc[2], 2).sum(axis=(1, 3, 5))
    return S / N


def restrict_image_T(g: np.ndarray, fine_shape: Sequence[int]) -> np.ndarray:
    """Adjoint of restrict_image: fine cell f receives g at its coarse cell divided by the number
    of existing fine cells of that cell's 2x2x2 block."""
    m = tuple(int(s) for s in fine_shape)
    mc = tuple((s + 1) // 2 for s in m)
    g = np.asarray(g, dtype=np.float64)
    assert g.shape == mc
    pad = [(0, 2 * c - s) for s, c in zip(m, mc)]
    N = np.pad(np.ones(m), pad).reshape(mc[0], 2, mc[1], 2, mc[2], 2).sum(axis=(1, 3, 5))
    up = g / N
    for ax in range(3):
        up = np.repeat(up, 2, axis=ax)
    return up[:m[0], :m[1], :m[2]]


def _prolong_weights_cells(mf: int, mc: int) -> np.ndarray:
    """Fine-by-coarse linear interpolation matrix for a cell-centred axis (clamped ends)."""
    P = np.zeros((mf, mc))
    for j in range(mf):
        t = (j + 0.5) / 2.0 - 0.5
        t = min(max(t, 0.0), mc - 1.0)
        i0 = int(math.floor(t))
        if i0 >= mc - 1:
            P[j, mc - 1] = 1.0
            continue
        w = t - i0
        P[j, i0] += 1.0 - w
        P[j, i0 + 1] += w
    return P


def _prolong_weights_nodes(mf: int, mc: int) -> np.ndarray:
    """Fine-by-coarse linear interpolation for the node axis (mf+1 by mc+1)."""
    P = np.zeros((mf + 1, mc + 1))
    for k in range(mf + 1):
        t = min(k / 2.0, float(mc))
        i0 = int(math.floor(t))
        if i0 >= mc:
            P[k, mc] = 1.0
            continue
        w = t - i0
        P[k, i0] += 1.0 - w
        P[k, i0 + 1] += w
    return P


def prolong_field(bc: np.ndarray, fine_shape: Sequence[int], pe: int) -> np.ndarray:
    """Linear prolongation of a staggered field map (caller layout) to the finer level."""
    coarse_cells = list(bc.shape)
    coarse_cells[pe] -= 1
    out = np.asarray(bc, dtype=np.float64)
    for ax in range(3):
        if ax == pe:
            P = _prolong_weights_nodes(int(fine_shape[ax]), coarse_cells[ax])
        else:
            P = _prolong_weights_cells(int(fine_shape[ax]), coarse_cells[ax])
        out = np.moveaxis(np.tensordot(P, np.moveaxis(out, ax, 0), axes=(1, 0)), 0, ax)
    return out


# --------------------------------------------------------------------------------------------
# Optimal-transport initialisation (Sec. 2.2)
# --------------------------------------------------------------------------------------------

def ot_shift(Ip: np.ndarray, Im: np.ndarray, eps: float) -> float:
    """Global positivity shift s = max(0, -min) + eps * max|.| over both images (R7)."""
    lo = min(float(np.min(Ip)), float(np.min(Im)))
    hi = max(float(np.max(np.abs(Ip))), float(np.max(np.abs(Im))))
    return max(0.0, -lo) + eps * hi


def nodal_cdf(i: np.ndarray) -> np.ndarray:
    """C_k = sum_{j<k} i_j / sum_j i_j for k = 0..m (R8)."""
    S = np.concatenate([[0.0], np.cumsum(i)])
    C = S / S[-1]
    C[0] = 0.0
    C[-1] = 1.0
    return C


def cdf_inverse_index(C: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Linear-spline pseudo-inverse of a nodal CDF in index units (R9).

    For r in (C_i, C_{i+1}] returns i + (r - C_i) / (C_{i+1} - C_i); r <= C_0 gives 0 and
    r >= C_m gives m.
    """
    m = C.size - 1
    r = np.asarray(r, dtype=np.float64)
    i = np.searchsorted(C, r, side="left") - 1
    out = np.empty_like(r)
    lo = i < 0
    hi = i >= m
    mid = ~(lo | hi)
    ii = i[mid]
    out[mid] = ii + (r[mid] - C[ii]) / (C[ii + 1] - C[ii])
    out[lo] = 0.0
    out[hi] = float(m)
    return out


@dataclasses.dataclass
class OTResult:
    b0: np.ndarray          # caller layout, staggered
    guarded_cells: int      # cells whose slope the guard clipped
    shift: float


def ot_init(Ip: np.ndarray, Im: np.ndarray, pe: int, h: Sequence[float], *, eps=1e-3,
            guard=True, guard_slope=0.99) -> OTResult:
    """Column-wise 1D OT initial field map (Sec. 2.2, Fig. 2/3 construction).

    Per column: shift to positive, nodal CDFs C+ and C-, linear-spline inverses, and
    b0_k = (1/4) [C+^{-1}(C-_k) - C-^{-1}(C+_k)], i.e. the average of the displacement of the
    halfway map T- = C_half^{-1} o C- and the negated displacement of T+ (R10).  Columns whose
    total mass is not positive get b0 = 0.  Guard (R11): in columns where some
    |D b0| > guard_slope, the slopes are clipped to +-guard_slope and b0 is re-integrated from
    b0_0 = 0.
    """
    hp = float(h[pe])
    s = ot_shift(Ip, Im, eps)
    P = to_cols(Ip, pe) + s
    M = to_cols(Im, pe) + s
    sh = P.shape[:-1]
    m = P.shape[-1]
    Pf = P.reshape(-1, m)
    Mf = M.reshape(-1, m)
    b0 = np.zeros((Pf.shape[0], m + 1))
    clipped = 0
    for c in range(Pf.shape[0]):
        if not (np.sum(Pf[c]) > 0.0 and np.sum(Mf[c]) > 0.0):
            continue
        Cp = nodal_cdf(Pf[c])
        Cm = nodal_cdf(Mf[c])
        col = 0.25 * hp * (cdf_inverse_index(Cp, Cm) - cdf_inverse_index(Cm, Cp))
        if guard:
            slope = np.diff(col) / hp
            bad = np.abs(slope) > guard_slope
            if np.any(bad):
                clipped += int(np.count_nonzero(bad))
                slope = np.clip(slope, -guard_slope, guard_slope)
                col = np.concatenate([[0.0], np.cumsum(slope * hp)])
        b0[c] = col
    return OTResult(from_cols(b0.reshape(sh + (m + 1,)), pe), clipped, s)


def gaussian_blur3(b: np.ndarray, sigma: float = 1.0) -> np.ndarray:
    """Optional smoothing of the OT field (Sec. 2.2, last step; Sec. 2.4, the InitializeOT
    description): convolution with the 3x3x3 Gaussian of standard deviation ``sigma`` (in voxels),
    normalised to sum 1, with periodic wrap-around (R25).  Written as the 27-term sum."""
    b = np.asarray(b, dtype=np.float64)
    offs = (-1, 0, 1)
    w = {(i, j, k): math.exp(-(i * i + j * j + k * k) / (2.0 * sigma * sigma))
         for i in offs for j in offs for k in offs}
    total = sum(w.values())
    out = np.zeros_like(b)
    for (i, j, k), wt in w.items():
        # out[x] = sum_d w(d) b[x + d], indices taken modulo the extents
        out += (wt / total) * np.roll(b, shift=(-i, -j, -k), axis=(0, 1, 2))
    return out


# --------------------------------------------------------------------------------------------
# Caller-layout wrappers
# --------------------------------------------------------------------------------------------

def objective(Ip, Im, b, pe, h, alpha=ALPHA, beta=BETA) -> Objective:
    hc = col_spacing(h, pe)
    return objective_cols(to_cols(Ip, pe), to_cols(Im, pe), to_cols(b, pe), hc, alpha, beta)


def objective_gradient(Ip, Im, b, pe, h, alpha=ALPHA, beta=BETA):
    """(Objective, grad in caller layout or None, Linearization in column form or None)."""
    hc = col_spacing(h, pe)
    obj, g, lin = objective_gradient_cols(to_cols(Ip, pe), to_cols(Im, pe), to_cols(b, pe), hc,
                                          alpha, beta)
    return obj, (None if g is None else from_cols(g, pe)), lin


def image_gradient(Ip, Im, b, pe, h):
    """(dJ/dI+, dJ/dI-) in caller layout (cells)."""
    hc = col_spacing(h, pe)
    gp, gm = image_gradient_cols(to_cols(Ip, pe), to_cols(Im, pe), to_cols(b, pe), hc)
    return from_cols(gp, pe), from_cols(gm, pe)


def gn_matvec(lin: Linearization, v, pe):
    return from_cols(gn_matvec_cols(lin, to_cols(v, pe)), pe)


def gn_diag(lin: Linearization, pe):
    return from_cols(gn_diag_cols(lin), pe)


def pcg_solve(lin: Linearization, rhs, pe, maxit, rtol) -> PCGResult:
    """PCG on H_J x = rhs (caller layout in and out)."""
    d = gn_diag_cols(lin)
    res = pcg(lambda v: gn_matvec_cols(lin, v), to_cols(rhs, pe), d, maxit, rtol)
    return PCGResult(from_cols(res.x, pe), res.iters, res.relres)


def transform(I, b, pe, h, sign):
    """Corrected image T[I, b, sign v] (caller layout, cells)."""
    T, _, _, _ = transform_cols(to_cols(I, pe), to_cols(b, pe), float(h[pe]), sign)
    return from_cols(T, pe)


def gauss_newton(Ip, Im, b, pe, h, **kw):
    hc = col_spacing(h, pe)
    bcol, hist = gauss_newton_cols(to_cols(Ip, pe), to_cols(Im, pe), to_cols(b, pe), hc, **kw)
    return from_cols(bcol, pe), hist


@dataclasses.dataclass
class SolveResult:
    b: np.ndarray
    T_plus: np.ndarray
    T_minus: np.ndarray
    b_ot: Optional[np.ndarray]
    ot_guarded: int
    levels: list          # per level: (shape, h, list of GNStep)
    status: int = STATUS_OK


def pyramid(Ip, Im, h, levels):
    """Images and spacings per level, finest first."""
    out = [(np.asarray(Ip, np.float64), np.asarray(Im, np.float64), tuple(float(x) for x in h))]
    for _ in range(levels - 1):
        P, M, hh = out[-1]
        out.append((restrict_image(P), restrict_image(M), tuple(2.0 * x for x in hh)))
    return out


def pyramid_objective(Ip, Im, fields, pe, h, alpha=ALPHA, beta=BETA, weights=None, grad=True):
    """sum_l w_l J_l(R^l I+, R^l I-, b_l, 2^l h) over the levels of the pyramid (Sec. 3.4; the
    field of each level given) and its gradients: (J, [dJ/db_l], dJ/dI+, dJ/dI-), the image
    gradients carried to the finest level by the adjoint restriction, coarsest level first.
    With grad=False: (J, None, None, None)."""
    L = len(fields)
    w = [1.0] * L if weights is None else [float(x) for x in weights]
    levels = pyramid(Ip, Im, h, L)
    if not grad:
        J = sum(wl * objective(P, M, b, pe, hl, alpha, beta).J
                for (P, M, hl), b, wl in zip(levels, fields, w))
        return J, None, None, None
    J = 0.0
    gb, gi = [], []
    for (P, M, hl), b, wl in zip(levels, fields, w):
        obj, g, _ = objective_gradient(P, M, b, pe, hl, alpha, beta)
        gp, gm = image_gradient(P, M, b, pe, hl)
        J += wl * obj.J
        gb.append(wl * g)
        gi.append((wl * gp, wl * gm))
    accp, accm = gi[-1]
    for l in range(L - 2, -1, -1):
        fine = levels[l][0].shape
        accp = gi[l][0] + restrict_image_T(accp, fine)
        accm = gi[l][1] + restrict_image_T(accm, fine)
    return J, gb, accp, accm


def solve(Ip, Im, pe, h=(1.0, 1.0, 1.0), *, alpha=ALPHA, beta=BETA, levels=1, gn_iters=5,
          pcg_iters=10, pcg_rtol=0.0, armijo_c=1e-4, ls_max_trials=10, ot_eps=1e-3,
          ot_guard=True, ot_blur=False, b_init=None, solver="gn",
          lbfgs_memory=10, admm_rho0=None) -> SolveResult:
    """The whole path: pyramid, OT on the coarsest level (or ``b_init`` there), GN-PCG on every
    level coarse to fine with prolongation in between, then the Jacobian-modulation correction
    (Sec. 2.4.7).  Failures are reported in ``status`` (R27).  ``solver`` = "lbfgs" runs
    ``gn_iters`` L-BFGS steps per level instead (Sec. 2.3.3; ``oracle.lbfgs``), "admm"
    ``gn_iters`` ADMM iterations (Sec. 2.3.2; ``oracle.admm``; PCG settings per column)."""
    if solver not in ("gn", "lbfgs", "admm"):
        raise ValueError(solver)
    finite = bool(np.all(np.isfinite(Ip)) and np.all(np.isfinite(Im)))
    status = STATUS_OK if finite else STATUS_NONFINITE
    pyr = pyramid(Ip, Im, h, levels)
    Pc, Mc, hcst = pyr[-1]
    b_ot = None
    guarded = 0
    if b_init is not None:
        b = np.asarray(b_init, dtype=np.float64)
    elif not finite:
        b = np.zeros(Pc.shape[:pe] + (Pc.shape[pe] + 1,) + Pc.shape[pe + 1:])
        b_ot = b.copy()
    else:
        ot = ot_init(Pc, Mc, pe, hcst, eps=ot_eps, guard=ot_guard)
        b = gaussian_blur3(ot.b0) if ot_blur else ot.b0
        b_ot = b.copy()
        guarded = ot.guarded_cells
    lev = []
    for li in range(levels - 1, -1, -1):
        P, M, hh = pyr[li]
        if li < levels - 1:
            b = prolong_field(b, P.shape, pe)
        if not finite:
            lev.append((P.shape, hh, []))
            continue
        if solver == "admm":
            from . import admm as _ad
            b, hist = _ad.admm_level(P, M, b, pe, hh, alpha=alpha, beta=beta, iters=gn_iters,
                                     pcg_iters=pcg_iters, pcg_rtol=pcg_rtol, rho0=admm_rho0,
                                     armijo_c=armijo_c, ls_max_trials=ls_max_trials)
        elif solver == "lbfgs":
            from . import lbfgs as _lb
            b, hist = _lb.lbfgs_level(P, M, b, pe, hh, alpha=alpha, beta=beta, iters=gn_iters,
                                      memory=lbfgs_memory, armijo_c=armijo_c,
                                      ls_max_trials=ls_max_trials)
        else:
            b, hist = gauss_newton(P, M, b, pe, hh, alpha=alpha, beta=beta, gn_iters=gn_iters,
                                   pcg_iters=pcg_iters, pcg_rtol=pcg_rtol, armijo_c=armijo_c,
                                   ls_max_trials=ls_max_trials)
        lev.append((P.shape, hh, hist))
        if status == STATUS_OK and hist:
            if math.isinf(hist[0].J):
                status = STATUS_BARRIER
            elif not hist[-1].accepted:
                status = STATUS_LINESEARCH
    P, M, hh = pyr[0]
    return SolveResult(b, transform(P, b, pe, hh, +1.0), transform(M, b, pe, hh, -1.0), b_ot,
                       guarded, lev, status)


# --------------------------------------------------------------------------------------------
# Metrics (Sec. 3.3)
# --------------------------------------------------------------------------------------------

def relative_improvement(Ip, Im, Tp, Tm) -> float:
    """100 (1 - |T+ - T-|^2 / |I+ - I-|^2): SSD of the corrected pair relative to the input."""
    num = float(np.sum((np.asarray(Tp) - np.asarray(Tm)) ** 2))
    den = float(np.sum((np.asarray(Ip, np.float64) - np.asarray(Im, np.float64)) ** 2))
    return 100.0 * (1.0 - num / den)


def field_errors(b, b_true, mask=None):
    """(relative 2-norm error, max-abs error, RMS error) of a field map, optionally masked."""
    d = np.asarray(b, np.float64) - np.asarray(b_true, np.float64)
    t = np.asarray(b_true, np.float64)
    if mask is not None:
        d = d[mask]
        t = t[mask]
    rel = float(np.linalg.norm(d) / max(np.linalg.norm(t), 1e-300))
    return rel, float(np.max(np.abs(d))) if d.size else 0.0, float(np.sqrt(np.mean(d * d)))
