"""FP64 NumPy oracle of the least-squares correction (Sec. 2.4.7): the field map defines a
push-forward matrix per column that carries the true image to each distorted input, and the
corrected image is the least-squares solution of both push-forwards against both inputs.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never imports this.

Readings (used identically by the HIP path):

* R32 the push-forward along a column is the mass-conserving one of the distortion model (the
  paper's simulation, Sec. 3.1): true cell j (edges at the nodes x_j, x_{j+1}) moves to
  [y_j, y_{j+1}] with y_k = x_k +- b_k, its mass is spread evenly over that interval and
  integrated over the regular cells of the distorted image; mass moved outside the column is
  lost.  Entry (i, j) of M+- is |[y_j, y_{j+1}] cap [x_i, x_{i+1}]| / (y_{j+1} - y_j).  It needs
  |d b / d v| < 1 (then y is increasing and a moved cell spans at most three output cells).
* R33 the least-squares problem min_I |M+ I - I+|^2 + |M- I - I-|^2 is solved per column by
  CGLS (conjugate gradients on the normal equations in the Hestenes-Stiefel form, Bjorck's
  Algorithm 7.4.1) from I = 0, for at most ``maxit`` iterations, stopping a column when
  |M^T r| / |M^T [I+; I-]| < rtol or when its search direction vanishes; from I = 0 it tends to
  the minimum-norm solution.
"""
from __future__ import annotations

import numpy as np

from . import rgp as _r


def _overlaps(bcol: np.ndarray, hp: float, sign: float):
    """Rows i (output cells), weights w of the push-forward for the three candidate output
    cells t = 0, 1, 2 of every moved cell j: arrays [..., m, 3] (weight 0 when unused)."""
    m = bcol.shape[-1] - 1
    X = np.arange(m + 1, dtype=np.float64) * hp
    y = X + sign * bcol
    lo, hi = y[..., :-1], y[..., 1:]
    length = hi - lo
    i0 = np.floor(lo / hp).astype(np.int64)
    rows = np.stack([i0, i0 + 1, i0 + 2], axis=-1)
    a = np.maximum(lo[..., None], rows * hp)
    b = np.minimum(hi[..., None], (rows + 1) * hp)
    ov = np.maximum(b - a, 0.0)
    ok = (rows >= 0) & (rows < m)
    w = np.where(ok, ov / length[..., None], 0.0)
    return np.clip(rows, 0, m - 1), w


def push(bcol, x, hp, sign, ov=None):
    """M x (column form): the distorted image of x under the field bcol."""
    rows, w = ov if ov is not None else _overlaps(bcol, hp, sign)
    m = x.shape[-1]
    flat = x.reshape(-1, m)
    R = rows.reshape(-1, m, 3)
    W = w.reshape(-1, m, 3)
    out = np.zeros_like(flat)
    cols = np.arange(flat.shape[0])[:, None]
    for t in range(3):
        np.add.at(out, (np.broadcast_to(cols, R[..., t].shape), R[..., t]), W[..., t] * flat)
    return out.reshape(x.shape)


def push_T(bcol, u, hp, sign, ov=None):
    """M^T u (column form)."""
    rows, w = ov if ov is not None else _overlaps(bcol, hp, sign)
    return _gather_T(u, rows, w)


def _gather_T(u, rows, w):
    m = u.shape[-1]
    flat = u.reshape(-1, m)
    R = rows.reshape(-1, m, 3)
    W = w.reshape(-1, m, 3)
    cols = np.arange(flat.shape[0])[:, None, None]
    return np.sum(W * flat[cols, R], axis=-1).reshape(u.shape)


def lsq_cols(Ip, Im, bcol, hp, *, maxit=30, rtol=1e-6):
    """CGLS per column (R33).  Returns (I, iterations per column)."""
    ovp = _overlaps(bcol, hp, +1.0)
    ovm = _overlaps(bcol, hp, -1.0)
    Mx = lambda x: (push(bcol, x, hp, +1.0, ovp), push(bcol, x, hp, -1.0, ovm))
    MT = lambda rp, rm: _gather_T(rp, *ovp) + _gather_T(rm, *ovm)
    x = np.zeros_like(Ip)
    rp, rm = Ip.copy(), Im.copy()
    s = MT(rp, rm)
    p = s.copy()
    gam = np.sum(s * s, axis=-1)
    gam0 = gam.copy()
    active = gam > 0.0
    iters = np.zeros(gam.shape, dtype=np.int64)
    for _ in range(maxit):
        if not np.any(active):
            break
        qp, qm = Mx(p)
        delta = np.sum(qp * qp, axis=-1) + np.sum(qm * qm, axis=-1)
        active &= delta > 0.0
        a = np.where(active, gam / np.where(delta > 0.0, delta, 1.0), 0.0)[..., None]
        x = x + a * p
        rp = rp - a * qp
        rm = rm - a * qm
        iters += active
        s = MT(rp, rm)
        gnew = np.sum(s * s, axis=-1)
        done = np.sqrt(gnew) < rtol * np.sqrt(gam0)
        cont = active & ~done
        beta = np.where(cont, gnew / np.where(gam > 0.0, gam, 1.0), 0.0)[..., None]
        p = np.where(cont[..., None], s + beta * p, p)
        gam = np.where(cont, gnew, gam)
        active = cont
    return x, iters


def lsq_correct(Ip, Im, b, pe, h=(1.0, 1.0, 1.0), *, maxit=30, rtol=1e-6):
    """The least-squares corrected image in the caller's layout, and the CGLS iterations of
    every column (column form shape)."""
    hp = float(h[pe])
    x, it = lsq_cols(_r.to_cols(Ip, pe), _r.to_cols(Im, pe), _r.to_cols(b, pe), hp,
                     maxit=maxit, rtol=rtol)
    return _r.from_cols(x, pe), it
