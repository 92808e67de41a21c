"""Plain-loop, dense-matrix version of the objective, gradient and Gauss-Newton operator.

TEST INFRASTRUCTURE ONLY.  Written cell by cell from Eq. (1)-(6) with explicit index arithmetic
and dense matrices, for tiny grids (a few hundred unknowns), to pin the vectorised oracle
independently of its array code.  Arrays are in column form: images [na][nb][m], field
[na][nb][m+1]; ``hc = (h_a, h_b, h_pe)``.
"""
from __future__ import annotations

import math

import numpy as np


def _sample(col, k):
    m = len(col)
    return float(col[k]) if 0 <= k < m else 0.0


def _interp(col, xi, hp):
    k0 = math.floor(xi)
    w = xi - k0
    v0 = _sample(col, k0)
    v1 = _sample(col, k0 + 1)
    return (1.0 - w) * v0 + w * v1, (v1 - v0) / hp


def node_index(shape_b, ia, ib, k):
    return (ia * shape_b[1] + ib) * shape_b[2] + k


def objective(Ip, Im, b, hc, alpha, beta):
    """(J, D, S, P) by explicit loops."""
    na, nb, m = Ip.shape
    ha, hb, hp = hc
    vol = ha * hb * hp
    D = 0.0
    P = 0.0
    for ia in range(na):
        for ib in range(nb):
            for j in range(m):
                b0 = float(b[ia, ib, j])
                b1 = float(b[ia, ib, j + 1])
                ab = 0.5 * (b0 + b1)
                db = (b1 - b0) / hp
                vp, _ = _interp(Ip[ia, ib], j + ab / hp, hp)
                vm, _ = _interp(Im[ia, ib], j - ab / hp, hp)
                r = vp * (1.0 + db) - vm * (1.0 - db)
                D += 0.5 * vol * r * r
                if abs(db) >= 1.0:
                    P = math.inf
                elif P != math.inf:
                    P += 0.5 * vol * db ** 4 / (1.0 - db * db)
    S = 0.0
    sh = b.shape
    steps = (ha, hb, hp)
    for ia in range(sh[0]):
        for ib in range(sh[1]):
            for k in range(sh[2]):
                here = float(b[ia, ib, k])
                nbrs = ((ia + 1, ib, k, 0), (ia, ib + 1, k, 1), (ia, ib, k + 1, 2))
                for (xa, xb, xk, ax) in nbrs:
                    if xa < sh[0] and xb < sh[1] and xk < sh[2]:
                        d = float(b[xa, xb, xk]) - here
                        S += 0.5 * vol * d * d / steps[ax] ** 2
    return D + alpha * S + beta * P, D, S, P


def dense_operators(Ip, Im, b, hc):
    """Dense residual r (cells), Jacobian Jr (cells x nodes), D (cells x nodes), L (nodes x nodes).

    Jr is assembled from the chain rule of r_j = I+(xi+)(1+Db_j) - I-(xi-)(1-Db_j) with
    xi+- = j +- Ab_j / h: dr_j/db_j = c1/2 - c2/h and dr_j/db_{j+1} = c1/2 + c2/h.
    """
    na, nb, m = Ip.shape
    ha, hb, hp = hc
    shb = b.shape
    nn = b.size
    nc = Ip.size
    r = np.zeros(nc)
    Jr = np.zeros((nc, nn))
    Dm = np.zeros((nc, nn))
    dbs = np.zeros(nc)
    cell = 0
    for ia in range(na):
        for ib in range(nb):
            for j in range(m):
                b0 = float(b[ia, ib, j])
                b1 = float(b[ia, ib, j + 1])
                ab = 0.5 * (b0 + b1)
                db = (b1 - b0) / hp
                vp, sp = _interp(Ip[ia, ib], j + ab / hp, hp)
                vm, sm = _interp(Im[ia, ib], j - ab / hp, hp)
                r[cell] = vp * (1.0 + db) - vm * (1.0 - db)
                c1 = sp * (1.0 + db) + sm * (1.0 - db)
                c2 = vp + vm
                n0 = node_index(shb, ia, ib, j)
                n1 = node_index(shb, ia, ib, j + 1)
                Jr[cell, n0] += 0.5 * c1 - c2 / hp
                Jr[cell, n1] += 0.5 * c1 + c2 / hp
                Dm[cell, n0] = -1.0 / hp
                Dm[cell, n1] = 1.0 / hp
                dbs[cell] = db
                cell += 1
    L = np.zeros((nn, nn))
    steps = (ha, hb, hp)
    for ia in range(shb[0]):
        for ib in range(shb[1]):
            for k in range(shb[2]):
                i = node_index(shb, ia, ib, k)
                for (xa, xb, xk, ax) in ((ia + 1, ib, k, 0), (ia, ib + 1, k, 1),
                                         (ia, ib, k + 1, 2)):
                    if xa < shb[0] and xb < shb[1] and xk < shb[2]:
                        jn = node_index(shb, xa, xb, xk)
                        w = 1.0 / steps[ax] ** 2
                        L[i, i] += w
                        L[jn, jn] += w
                        L[i, jn] -= w
                        L[jn, i] -= w
    return r, Jr, Dm, L, dbs


def _dphi(z):
    return 2.0 * z ** 3 * (2.0 - z * z) / (1.0 - z * z) ** 2


def _d2phi(z):
    return 2.0 * z * z * (6.0 - 3.0 * z * z + z ** 4) / (1.0 - z * z) ** 3


def gradient(Ip, Im, b, hc, alpha, beta):
    """grad J = vol Jr^T r + alpha vol L b + beta (vol/2) D^T phi'(Db), from dense matrices."""
    vol = hc[0] * hc[1] * hc[2]
    r, Jr, Dm, L, dbs = dense_operators(Ip, Im, b, hc)
    g = vol * Jr.T @ r + alpha * vol * L @ b.reshape(-1)
    g += 0.5 * beta * vol * Dm.T @ np.array([_dphi(z) for z in dbs])
    return g.reshape(b.shape)


def gn_hessian(Ip, Im, b, hc, alpha, beta):
    """Dense H_J = vol Jr^T Jr + alpha vol L + beta (vol/2) D^T diag(phi'') D."""
    vol = hc[0] * hc[1] * hc[2]
    r, Jr, Dm, L, dbs = dense_operators(Ip, Im, b, hc)
    H = vol * Jr.T @ Jr + alpha * vol * L
    H += 0.5 * beta * vol * Dm.T @ np.diag([_d2phi(z) for z in dbs]) @ Dm
    return H
