"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check is a closed form, an invariant, a
special case that reduces to a textbook or library routine, finite differences, or a plain-loop /
dense-matrix brute force written separately (``oracle.loops``).
"""
import math

import numpy as np
import pytest

from oracle import loops
from oracle import rgp

ALPHA, BETA = 300.0, 1e-4


def _tiny(seed=0, shape=(3, 4, 5), hc=(1.1, 0.9, 1.3), base=0.3, amp=0.05):
    """Tiny column-form problem whose sample positions stay away from knots."""
    rng = np.random.default_rng(seed)
    na, nb, m = shape
    Ip = rng.uniform(0.2, 1.0, shape)
    Im = rng.uniform(0.2, 1.0, shape)
    b = base * hc[2] + amp * rng.standard_normal((na, nb, m + 1))
    return Ip, Im, b, hc


def _knot_distance(b, hc):
    Ab = rgp.avg(b)
    m = Ab.shape[-1]
    j = np.arange(m)
    xi = np.concatenate([j + Ab / hc[2], j - Ab / hc[2]])
    return float(np.min(np.abs(xi - np.round(xi))))


# ------------------------------------------------------------------------------------------
# Zero field is the identity (Eq. 1 with b = 0)
# ------------------------------------------------------------------------------------------

def test_zero_field_is_identity():
    rng = np.random.default_rng(1)
    Ip = rng.uniform(-0.1, 1.0, (5, 6, 7))
    Im = rng.uniform(-0.1, 1.0, (5, 6, 7))
    for pe in range(3):
        nshape = list(Ip.shape)
        nshape[pe] += 1
        b = np.zeros(nshape)
        h = (1.0, 1.5, 0.75)
        Tp = rgp.transform(Ip, b, pe, h, +1.0)
        Tm = rgp.transform(Im, b, pe, h, -1.0)
        assert np.array_equal(Tp, Ip) and np.array_equal(Tm, Im)
        o = rgp.objective(Ip, Im, b, pe, h)
        vol = h[0] * h[1] * h[2]
        assert o.S == 0.0 and o.P == 0.0
        assert o.D == pytest.approx(0.5 * vol * np.sum((Ip - Im) ** 2), rel=1e-14)
        res = rgp.solve(Ip, Im, pe, h, levels=1, gn_iters=0, b_init=b)
        assert np.array_equal(res.T_plus, Ip) and np.array_equal(res.T_minus, Im)


# ------------------------------------------------------------------------------------------
# Mass conservation of the modulated transform (Eq. 1)
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("c", [2.0, -3.0, 1.37, -0.61])
def test_mass_constant_shift(c):
    rng = np.random.default_rng(2)
    m = 40
    I = np.zeros((3, 4, m))
    I[..., 8:30] = rng.uniform(0.1, 1.0, (3, 4, 22))  # support >= |c| + 1 cells from both ends
    b = np.full((3, 4, m + 1), c)
    T, _, _, _ = rgp.transform_cols(I, b, 1.0, +1.0)
    np.testing.assert_allclose(T.sum(axis=-1), I.sum(axis=-1), rtol=1e-14)
    T, _, _, _ = rgp.transform_cols(I, b, 1.0, -1.0)
    np.testing.assert_allclose(T.sum(axis=-1), I.sum(axis=-1), rtol=1e-14)


def test_mass_smooth_field_second_order():
    """h sum_j T_j -> int_0^L I(y) dy at O(h^2) for a smooth field vanishing at both ends.

    Change of variables y = x + b(x) makes the continuous corrected mass equal to the mass of
    I over [b(0), L + b(L)] = [0, L].  The linear-interpolation error oscillates with the
    sub-cell sample position, so the pin is an h^2 error bound over six refinements rather than a
    fixed ratio; dropping the (1 + D b) modulation gives an O(1) error and fails it.
    """
    L = 10.0

    def err(m, mu, sig, amp, modulate=True):
        h = L / m
        xc = (np.arange(m) + 0.5) * h
        xn = np.arange(m + 1) * h
        I = np.exp(-((xc - mu) ** 2) / (2 * sig * sig))[None, None, :]
        b = (amp * np.sin(np.pi * xn / L) + 0.3 * np.sin(2 * np.pi * xn / L))[None, None, :]
        T, val, _, _ = rgp.transform_cols(I, b, h, +1.0)
        if not modulate:
            T = val
        ex = sig * math.sqrt(math.pi / 2) * (math.erf((L - mu) / (sig * math.sqrt(2)))
                                             - math.erf(-mu / (sig * math.sqrt(2))))
        return abs(h * T.sum() - ex) / ex

    for mu, sig, amp in [(4.7, 0.9, 0.8), (5.0, 1.2, 0.8), (5.0, 0.8, 1.0)]:
        ms = [40, 80, 160, 320, 640, 1280]
        es = [err(m, mu, sig, amp) for m in ms]
        scaled = [e * m * m for m, e in zip(ms, es)]   # bounded iff the error is O(h^2)
        assert max(scaled[3:]) <= max(scaled[:3])
        assert es[-1] < 1e-5
        assert err(320, mu, sig, amp, modulate=False) > 1e-2


# ------------------------------------------------------------------------------------------
# Symmetry J(b; I+, I-) = J(-b; I-, I+)
# ------------------------------------------------------------------------------------------

def test_polarity_swap_symmetry_exact():
    Ip, Im, b, hc = _tiny(3, shape=(4, 5, 9), base=0.7, amp=0.2)
    o1, g1, _ = rgp.objective_gradient_cols(Ip, Im, b, hc)
    o2, g2, _ = rgp.objective_gradient_cols(Im, Ip, -b, hc)
    assert o1.J == o2.J and o1.D == o2.D and o1.S == o2.S and o1.P == o2.P
    assert np.array_equal(g2, -g1)


# ------------------------------------------------------------------------------------------
# Smoothness term (Eq. 5) and the Laplacian
# ------------------------------------------------------------------------------------------

def test_laplacian_closed_forms():
    rng = np.random.default_rng(4)
    hc = (1.2, 0.8, 1.7)
    shape = (3, 4, 6)
    b = rng.standard_normal(shape)
    # b^T L b equals the plain sum of squared neighbour differences
    sq = 0.0
    for ia in range(shape[0]):
        for ib in range(shape[1]):
            for k in range(shape[2]):
                if ia + 1 < shape[0]:
                    sq += (b[ia + 1, ib, k] - b[ia, ib, k]) ** 2 / hc[0] ** 2
                if ib + 1 < shape[1]:
                    sq += (b[ia, ib + 1, k] - b[ia, ib, k]) ** 2 / hc[1] ** 2
                if k + 1 < shape[2]:
                    sq += (b[ia, ib, k + 1] - b[ia, ib, k]) ** 2 / hc[2] ** 2
    assert float(np.sum(b * rgp.laplacian(b, hc))) == pytest.approx(sq, rel=1e-13)
    assert rgp.smooth_sq(b, hc) == pytest.approx(sq, rel=1e-13)
    # constants are in the kernel
    assert np.max(np.abs(rgp.laplacian(np.full(shape, 3.5), hc))) < 1e-13
    # dense matrix: symmetric, PSD, one-dimensional kernel, diagonal as stated
    n = b.size
    Lm = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        Lm[:, i] = rgp.laplacian(e.reshape(shape), hc).ravel()
    np.testing.assert_allclose(Lm, Lm.T, atol=1e-14)
    ev = np.linalg.eigvalsh(Lm)
    assert ev[0] > -1e-12 and abs(ev[0]) < 1e-12 and ev[1] > 1e-3
    np.testing.assert_allclose(np.diag(Lm), rgp.laplacian_diag(shape, hc).ravel(), rtol=1e-14)
    # directional derivative of S is exactly vol (L b) . v
    v = rng.standard_normal(shape)
    vol = hc[0] * hc[1] * hc[2]
    eps = 1e-3
    Sp = 0.5 * vol * rgp.smooth_sq(b + eps * v, hc)
    Sm = 0.5 * vol * rgp.smooth_sq(b - eps * v, hc)
    assert (Sp - Sm) / (2 * eps) == pytest.approx(vol * float(np.sum(rgp.laplacian(b, hc) * v)),
                                                  rel=1e-10)


# ------------------------------------------------------------------------------------------
# Barrier phi (Eq. 3)
# ------------------------------------------------------------------------------------------

def test_phi_closed_forms():
    z = np.linspace(-0.95, 0.95, 381)
    np.testing.assert_allclose(rgp.phi(z), 1.0 / (1.0 - z * z) - 1.0 - z * z, atol=1e-12,
                               rtol=1e-12)
    assert np.all(rgp.phi(z) >= 0.0)
    assert np.all(rgp.d2phi(z) >= 0.0)
    assert np.all(np.isinf(rgp.phi(np.array([-1.0, 1.0, 1.5, -7.0]))))
    zs = np.linspace(-0.1, 0.1, 41)
    series = sum((4 + 2 * n) * (3 + 2 * n) * zs ** (2 + 2 * n) for n in range(12))
    np.testing.assert_allclose(rgp.d2phi(zs), series, rtol=1e-14, atol=1e-300)
    e = 1e-6
    zz = np.linspace(-0.9, 0.9, 37)
    np.testing.assert_allclose((rgp.phi(zz + e) - rgp.phi(zz - e)) / (2 * e), rgp.dphi(zz),
                               rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose((rgp.dphi(zz + e) - rgp.dphi(zz - e)) / (2 * e), rgp.d2phi(zz),
                               rtol=1e-7, atol=1e-9)


# ------------------------------------------------------------------------------------------
# Gradient, residual Jacobian and GN operator
# ------------------------------------------------------------------------------------------

def test_gradient_matches_central_differences():
    Ip, Im, b, hc = _tiny(5, shape=(4, 5, 8))
    hfd = 1e-6
    assert _knot_distance(b, hc) > 10 * hfd * 2
    obj, g, _ = rgp.objective_gradient_cols(Ip, Im, b, hc, ALPHA, BETA)
    rng = np.random.default_rng(50)
    for _ in range(6):
        v = rng.standard_normal(b.shape)
        Jp = rgp.objective_cols(Ip, Im, b + hfd * v, hc, ALPHA, BETA).J
        Jm = rgp.objective_cols(Ip, Im, b - hfd * v, hc, ALPHA, BETA).J
        fd = (Jp - Jm) / (2 * hfd)
        assert fd == pytest.approx(float(np.sum(g * v)), rel=1e-7)


def test_residual_jacobian_fd_and_adjoint():
    Ip, Im, b, hc = _tiny(6, shape=(3, 4, 7))
    _, _, lin = rgp.objective_gradient_cols(Ip, Im, b, hc)
    hp = hc[2]

    def resid(bb):
        Tp, _, _, _ = rgp.transform_cols(Ip, bb, hp, +1.0)
        Tm, _, _, _ = rgp.transform_cols(Im, bb, hp, -1.0)
        return Tp - Tm

    rng = np.random.default_rng(60)
    v = rng.standard_normal(b.shape)
    e = 1e-6
    fd = (resid(b + e * v) - resid(b - e * v)) / (2 * e)
    Jv = lin.c1 * rgp.avg(v) + lin.c2 * rgp.dif(v, hp)
    np.testing.assert_allclose(fd, Jv, rtol=1e-6, atol=1e-7 * np.max(np.abs(Jv)))
    w = rng.standard_normal(lin.c1.shape)
    JTw = rgp.avg_T(lin.c1 * w) + rgp.dif_T(lin.c2 * w, hp)
    assert float(np.sum(Jv * w)) == pytest.approx(float(np.sum(v * JTw)), rel=1e-13)
    # adjoints of the two PE operators on their own
    u = rng.standard_normal(lin.c1.shape)
    assert float(np.sum(rgp.avg(v) * u)) == pytest.approx(float(np.sum(v * rgp.avg_T(u))), rel=1e-13)
    assert float(np.sum(rgp.dif(v, hp) * u)) == pytest.approx(
        float(np.sum(v * rgp.dif_T(u, hp))), rel=1e-13)


@pytest.mark.parametrize("seed", [7, 8])
def test_loops_match_vectorised(seed):
    Ip, Im, b, hc = _tiny(seed, shape=(3, 4, 5), base=0.9, amp=0.3)
    o = rgp.objective_cols(Ip, Im, b, hc, ALPHA, BETA)
    Jl, Dl, Sl, Pl = loops.objective(Ip, Im, b, hc, ALPHA, BETA)
    assert o.J == pytest.approx(Jl, rel=1e-14)
    assert o.D == pytest.approx(Dl, rel=1e-14)
    assert o.S == pytest.approx(Sl, rel=1e-14)
    assert o.P == pytest.approx(Pl, rel=1e-13)
    _, g, lin = rgp.objective_gradient_cols(Ip, Im, b, hc, ALPHA, BETA)
    gl = loops.gradient(Ip, Im, b, hc, ALPHA, BETA)
    assert np.linalg.norm(g - gl) <= 1e-14 * np.linalg.norm(gl)
    H = loops.gn_hessian(Ip, Im, b, hc, ALPHA, BETA)
    v = np.random.default_rng(seed + 100).standard_normal(b.shape)
    Hv = rgp.gn_matvec_cols(lin, v).ravel()
    assert np.linalg.norm(Hv - H @ v.ravel()) <= 1e-13 * np.linalg.norm(H @ v.ravel())
    d = rgp.gn_diag_cols(lin).ravel()
    np.testing.assert_allclose(d, np.diag(H), rtol=1e-13)



def test_knot_rule_is_right_sided():
    """Where a sample position is a whole number (every cell at b = 0, and at a field of whole
    voxels) the image slope is the right-sided one, (I_{j+1} - I_j) / h with I = 0 past the last
    cell (R1, R2): the linearisation's c1 = I+' + I-' at b = 0 written out, and the gradient and
    GN operator against the plain-loop brute force at both fields."""
    rng = np.random.default_rng(21)
    hc = (1.1, 0.9, 1.3)
    Ip = rng.uniform(0.2, 1.0, (3, 4, 6))
    Im = rng.uniform(0.2, 1.0, (3, 4, 6))

    def right_slope(I):
        nxt = np.concatenate([I[..., 1:], np.zeros(I.shape[:-1] + (1,))], axis=-1)
        return (nxt - I) / hc[2]

    for b in (np.zeros((3, 4, 7)), np.full((3, 4, 7), 2.0 * hc[2])):
        _, g, lin = rgp.objective_gradient_cols(Ip, Im, b, hc, ALPHA, BETA)
        if not np.any(b):
            np.testing.assert_allclose(lin.c1, right_slope(Ip) + right_slope(Im), rtol=1e-14,
                                       atol=1e-14)
        # (rounding-level bars: r = T+ - T- cancels, and the two sides sum in different orders)
        gl = loops.gradient(Ip, Im, b, hc, ALPHA, BETA)
        assert np.linalg.norm(g - gl) <= 1e-11 * np.linalg.norm(gl)
        H = loops.gn_hessian(Ip, Im, b, hc, ALPHA, BETA)
        v = rng.standard_normal(b.shape)
        ref = H @ v.ravel()
        assert np.linalg.norm(rgp.gn_matvec_cols(lin, v).ravel() - ref) <= 1e-11 * np.linalg.norm(ref)

def test_gn_operator_dense_4x5x6_with_pe_first():
    """Brute-force H_J on a 4x5x6 grid with the PE axis first in caller layout."""
    rng = np.random.default_rng(9)
    shape = (6, 4, 5)          # pe = 0: six cells along PE
    pe = 0
    h = (1.3, 0.9, 1.1)
    Ip = rng.uniform(0.1, 1.0, shape)
    Im = rng.uniform(0.1, 1.0, shape)
    b = 0.4 + 0.1 * rng.standard_normal((7, 4, 5))
    obj, g, lin = rgp.objective_gradient(Ip, Im, b, pe, h)
    hc = rgp.col_spacing(h, pe)
    Pc, Mc, bc = rgp.to_cols(Ip, pe), rgp.to_cols(Im, pe), rgp.to_cols(b, pe)
    H = loops.gn_hessian(Pc, Mc, bc, hc, ALPHA, BETA)
    v = rng.standard_normal(b.shape)
    Hv = rgp.to_cols(rgp.gn_matvec(lin, v, pe), pe).ravel()
    ref = H @ rgp.to_cols(v, pe).ravel()
    assert np.linalg.norm(Hv - ref) <= 1e-12 * np.linalg.norm(ref)
    np.testing.assert_allclose(rgp.to_cols(rgp.gn_diag(lin, pe), pe).ravel(), np.diag(H),
                               rtol=1e-12)
    gl = loops.gradient(Pc, Mc, bc, hc, ALPHA, BETA)
    assert np.linalg.norm(rgp.to_cols(g, pe) - gl) <= 1e-13 * np.linalg.norm(gl)
    # the GN operator is symmetric positive semi-definite
    np.testing.assert_allclose(H, H.T, atol=1e-9 * np.max(np.abs(H)))
    assert np.linalg.eigvalsh(H)[0] > -1e-9 * np.max(np.abs(H))


def test_barrier_violation_is_infinite_value():
    Ip, Im, b, hc = _tiny(10, shape=(2, 3, 6))
    b = b.copy()
    b[1, 2, 3] += 1.5 * hc[2]   # slope >= 1 somewhere
    o = rgp.objective_cols(Ip, Im, b, hc)
    assert math.isinf(o.J) and math.isinf(o.P) and math.isfinite(o.D)
    o2, g, lin = rgp.objective_gradient_cols(Ip, Im, b, hc)
    assert math.isinf(o2.J) and g is None and lin is None


# ------------------------------------------------------------------------------------------
# PCG (Sec. 2.3.1; textbook CG)
# ------------------------------------------------------------------------------------------

def test_pcg_equals_direct_solve_and_orthogonality():
    Ip, Im, b, hc = _tiny(11, shape=(3, 4, 6), base=0.6, amp=0.2)
    _, g, lin = rgp.objective_gradient_cols(Ip, Im, b, hc, ALPHA, BETA)
    H = loops.gn_hessian(Ip, Im, b, hc, ALPHA, BETA)
    d = rgp.gn_diag_cols(lin)
    rec = []
    res = rgp.pcg(lambda v: rgp.gn_matvec_cols(lin, v), -g, d, g.size, 1e-13, record=rec)
    x = np.linalg.solve(H, -g.ravel())
    assert np.linalg.norm(res.x.ravel() - x) <= 1e-8 * np.linalg.norm(x)
    # preconditioned residuals are mutually orthogonal: r_i^T D^{-1} r_j = 0
    k = min(len(rec), 8)
    for i in range(k):
        for j in range(i):
            a = float(np.sum(rec[i] * rec[j] / d))
            s = math.sqrt(float(np.sum(rec[i] ** 2 / d)) * float(np.sum(rec[j] ** 2 / d)))
            assert abs(a) <= 1e-8 * s


def test_pcg_stopping_rules():
    Ip, Im, b, hc = _tiny(12, shape=(3, 4, 6))
    _, g, lin = rgp.objective_gradient_cols(Ip, Im, b, hc)
    d = rgp.gn_diag_cols(lin)
    H = lambda v: rgp.gn_matvec_cols(lin, v)  # noqa: E731
    r = rgp.pcg(H, -g, d, 3, 0.0)
    assert r.iters == 3
    r = rgp.pcg(H, -g, d, 100, 0.5)
    assert r.relres < 0.5 and r.iters < 100
    r = rgp.pcg(H, np.zeros_like(g), d, 10, 0.0)
    assert r.iters == 0 and np.all(r.x == 0)


# ------------------------------------------------------------------------------------------
# Gauss-Newton with Armijo (Sec. 2.3.1)
# ------------------------------------------------------------------------------------------

def test_gauss_newton_armijo_and_monotone():
    import synth
    p = synth.make_workload("c1", scale=100.0)
    ot = rgp.ot_init(p.I_plus, p.I_minus, p.pe, p.h)
    b, hist = rgp.gauss_newton(p.I_plus, p.I_minus, ot.b0, p.pe, p.h, gn_iters=4, pcg_iters=10)
    Js = [st.J for st in hist] + [rgp.objective(p.I_plus, p.I_minus, b, p.pe, p.h).J]
    for k, st in enumerate(hist):
        assert st.accepted
        assert Js[k + 1] <= st.J + 1e-4 * st.gamma * st.gq + 1e-9 * abs(st.J)
        assert st.gq < 0
    assert all(Js[k + 1] < Js[k] for k in range(len(hist)))


# ------------------------------------------------------------------------------------------
# Optimal-transport initialisation (Sec. 2.2)
# ------------------------------------------------------------------------------------------

def test_ot_identity_and_antisymmetry():
    import synth
    p = synth.make_workload("c1")
    ot = rgp.ot_init(p.I_plus, p.I_plus, p.pe, p.h)
    assert np.all(ot.b0 == 0.0)
    a = rgp.ot_init(p.I_plus, p.I_minus, p.pe, p.h)
    s = rgp.ot_init(p.I_minus, p.I_plus, p.pe, p.h)
    assert np.array_equal(s.b0, -a.b0)
    assert a.guarded_cells == s.guarded_cells
    # b0 vanishes at both column ends (C_0 and C_m are fixed)
    b0 = np.moveaxis(a.b0, p.pe, -1)
    assert np.all(b0[..., 0] == 0.0)


@pytest.mark.parametrize("c", [1, 2, 3])
def test_ot_known_integer_shift(c):
    m = 64
    j = np.arange(m)
    f = np.where((j >= 20) & (j < 44), 1.0 + np.sin(0.3 * j) ** 2, 0.0)
    ip = np.roll(f, c)
    im = np.roll(f, -c)
    I_p = np.broadcast_to(ip, (2, 3, m)).copy()
    I_m = np.broadcast_to(im, (2, 3, m)).copy()
    ot = rgp.ot_init(I_p, I_m, 2, (1.0, 1.0, 1.0), eps=1e-12, guard=False)
    Cp = rgp.nodal_cdf(ip + ot.shift)
    Cm = rgp.nodal_cdf(im + ot.shift)
    sel = (Cp > 1e-6) & (Cp < 1 - 1e-6) & (Cm > 1e-6) & (Cm < 1 - 1e-6)
    assert np.count_nonzero(sel) > 10
    np.testing.assert_allclose(ot.b0[0, 0][sel], float(c), atol=1e-9)


def test_ot_gaussians_closed_form():
    """1D W2 between Gaussians: b0(X) = [(mu+ - mu-) + s+(X-mu-)/s- - s-(X-mu+)/s+] / 4."""
    Lx = 60.0
    mup, sp, mum, sm = 31.0, 3.0, 28.5, 4.0

    def err(m):
        h = Lx / m
        xc = (np.arange(m) + 0.5) * h
        X = np.arange(m + 1) * h
        ip = np.exp(-((xc - mup) ** 2) / (2 * sp * sp)) / sp
        im = np.exp(-((xc - mum) ** 2) / (2 * sm * sm)) / sm
        ot = rgp.ot_init(ip[None, None, :], im[None, None, :], 2, (1.0, 1.0, h), eps=0.0,
                         guard=False)
        ref = 0.25 * ((mup - mum) + sp * (X - mum) / sm - sm * (X - mup) / sp)
        bulk = np.abs(X - 0.5 * (mup + mum)) < 5.0
        return float(np.max(np.abs(ot.b0[0, 0][bulk] - ref[bulk])))

    e1, e2 = err(300), err(600)
    assert e1 < 5e-3
    assert 3.0 < e1 / e2 < 5.0


def test_ot_inverse_matches_library_interp_and_min_rule():
    rng = np.random.default_rng(13)
    i = rng.uniform(0.01, 1.0, 37)
    C = rgp.nodal_cdf(i)
    X = np.arange(C.size, dtype=np.float64)
    r = np.concatenate([rng.uniform(0, 1, 500), C, [0.0, 1.0]])
    np.testing.assert_allclose(rgp.cdf_inverse_index(C, r), np.interp(r, C, X), rtol=0,
                               atol=1e-13)
    # min-rule of the pseudo-inverse: smallest node x with C(x) >= r is ceil of the spline value
    rs = rng.uniform(1e-9, 1.0, 10000)
    brute = np.array([np.min(np.nonzero(C >= t)[0]) for t in rs])
    np.testing.assert_array_equal(np.ceil(rgp.cdf_inverse_index(C, rs) - 1e-12), brute)


def test_ot_guard_clips_and_reintegrates():
    m = 30
    ip = np.full(m, 1e-3)
    ip[10] = 50.0                      # a spike: the transport has steep slopes
    im = np.full(m, 1e-3)
    im[14] = 50.0
    I_p = ip[None, None, :]
    I_m = im[None, None, :]
    raw = rgp.ot_init(I_p, I_m, 2, (1.0, 1.0, 1.0), guard=False)
    gd = rgp.ot_init(I_p, I_m, 2, (1.0, 1.0, 1.0), guard=True)
    slope_raw = np.diff(raw.b0[0, 0])
    assert np.max(np.abs(slope_raw)) > 0.99
    slope = np.diff(gd.b0[0, 0])
    assert np.max(np.abs(slope)) <= 0.99 + 1e-15
    assert gd.guarded_cells == int(np.count_nonzero(np.abs(slope_raw) > 0.99))
    np.testing.assert_allclose(slope, np.clip(slope_raw, -0.99, 0.99), atol=1e-12)
    assert gd.b0[0, 0, 0] == 0.0


def test_ot_zero_column_gives_zero_field():
    rng = np.random.default_rng(14)
    Ip = rng.uniform(0.0, 1.0, (3, 8, 4))
    Im = rng.uniform(0.0, 1.0, (3, 8, 4))
    Ip[1, :, 2] = 0.0
    Im[1, :, 2] = 0.0
    ot = rgp.ot_init(Ip, Im, 1, (1.0, 1.0, 1.0))
    assert np.all(ot.b0[1, :, 2] == 0.0)
    z = rgp.ot_init(np.zeros((2, 5, 3)), np.zeros((2, 5, 3)), 1, (1.0, 1.0, 1.0))
    assert np.all(z.b0 == 0.0) and z.shift == 0.0


# ------------------------------------------------------------------------------------------
# Pyramid transfers
# ------------------------------------------------------------------------------------------

def test_restrict_invariants():
    rng = np.random.default_rng(15)
    I = rng.standard_normal((6, 8, 4))
    R = rgp.restrict_image(I)
    assert R.shape == (3, 4, 2)
    assert float(R.sum()) == pytest.approx(float(I.sum()) / 8.0, rel=1e-13)
    assert R[1, 2, 1] == pytest.approx(I[2:4, 4:6, 2:4].mean(), rel=1e-14)
    odd = rgp.restrict_image(np.full((5, 7, 3), 2.5))
    assert odd.shape == (3, 4, 2) and np.allclose(odd, 2.5, rtol=0, atol=1e-15)
    I2 = rng.standard_normal((5, 7, 3))
    R2 = rgp.restrict_image(I2)
    assert R2[2, 3, 1] == pytest.approx(I2[4, 6, 2], rel=1e-15)   # corner block of one cell


@pytest.mark.parametrize("shape", [(6, 8, 4), (5, 7, 3), (1, 3, 2), (3, 1, 5)])
def test_restrict_adjoint_identity_and_dense_matrix(shape):
    """R^T against the adjoint identity <R x, y> = <x, R^T y> and against the transpose of the
    dense matrix whose columns are the restrictions of the unit images."""
    rng = np.random.default_rng(16)
    mc = tuple((m + 1) // 2 for m in shape)
    x, y = rng.standard_normal(shape), rng.standard_normal(mc)
    Ry = rgp.restrict_image_T(y, shape)
    assert Ry.shape == shape
    assert float(np.sum(rgp.restrict_image(x) * y)) == pytest.approx(float(np.sum(x * Ry)),
                                                                      rel=1e-13)
    n = int(np.prod(shape))
    Rd = np.stack([rgp.restrict_image(e.reshape(shape)).ravel() for e in np.eye(n)], axis=1)
    np.testing.assert_allclose(Ry.ravel(), Rd.T @ y.ravel(), rtol=1e-14, atol=1e-15)


def _pyramid_case(seed, shape=(6, 8, 5), pe=1, levels=3):
    rng = np.random.default_rng(seed)
    Ip = 0.6 + 0.4 * rng.random(shape)
    Im = 0.6 + 0.4 * rng.random(shape)
    fields, s = [], tuple(shape)
    for l in range(levels):
        if l:
            s = tuple((m + 1) // 2 for m in s)
        ns = list(s)
        ns[pe] += 1
        fields.append(0.08 * rng.standard_normal(ns))
    return Ip, Im, fields


def test_pyramid_objective_gradients_against_central_differences():
    """The objective summed over three pyramid levels: the field gradients against central
    differences along random directions of all three fields, the image gradients (J is quadratic
    in the finest images, which every level's images depend on linearly) exactly."""
    pe, h, w = 1, (1.0, 1.2, 0.9), (1.0, 0.5, 2.0)
    Ip, Im, fields = _pyramid_case(17, pe=pe)
    J, gb, gp, gm = rgp.pyramid_objective(Ip, Im, fields, pe, h, weights=w)
    rng = np.random.default_rng(18)
    e = 1e-5
    for _ in range(3):
        d = [rng.standard_normal(b.shape) for b in fields]
        Ju = rgp.pyramid_objective(Ip, Im, [b + e * x for b, x in zip(fields, d)], pe, h,
                                   weights=w)[0]
        Jd = rgp.pyramid_objective(Ip, Im, [b - e * x for b, x in zip(fields, d)], pe, h,
                                   weights=w)[0]
        an = sum(float(np.sum(g * x)) for g, x in zip(gb, d))
        assert (Ju - Jd) / (2 * e) == pytest.approx(an, rel=1e-6)
    e = 0.5
    for _ in range(3):
        dp, dm = rng.standard_normal(Ip.shape), rng.standard_normal(Im.shape)
        Ju = rgp.pyramid_objective(Ip + e * dp, Im + e * dm, fields, pe, h, weights=w)[0]
        Jd = rgp.pyramid_objective(Ip - e * dp, Im - e * dm, fields, pe, h, weights=w)[0]
        assert (Ju - Jd) / (2 * e) == pytest.approx(float(np.sum(gp * dp + gm * dm)), rel=1e-10)


def test_pyramid_objective_one_level_and_level_sum():
    """One level is the plain objective and its gradients; more levels add the objectives of the
    restricted pairs at doubled spacings."""
    pe, h = 2, (0.9, 1.1, 1.0)
    Ip, Im, fields = _pyramid_case(19, shape=(5, 6, 7), pe=pe, levels=2)
    J1, gb1, gp1, gm1 = rgp.pyramid_objective(Ip, Im, fields[:1], pe, h)
    obj, g, _ = rgp.objective_gradient(Ip, Im, fields[0], pe, h)
    gp, gm = rgp.image_gradient(Ip, Im, fields[0], pe, h)
    assert J1 == obj.J
    np.testing.assert_array_equal(gb1[0], g)
    np.testing.assert_array_equal(gp1, gp)
    np.testing.assert_array_equal(gm1, gm)
    J2 = rgp.pyramid_objective(Ip, Im, fields, pe, h)[0]
    Jc = rgp.objective(rgp.restrict_image(Ip), rgp.restrict_image(Im), fields[1], pe,
                       tuple(2 * x for x in h)).J
    assert J2 == pytest.approx(obj.J + Jc, rel=1e-14)
    assert rgp.pyramid_objective(Ip, Im, fields, pe, h, grad=False)[0] == pytest.approx(J2,
                                                                                       rel=1e-14)


@pytest.mark.parametrize("pe", [0, 1, 2])
def test_prolong_reproduces_linear_fields(pe):
    mf = [10, 9, 7]
    mc = [(s + 1) // 2 for s in mf]
    hf = 1.0
    hcoarse = 2.0 * hf

    def coords(m, h, nodes):
        k = np.arange(m + (1 if nodes else 0), dtype=np.float64)
        return k * h if nodes else (k + 0.5) * h

    def field(m, h):
        ax = [coords(m[d], h, d == pe) for d in range(3)]
        X = np.meshgrid(*ax, indexing="ij")
        return 0.3 * X[0] - 0.2 * X[1] + 0.1 * X[2] + 1.0, ax

    bc, _ = field(mc, hcoarse)
    bf_true, axf = field(mf, hf)
    bf = rgp.prolong_field(bc, mf, pe)
    assert bf.shape == bf_true.shape
    # exact where no clamping happens: cross-axis fine centres inside the coarse centre range
    sel = []
    for d in range(3):
        if d == pe:
            sel.append(np.ones(axf[d].size, bool))
        else:
            lo, hi = 0.5 * hcoarse, (mc[d] - 0.5) * hcoarse
            sel.append((axf[d] >= lo) & (axf[d] <= hi))
    mask = sel[0][:, None, None] & sel[1][None, :, None] & sel[2][None, None, :]
    np.testing.assert_allclose(bf[mask], bf_true[mask], rtol=0, atol=1e-12)
    const = rgp.prolong_field(np.full(bc.shape, -1.25), mf, pe)
    assert np.allclose(const, -1.25, rtol=0, atol=1e-15)


@pytest.mark.parametrize("pe", [0, 1, 2])
def test_prolong_outer_half_cells_are_constant(pe):
    """Hand-computed prolongation (R16) of a separable coarse field f0(i) + f1(j) + f2(k) from
    coarse cells (2, 2) across and 1 cell (2 nodes) along PE to fine cells (4, 3) across and 2
    cells (3 nodes) along PE.  Fine cell centres in coarse index units: (j + 1/2)/2 - 1/2, i.e.
    -0.25, 0.25, 0.75, 1.25 for 4 fine cells; fine nodes: k/2.  The outer half cells (-0.25 and
    1.25) take the nearest coarse value (linear extrapolation would give -2.5 and 12.5 below)."""
    f0c, f0f = [0.0, 10.0], [0.0, 2.5, 7.5, 10.0]        # cross axis, 2 -> 4 cells
    f1c, f1f = [3.0, -1.0], [3.0, 2.0, 0.0]              # cross axis, 2 -> 3 cells
    f2c, f2f = [1.0, 5.0], [1.0, 3.0, 5.0]               # PE axis, 2 -> 3 nodes
    bc_cols = (np.asarray(f0c)[:, None, None] + np.asarray(f1c)[None, :, None]
               + np.asarray(f2c)[None, None, :])
    want_cols = (np.asarray(f0f)[:, None, None] + np.asarray(f1f)[None, :, None]
                 + np.asarray(f2f)[None, None, :])
    bc = np.moveaxis(bc_cols, -1, pe)
    fine_cells = [4, 3]
    fine_cells.insert(pe, 2)
    got = rgp.prolong_field(bc, fine_cells, pe)
    np.testing.assert_allclose(np.moveaxis(got, pe, -1), want_cols, rtol=0, atol=1e-13)


# ------------------------------------------------------------------------------------------
# Failure branches of the Gauss-Newton solve and the status of a solve (R14, R27)
# ------------------------------------------------------------------------------------------

def test_gauss_newton_stops_with_b_unchanged_when_no_trial_is_accepted():
    """The 32x32x24 pair with images x3000 and one Armijo trial: gamma = 1 fails at the first
    step, so the iteration stops there (no further steps), b is returned bitwise unchanged, and
    the record says accepted = False, gamma = 0, one trial.  The rejection is confirmed with the
    plain-loop objective at b + q."""
    import synth
    from oracle import loops
    p = synth.make_workload("c1", scale=3000.0)
    b0 = rgp.ot_init(p.I_plus, p.I_minus, p.pe, p.h).b0
    b, hist = rgp.gauss_newton(p.I_plus, p.I_minus, b0, p.pe, p.h, gn_iters=3, pcg_iters=10,
                               ls_max_trials=1)
    assert len(hist) == 1
    st = hist[0]
    assert not st.accepted and st.trials == 1 and st.gamma == 0.0
    assert np.array_equal(b, b0)
    hc = rgp.col_spacing(p.h, p.pe)
    Pc, Mc, bcol = (rgp.to_cols(x, p.pe) for x in (p.I_plus, p.I_minus, b0))
    obj, g, lin = rgp.objective_gradient_cols(Pc, Mc, bcol, hc)
    q = rgp.pcg(lambda v: rgp.gn_matvec_cols(lin, v), -g, rgp.gn_diag_cols(lin), 10, 0.0).x
    J_trial = loops.objective(Pc, Mc, bcol + q, hc, rgp.ALPHA, rgp.BETA)[0]
    assert J_trial > obj.J + 1e-4 * float(np.sum(g * q))



def test_armijo_rejects_a_finite_increase_and_takes_the_largest_halving():
    """One column (16 cells) with alpha = 0.1, beta = 1, where the full Gauss-Newton step raises J
    to a finite value: the line search must reject gamma = 1 and accept the largest
    gamma = 2^-k with J(b + gamma q) <= J(b) + c gamma g^T q (R14).  Every candidate is re-evaluated
    with the plain-loop objective."""
    rng = np.random.default_rng(0)
    m, hc, alpha, beta, c = 16, (1.0, 1.0, 1.0), 0.1, 1.0, 1e-4
    Ip = rng.uniform(0.0, 1.0, (1, 1, m))
    Im = np.roll(Ip, 1, axis=-1) + 0.3 * rng.uniform(0.0, 1.0, (1, 1, m))
    b = 0.05 * rng.standard_normal((1, 1, m + 1))
    b1, hist = rgp.gauss_newton_cols(Ip, Im, b, hc, alpha=alpha, beta=beta, gn_iters=1,
                                     pcg_iters=20, armijo_c=c)
    st = hist[0]
    assert st.accepted and st.trials >= 2 and st.gamma == 2.0 ** (1 - st.trials)
    q = (b1 - b) / st.gamma
    J0 = loops.objective(Ip, Im, b, hc, alpha, beta)[0]
    assert J0 == pytest.approx(st.J, rel=1e-13)
    for k in range(st.trials):
        g_k = 2.0 ** -k
        J_k = loops.objective(Ip, Im, b + g_k * q, hc, alpha, beta)[0]
        ok = J_k <= J0 + c * g_k * st.gq
        assert ok == (k == st.trials - 1), (k, J_k, J0)
        if k == 0:
            assert math.isfinite(J_k) and J_k > J0   # the rejected full step is a finite increase

def test_ot_shift_with_negative_intensities():
    """Hand-computed shifts (R7): s = max(0, -min) + eps * max|.| over both images, where the
    largest magnitude may be a negative value."""
    Ip = np.array([-2.0, 1.0, 3.0]).reshape(1, 1, 3)
    Im = np.array([0.5, -1.0, 4.0]).reshape(1, 1, 3)
    assert rgp.ot_shift(Ip, Im, 0.25) == 2.0 + 0.25 * 4.0
    Ip = np.array([-5.0, 1.0]).reshape(1, 1, 2)
    Im = np.array([2.0, 3.0]).reshape(1, 1, 2)
    assert rgp.ot_shift(Ip, Im, 0.2) == 5.0 + 0.2 * 5.0
    assert rgp.ot_shift(-Ip, -Im, 0.0) == 3.0
    assert rgp.ot_shift(np.abs(Ip), np.abs(Im), 0.0) == 0.0


def test_ot_of_images_with_negative_values_is_that_of_the_shifted_images():
    """OT with a negative minimum equals OT of the images already shifted by that same amount
    with no further shift (their minimum is then positive); with eps = 0 the OT field does not
    change when a constant is added to both images before the shift is taken."""
    import synth
    p = synth.make_workload("c1")
    rng = np.random.default_rng(5)
    Ip = p.I_plus - 0.3 + 0.05 * rng.standard_normal(p.shape)
    Im = p.I_minus - 0.3 + 0.05 * rng.standard_normal(p.shape)
    assert min(Ip.min(), Im.min()) < 0
    eps = 1e-3
    s = rgp.ot_shift(Ip, Im, eps)
    a = rgp.ot_init(Ip, Im, p.pe, p.h, eps=eps, guard=False)
    b = rgp.ot_init(Ip + s, Im + s, p.pe, p.h, eps=0.0, guard=False)
    assert a.shift == s and b.shift == 0.0
    np.testing.assert_allclose(a.b0, b.b0, rtol=0, atol=1e-12)
    a0 = rgp.ot_init(Ip, Im, p.pe, p.h, eps=0.0, guard=False)
    c0 = rgp.ot_init(Ip + 0.2, Im + 0.2, p.pe, p.h, eps=0.0, guard=False)
    np.testing.assert_allclose(c0.shift + 0.2, a0.shift, rtol=0, atol=1e-14)
    np.testing.assert_allclose(a0.b0, c0.b0, rtol=0, atol=1e-9)


def test_solve_status_nonfinite_image():
    """A NaN in one image: no Gauss-Newton step runs on any level, the initial field is zero in
    place of OT (or the caller's b_init), and the status is the non-finite code."""
    import synth
    p = synth.make_pair((12, 14, 10), 1, seed=3, n_blobs=8, blob_sigma=(2.0, 4.0),
                        blob_amp=(0.2, 1.0), bmax=1.5, lobe_tau=(3.0, 5.0), n_lobes=2,
                        noise="gauss", noise_sigma=0.01)
    Ip = p.I_plus.copy()
    Ip[3, 4, 5] = np.nan
    r = rgp.solve(Ip, p.I_minus, p.pe, levels=2, gn_iters=2, pcg_iters=4)
    assert r.status == rgp.STATUS_NONFINITE
    assert np.all(r.b == 0.0) and all(len(lv[2]) == 0 for lv in r.levels)
    b_init = 0.1 * np.ones((12, 15, 10))
    Im = p.I_minus.copy()
    Im[0, 0, 0] = np.inf
    r = rgp.solve(p.I_plus, Im, p.pe, levels=1, gn_iters=2, pcg_iters=4, b_init=b_init)
    assert r.status == rgp.STATUS_NONFINITE and np.array_equal(r.b, b_init)


def test_solve_status_barrier_and_line_search():
    """A caller field with a slope of 2 somewhere: J = +inf at the first step, the level stops
    with b unchanged and the status is the barrier code.  Images x30000 with one Armijo trial:
    the first step fails on both levels (the finer one still runs, from the prolonged field), the
    status is the line-search code and the result is the prolonged OT field."""
    import synth
    p = synth.make_workload("c1")
    b = 0.05 * np.ones((32, 33, 24))
    b[5, 10, 7] += 2.0
    r = rgp.solve(p.I_plus, p.I_minus, p.pe, levels=1, gn_iters=3, pcg_iters=4, b_init=b)
    assert r.status == rgp.STATUS_BARRIER
    assert np.array_equal(r.b, b) and len(r.levels[0][2]) == 1
    assert math.isinf(r.levels[0][2][0].J) and not r.levels[0][2][0].accepted
    p = synth.make_workload("c1", scale=30000.0)
    r = rgp.solve(p.I_plus, p.I_minus, p.pe, levels=2, gn_iters=3, pcg_iters=10,
                  ls_max_trials=1)
    assert r.status == rgp.STATUS_LINESEARCH
    assert [len(lv[2]) for lv in r.levels] == [1, 1]
    assert not r.levels[0][2][0].accepted and not r.levels[1][2][0].accepted
    np.testing.assert_array_equal(r.b, rgp.prolong_field(r.b_ot, p.shape, p.pe))


# ------------------------------------------------------------------------------------------
# End to end: a pair distorted with a known field gets that field back
# ------------------------------------------------------------------------------------------


def test_two_level_ot_of_a_shifted_bump_keeps_physical_units():
    """A bump shifted by +-2 fine cells along PE: restricted to the coarse level it is shifted by
    +-1 coarse cell, so OT there gives b = +1 coarse cell = +2 in physical units (the coarse
    spacing is 2h, R16, and b keeps physical units), and the prolonged field is +2 too."""
    m = 40
    x = np.arange(m, dtype=np.float64)

    def bump(c):
        return np.exp(-0.5 * ((x - c) / 2.5) ** 2) * (np.abs(x - c) < 9.0)

    Ip = np.broadcast_to(bump(20.0 + 2.0)[None, :, None], (4, m, 3)).copy()
    Im = np.broadcast_to(bump(20.0 - 2.0)[None, :, None], (4, m, 3)).copy()
    r = rgp.solve(Ip, Im, 1, (1.0, 1.0, 1.0), levels=2, gn_iters=0, ot_eps=1e-12,
                  ot_guard=False)
    assert r.b_ot.shape == (2, 21, 2)
    bulk = slice(7, 14)                       # coarse nodes well inside both bumps' mass
    np.testing.assert_allclose(r.b_ot[:, bulk, :], 2.0, rtol=0, atol=1e-9)
    assert r.b.shape == (4, 41, 3)
    np.testing.assert_allclose(r.b[:, 2 * bulk.start + 1:2 * bulk.stop - 1, :], 2.0, rtol=0,
                               atol=1e-9)

def test_known_field_recovery():
    import synth
    p = synth.make_workload("c1", scale=1000.0)
    res = rgp.solve(p.I_plus, p.I_minus, p.pe, p.h, levels=1, gn_iters=5, pcg_iters=10)
    Itc = np.moveaxis(p.I_true, p.pe, -1)
    thr = 0.1 * Itc.max()
    mk = np.zeros(Itc.shape[:-1] + (Itc.shape[-1] + 1,), bool)
    mk[..., :-1] |= Itc > thr
    mk[..., 1:] |= Itc > thr
    mask = np.moveaxis(mk, -1, p.pe)
    rel, mx, rms = rgp.field_errors(res.b, p.b_true, mask)
    assert rms <= 0.25
    ri = rgp.relative_improvement(p.I_plus, p.I_minus, res.T_plus, res.T_minus)
    assert ri > 90.0


# ------------------------------------------------------------------------------------------
# Gradient with respect to the images (the adjoint of the interpolation and modulation)
# ------------------------------------------------------------------------------------------

def test_interpolation_adjoint_identity():
    """<A(I), u> = <I, A^T(u)> for the linear interpolation at shifted positions, samples outside
    the column dropped on both sides."""
    rng = np.random.default_rng(70)
    na, nb, m = 3, 4, 9
    I = rng.standard_normal((na, nb, m))
    xi = np.arange(m) + rng.uniform(-2.5, 2.5, (na, nb, m))
    u = rng.standard_normal((na, nb, m))
    val, _ = rgp.interp_lin(I, xi, 1.0)
    G = rgp.interp_lin_T(u, xi, m)
    assert float(np.sum(val * u)) == pytest.approx(float(np.sum(I * G)), rel=1e-13)


def test_image_gradient_is_the_exact_derivative_of_D():
    """D is a quadratic form in each image (the sample positions depend on b only), so central
    differences of the plain-loop objective are exact up to rounding, for every entry."""
    Ip, Im, b, hc = _tiny(71, shape=(2, 3, 6), base=0.8, amp=0.2)
    gp, gm = rgp.image_gradient_cols(Ip, Im, b, hc)
    e = 1e-3
    for which, I, g in (("+", Ip, gp), ("-", Im, gm)):
        fd = np.zeros_like(I)
        for idx in np.ndindex(I.shape):
            Iu, Id = I.copy(), I.copy()
            Iu[idx] += e
            Id[idx] -= e
            args_u = (Iu, Im) if which == "+" else (Ip, Iu)
            args_d = (Id, Im) if which == "+" else (Ip, Id)
            Ju = loops.objective(*args_u, b, hc, ALPHA, BETA)[0]
            Jd = loops.objective(*args_d, b, hc, ALPHA, BETA)[0]
            fd[idx] = (Ju - Jd) / (2 * e)
        np.testing.assert_allclose(g, fd, rtol=1e-8, atol=1e-10 * np.max(np.abs(fd)))


def test_image_gradient_random_directions_and_polarity_swap():
    Ip, Im, b, hc = _tiny(72, shape=(4, 5, 11), base=1.7, amp=0.4)
    gp, gm = rgp.image_gradient_cols(Ip, Im, b, hc)
    rng = np.random.default_rng(73)
    for _ in range(4):
        dp, dm = rng.standard_normal(Ip.shape), rng.standard_normal(Im.shape)
        e = 0.5   # exact for a quadratic
        Ju = rgp.objective_cols(Ip + e * dp, Im + e * dm, b, hc).D   # only D holds the images
        Jd = rgp.objective_cols(Ip - e * dp, Im - e * dm, b, hc).D
        assert (Ju - Jd) / (2 * e) == pytest.approx(float(np.sum(gp * dp + gm * dm)), rel=1e-10)
    # swapping the acquisitions and negating b leaves J unchanged and swaps the gradients
    sp, sm = rgp.image_gradient_cols(Im, Ip, -b, hc)
    np.testing.assert_allclose(sp, gm, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(sm, gp, rtol=1e-13, atol=1e-15)


# ---- optional blur of the OT field (3x3x3 Gaussian, sigma 1, periodic) ---------------------------

def _blur_fft(b, sigma=1.0):
    """The same blur as a circular FFT convolution (how the paper applies it): the 27 weights are
    placed at their offsets modulo the extents (adding up where a short axis folds them)."""
    K = np.zeros(b.shape)
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            for k in (-1, 0, 1):
                K[i % b.shape[0], j % b.shape[1], k % b.shape[2]] += np.exp(
                    -(i * i + j * j + k * k) / (2 * sigma * sigma))
    K /= K.sum()
    return np.real(np.fft.ifftn(np.fft.fftn(b) * np.fft.fftn(K)))


@pytest.mark.parametrize("shape", [(5, 6, 7), (2, 9, 4), (1, 5, 3), (8, 3, 1)])
def test_blur_matches_fft_circular_convolution(shape):
    b = np.random.default_rng(41).standard_normal(shape)
    assert np.max(np.abs(rgp.gaussian_blur3(b) - _blur_fft(b))) < 1e-13


def test_blur_of_a_corner_delta_gives_the_wrapped_gaussian_weights():
    b = np.zeros((5, 6, 7))
    b[0, 0, 0] = 1.0
    out = rgp.gaussian_blur3(b)
    a = math.exp(-0.5)
    z = (1 + 2 * a) ** 3  # sum of the 27 weights exp(-|d|^2 / 2)
    assert out[0, 0, 0] == pytest.approx(1.0 / z, rel=1e-14)
    assert out[4, 0, 0] == pytest.approx(a / z, rel=1e-14)            # offset -1 wraps to m-1
    assert out[1, 5, 0] == pytest.approx(a * a / z, rel=1e-14)
    assert out[4, 5, 6] == pytest.approx(a ** 3 / z, rel=1e-14)
    assert out[2, 0, 0] == 0.0 and out[0, 3, 3] == 0.0                  # outside the 3x3x3 box
    assert out.sum() == pytest.approx(1.0, rel=1e-14)


def test_blur_keeps_constants_and_the_total_and_is_separable():
    b = np.random.default_rng(42).standard_normal((6, 5, 7))
    assert np.max(np.abs(rgp.gaussian_blur3(np.full((4, 5, 6), 2.5)) - 2.5)) < 1e-14
    assert rgp.gaussian_blur3(b).sum() == pytest.approx(b.sum(), abs=1e-12)
    a = math.exp(-0.5)
    sep = b
    for ax in range(3):  # three 1D passes with [a, 1, a] / (1 + 2a)
        sep = (a * np.roll(sep, 1, axis=ax) + sep + a * np.roll(sep, -1, axis=ax)) / (1 + 2 * a)
    assert np.max(np.abs(rgp.gaussian_blur3(b) - sep)) < 1e-14


# ---- L-BFGS (Sec. 2.3.3) ----------------------------------------------------------------------

def test_lbfgs_two_loop_equals_dense_bfgs_updates():
    """The two-loop recursion applies the inverse Hessian that the BFGS update formula builds
    from H0 = (s^T y / y^T y) I of the newest pair, one pair at a time (oldest first):
    H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T, written out densely."""
    from oracle import lbfgs as lb
    rng = np.random.default_rng(70)
    n, k = 12, 5
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    pairs = []
    for _ in range(k):
        s = rng.standard_normal(n)
        y = A @ s
        pairs.append((s, y, 1.0 / float(s @ y)))
    g = rng.standard_normal(n)
    s_new, y_new, _ = pairs[-1]
    H = (float(s_new @ y_new) / float(y_new @ y_new)) * np.eye(n)
    I = np.eye(n)
    for s, y, rho in pairs:
        H = (I - rho * np.outer(s, y)) @ H @ (I - rho * np.outer(y, s)) + rho * np.outer(s, s)
    np.testing.assert_allclose(lb.two_loop(g, pairs), H @ g, rtol=1e-11, atol=1e-12)
    # the secant condition of the newest pair holds for the dense H
    np.testing.assert_allclose(H @ y_new, s_new, rtol=1e-10)


def test_lbfgs_minimises_a_convex_quadratic():
    """On f(x) = x^T A x / 2 - c^T x (A SPD, condition ~1e2) the driver with Armijo steps reaches
    A^{-1} c: a wrong sign of y or s, a dropped pair or a wrong H0 stalls it."""
    from oracle import lbfgs as lb
    rng = np.random.default_rng(71)
    n = 30
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(np.linspace(1.0, 100.0, n)) @ Q.T
    c = rng.standard_normal(n)

    def fun(x, want_grad=True):
        J = 0.5 * float(x @ A @ x) - float(c @ x)
        return J, (A @ x - c if want_grad else None)

    x, hist = lb.lbfgs(fun, np.zeros(n), iters=120, memory=8)
    np.testing.assert_allclose(x, np.linalg.solve(A, c), rtol=0, atol=1e-7)
    # every step is accepted until |g|^2 reaches the rounding level of J (the line search then
    # cannot see a decrease and the run stops there)
    assert all(h.accepted for h in hist if h.gnorm > 1e-6)
    assert max(h.pcg_iters for h in hist) == 8        # pairs in use never exceed the memory


def test_lbfgs_first_step_and_armijo_invariants():
    """On the small workload scaled by 1000: the first direction is -g / max|g| (so g.d =
    -|g|^2 / max|g|), every accepted step satisfies the Armijo condition, J decreases, and the
    number of pairs grows by one per step up to the memory."""
    import synth
    from oracle import lbfgs as lb
    p = synth.make_workload("c1", scale=1000.0)
    b0 = np.zeros(rgp.to_cols(np.zeros(p.shape), p.pe).shape[:-1] + (p.shape[p.pe] + 1,))
    Ipc, Imc = rgp.to_cols(p.I_plus, p.pe), rgp.to_cols(p.I_minus, p.pe)
    hc = rgp.col_spacing((1.0, 1.0, 1.0), p.pe)
    _, g0, _ = rgp.objective_gradient_cols(Ipc, Imc, b0, hc)
    b, hist = lb.lbfgs_cols(Ipc, Imc, b0, hc, iters=12, memory=4)
    gm = float(np.max(np.abs(g0)))
    assert hist[0].gq == pytest.approx(-float(np.sum(g0 * g0)) / gm, rel=1e-12)
    assert hist[0].pcg_relres == pytest.approx(1.0 / gm, rel=1e-15)
    assert [h.pcg_iters for h in hist] == [0, 1, 2, 3, 4, 4, 4, 4, 4, 4, 4, 4]
    for a, nxt in zip(hist[:-1], hist[1:]):
        assert a.accepted
        assert nxt.J <= a.J + 1e-4 * a.gamma * a.gq
        assert nxt.J < a.J


# ---- least-squares correction (Sec. 2.4.7) ----------------------------------------------------

def test_lsq_push_forward_is_the_distortion_model():
    """The push-forward matrix applied to the true image reproduces the synthetic distortion of
    the input generator (an independent implementation through cumulative mass and np.interp),
    for both polarities, and its transpose is its adjoint."""
    import synth
    from synth.phantom import push_forward
    from oracle import lsq
    p = synth.make_workload("c1")
    bc, xc = rgp.to_cols(p.b_true, p.pe), rgp.to_cols(p.I_true, p.pe)
    for sign in (1.0, -1.0):
        ref = push_forward(p.I_true, p.b_true, p.pe, p.h, sign)
        got = rgp.from_cols(lsq.push(bc, xc, 1.0, sign), p.pe)
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)
        u = np.random.default_rng(72).standard_normal(xc.shape)
        lhs = float(np.sum(lsq.push(bc, xc, 1.0, sign) * u))
        rhs = float(np.sum(xc * lsq.push_T(bc, u, 1.0, sign)))
        assert lhs == pytest.approx(rhs, rel=1e-12)


def test_lsq_recovers_the_true_image_from_a_noise_free_pair():
    """Both acquisitions synthesised from a known image and field without noise: the
    least-squares correction with that field gives the image back."""
    import synth
    from synth.phantom import push_forward
    from oracle import lsq
    p = synth.make_workload("c1")
    Ip = push_forward(p.I_true, p.b_true, p.pe, p.h, 1.0)
    Im = push_forward(p.I_true, p.b_true, p.pe, p.h, -1.0)
    x, it = lsq.lsq_correct(Ip, Im, p.b_true, p.pe, maxit=200, rtol=1e-13)
    np.testing.assert_allclose(x, p.I_true, rtol=0, atol=1e-9 * np.abs(p.I_true).max())


def test_lsq_cgls_equals_dense_least_squares_and_zero_field():
    """On a tiny grid CGLS run to convergence equals np.linalg.lstsq on the dense stacked
    push-forward matrices of every column; with b = 0 both matrices are the identity and the
    solution is the mean of the two images after one iteration."""
    from oracle import lsq
    rng = np.random.default_rng(73)
    shape, pe = (3, 9, 4), 1
    b = 0.7 * rng.standard_normal((3, 10, 4))
    b *= 0.8 / np.max(np.abs(np.diff(b, axis=pe)))
    Ip, Im = rng.uniform(0, 1, shape), rng.uniform(0, 1, shape)
    x, _ = lsq.lsq_correct(Ip, Im, b, pe, maxit=60, rtol=1e-15)
    bc, xc = rgp.to_cols(b, pe), rgp.to_cols(x, pe)
    Pc, Mc = rgp.to_cols(Ip, pe), rgp.to_cols(Im, pe)
    m = shape[pe]
    E = np.eye(m)
    for a in range(bc.shape[0]):
        for c in range(bc.shape[1]):
            col = bc[a, c]
            Mp = np.stack([lsq.push(col[None], E[j][None], 1.0, 1.0)[0] for j in range(m)], 1)
            Mm = np.stack([lsq.push(col[None], E[j][None], 1.0, -1.0)[0] for j in range(m)], 1)
            A = np.vstack([Mp, Mm])
            ref = np.linalg.lstsq(A, np.concatenate([Pc[a, c], Mc[a, c]]), rcond=None)[0]
            np.testing.assert_allclose(xc[a, c], ref, rtol=0, atol=1e-10)
    x0, it0 = lsq.lsq_correct(Ip, Im, np.zeros_like(b), pe, maxit=5, rtol=1e-12)
    np.testing.assert_allclose(x0, 0.5 * (Ip + Im), rtol=0, atol=1e-14)
    assert int(it0.max()) == 1


# ---- ADMM (Sec. 2.3.2, Eq. 8-11) --------------------------------------------------------------

def _dense_pe_laplacian(bshape, hp):
    """Neumann second differences along the last (PE) axis, written out densely."""
    n = int(np.prod(bshape))
    L = np.zeros((n, n))
    idx = np.arange(n).reshape(bshape)
    m1 = bshape[-1]
    for k in range(m1 - 1):
        a, b = idx[..., k].ravel(), idx[..., k + 1].ravel()
        L[a, a] += 1.0 / hp ** 2
        L[b, b] += 1.0 / hp ** 2
        L[a, b] -= 1.0 / hp ** 2
        L[b, a] -= 1.0 / hp ** 2
    return L


def test_admm_b_update_gradient_and_bands_dense():
    """F_rho = D + alpha S3 + beta P + (rho vol / 2)|b - c|^2: its gradient and Gauss-Newton
    bands equal the plain-loop data and barrier parts (alpha = 0) plus a densely written PE
    Laplacian and the proximal identity; its value matches the plain-loop objective plus those
    terms; the bands are tridiagonal per column."""
    from oracle import admm
    Ip, Im, b, hc = _tiny(12, shape=(3, 4, 6), base=0.7, amp=0.25)
    rng = np.random.default_rng(74)
    c = b + 0.05 * rng.standard_normal(b.shape)
    rho = 37.0
    vol = hc[0] * hc[1] * hc[2]
    L3 = _dense_pe_laplacian(b.shape, hc[2])
    g, dg, of = admm.f_rho_gradient(Ip, Im, b, hc, c, rho, ALPHA, BETA)
    gref = loops.gradient(Ip, Im, b, hc, 0.0, BETA).ravel() + ALPHA * vol * L3 @ b.ravel() \
        + rho * vol * (b - c).ravel()
    assert np.linalg.norm(g.ravel() - gref) <= 1e-13 * np.linalg.norm(gref)
    H = loops.gn_hessian(Ip, Im, b, hc, 0.0, BETA) + ALPHA * vol * L3 + rho * vol * np.eye(b.size)
    v = rng.standard_normal(b.shape)
    np.testing.assert_allclose(admm.tri_matvec(dg, of, v).ravel(), H @ v.ravel(), rtol=1e-12,
                               atol=1e-12 * np.abs(H).max())
    np.testing.assert_allclose(dg.ravel(), np.diag(H), rtol=1e-13)
    J, D, Sp, P = admm.f_rho(Ip, Im, b, hc, c, rho, ALPHA, BETA)
    Jl, Dl, _, Pl = loops.objective(Ip, Im, b, hc, ALPHA, BETA)
    s3 = 0.5 * vol * float(b.ravel() @ L3 @ b.ravel())
    prox = 0.5 * rho * vol * float(np.sum((b - c) ** 2))
    assert J == pytest.approx(Dl + ALPHA * s3 + BETA * Pl + prox, rel=1e-13)
    assert ALPHA * Sp == pytest.approx(ALPHA * s3 + prox, rel=1e-13)


def test_admm_z_update_equals_dense_solve_of_the_periodic_problem():
    """The FFT z-update solves (alpha L12 + rho I) z = rho v, with L12 the Hessian of
    G / (alpha vol) recovered from G's values (G is quadratic: A_ij = G(e_i + e_j) - G(e_i) -
    G(e_j)); the periodic differences are those of the definition, extents 1, 2 and 5 included."""
    from oracle import admm
    rng = np.random.default_rng(75)
    hc = (1.3, 0.8, 1.1)
    vol = hc[0] * hc[1] * hc[2]
    for shape in ((5, 4, 3), (1, 3, 2), (2, 5, 2)):
        n = int(np.prod(shape))
        E = np.eye(n)
        Gd = np.array([admm.g_value(E[i].reshape(shape), hc, 1.0) for i in range(n)])
        A = np.zeros((n, n))
        for i in range(n):
            for j in range(n):
                A[i, j] = admm.g_value((E[i] + E[j]).reshape(shape), hc, 1.0) - Gd[i] - Gd[j]
        v = rng.standard_normal(shape)
        rho, alpha = 3.7, 2.0
        z = np.linalg.solve(alpha * A / vol + rho * np.eye(n), rho * v.ravel())
        np.testing.assert_allclose(admm.z_update(v, rho, alpha, hc).ravel(), z, rtol=1e-12,
                                   atol=1e-12)


def test_admm_block_pcg_per_column_and_dense_solves():
    """BlockPCG run to convergence equals the dense solve of every column's tridiagonal system;
    a column's result does not depend on the other columns (a change to one leaves the rest)."""
    from oracle import admm
    rng = np.random.default_rng(76)
    shape = (3, 4, 9)
    off = -0.4 - 0.2 * rng.uniform(size=shape)
    off[..., -1] = 0.0
    diag = 2.5 + rng.uniform(size=shape)
    rhs = rng.standard_normal(shape)
    x, its, rel = admm.block_pcg(diag, off, rhs, 50, 1e-14)
    for a in range(3):
        for c in range(4):
            T = np.diag(diag[a, c]) + np.diag(off[a, c, :-1], 1) + np.diag(off[a, c, :-1], -1)
            np.testing.assert_allclose(x[a, c], np.linalg.solve(T, rhs[a, c]), rtol=1e-11,
                                       atol=1e-12)
    rhs2 = rhs.copy()
    rhs2[1, 2] *= 3.0
    x2, _, _ = admm.block_pcg(diag, off, rhs2, 3, 0.0)
    x3, _, _ = admm.block_pcg(diag, off, rhs, 3, 0.0)
    mask = np.ones((3, 4), bool)
    mask[1, 2] = False
    np.testing.assert_array_equal(x2[mask], x3[mask])


def test_admm_reaches_a_stationary_point_of_the_split_objective():
    """Many ADMM iterations on the small workload (images x30) from b = 0 drive the gradient of
    D + alpha (S3 + periodic S1 + S2) + beta P - the objective the splitting minimises - to below
    1/200 of its initial norm; rho changes only by factors of 2."""
    import synth
    from oracle import admm
    p = synth.make_workload("c1", scale=30.0)
    Ipc, Imc = rgp.to_cols(p.I_plus, p.pe), rgp.to_cols(p.I_minus, p.pe)
    hc = rgp.col_spacing((1.0, 1.0, 1.0), p.pe)
    vol = hc[0] * hc[1] * hc[2]

    def grad(b):
        _, g, _ = rgp.objective_gradient_cols(Ipc, Imc, b, hc)
        return (g - ALPHA * vol * rgp.laplacian(b, hc) + ALPHA * vol * admm.pe_laplacian(b, hc[2])
                + ALPHA * vol * admm.cross_laplacian_periodic(b, hc))

    b0 = np.zeros(Ipc.shape[:-1] + (Ipc.shape[-1] + 1,))
    b, hist = admm.admm_cols(Ipc, Imc, b0, hc, iters=200, pcg_iters=10, pcg_rtol=0.1)
    assert all(h.accepted for h in hist)
    assert np.linalg.norm(grad(b)) <= 5e-3 * np.linalg.norm(grad(b0))
    rhos = np.array([h.rho for h in hist])
    ratio = rhos[1:] / rhos[:-1]
    assert np.all(np.isin(ratio, [0.5, 1.0, 2.0])) and np.any(ratio != 1.0)
