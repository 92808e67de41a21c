"""Mistakes planted in the FP64 oracle must fail its pins (CPU only).

Each case patches one plausible slip into ``oracle.rgp`` for the duration of the test (a dropped
term, a wrong sign, index or factor, a transposed role) and runs the pins of
``tests/test_oracle_pins.py`` that cover that part; at least one of them has to fail.  A case that
passes every pin would mean the pins could not tell that version of the oracle from the paper's
arithmetic.
"""
import math

import numpy as np
import pytest

from oracle import rgp
from tests import test_oracle_pins as pins

ORIG = {name: getattr(rgp, name) for name in (
    "transform_cols", "_positions", "interp_lin", "phi", "dphi", "d2phi", "smooth_sq",
    "laplacian", "laplacian_diag", "gn_matvec_cols", "gn_diag_cols", "pcg", "nodal_cdf",
    "cdf_inverse_index", "ot_shift", "restrict_image", "restrict_image_T",
    "_prolong_weights_cells", "_prolong_weights_nodes", "avg_T", "dif_T", "interp_lin_T",
    "gaussian_blur3")}


def _transform_unmodulated(I, b, hp, sign):
    T, val, slope, Db = ORIG["transform_cols"](I, b, hp, sign)
    return val, val, slope, Db


def _positions_flipped(m, Ab, hp, sign):
    return ORIG["_positions"](m, Ab, hp, -sign)


def _interp_left_sided(I, xi, hp):
    # the interval [ceil(xi) - 1, ceil(xi)]: differs from the right-sided rule only at knots
    m = I.shape[-1]
    k0 = (np.ceil(xi) - 1.0).astype(np.int64)
    w = xi - k0

    def sample(k):
        ok = (k >= 0) & (k < m)
        return np.where(ok, np.take_along_axis(I, np.clip(k, 0, m - 1), axis=-1), 0.0)

    v0, v1 = sample(k0), sample(k0 + 1)
    return (1.0 - w) * v0 + w * v1, (v1 - v0) / hp


def _phi_no_denominator(z):
    z = np.asarray(z, dtype=np.float64)
    inside = np.abs(z) < 1.0
    return np.where(inside, np.where(inside, z, 0.0) ** 4, np.inf)


def _dphi_numerator_only(z):
    z = np.asarray(z, dtype=np.float64)
    return 4.0 * z ** 3


def _laplacian_zero_padded(b, hc):
    out = np.zeros_like(b)
    for ax in range(3):
        p = np.pad(b, [(1, 1) if a == ax else (0, 0) for a in range(3)])
        n = b.shape[ax]
        lo = np.take(p, range(0, n), axis=ax)
        hi = np.take(p, range(2, n + 2), axis=ax)
        out += (2.0 * b - lo - hi) / (hc[ax] ** 2)
    return out


def _smooth_sq_two_axes(b, hc):
    return sum(float(np.sum(np.diff(b, axis=ax) ** 2)) / hc[ax] ** 2 for ax in (0, 1))


def _gn_matvec_no_smoothness(lin, v):
    return ORIG["gn_matvec_cols"](lin, v) - lin.alpha * lin.vol * ORIG["laplacian"](v, lin.hc)


def _gn_diag_no_smoothness(lin):
    d = ORIG["gn_diag_cols"](lin)
    return d - lin.alpha * lin.vol * ORIG["laplacian_diag"](d.shape, lin.hc)


def _pcg_unpreconditioned(apply_H, rhs, diag, maxit, rtol, **kw):
    return ORIG["pcg"](apply_H, rhs, np.ones_like(diag), maxit, rtol, **kw)


def _nodal_cdf_inclusive(i):
    S = np.concatenate([np.cumsum(i), [float(np.sum(i))]])   # C_k = sum_{j <= k}: one too many
    C = S / S[-1]
    C[-1] = 1.0
    return C


def _cdf_inverse_no_spline(C, r):
    # the min-rule index without the linear spline between nodes
    return np.floor(ORIG["cdf_inverse_index"](C, r))


def _ot_shift_ignores_negatives(Ip, Im, eps):
    hi = max(float(np.max(np.abs(Ip))), float(np.max(np.abs(Im))))
    return eps * hi


def _restrict_sum(I):
    return 8.0 * ORIG["restrict_image"](I)


def _restrict_T_unscaled(g, fine_shape):
    m = tuple(int(s) for s in fine_shape)
    up = np.asarray(g, dtype=np.float64)
    for ax in range(3):
        up = np.repeat(up, 2, axis=ax)
    return up[:m[0], :m[1], :m[2]]


def _prolong_cells_extrapolated(mf, mc):
    P = np.zeros((mf, mc))
    for j in range(mf):
        t = (j + 0.5) / 2.0 - 0.5
        i0 = min(max(int(math.floor(t)), 0), max(mc - 2, 0))
        if mc == 1:
            P[j, 0] = 1.0
            continue
        w = t - i0
        P[j, i0] += 1.0 - w
        P[j, i0 + 1] += w
    return P


def _prolong_nodes_at_cell_positions(mf, mc):
    # the node axis interpolated as if its samples sat at cell centres
    P = np.zeros((mf + 1, mc + 1))
    for k in range(mf + 1):
        t = min(max((k + 0.5) / 2.0 - 0.5, 0.0), float(mc))
        i0 = min(int(math.floor(t)), mc - 1)
        w = t - i0
        P[k, i0] += 1.0 - w
        P[k, i0 + 1] += w
    return P


def _avg_T_one_sided(u):
    out = np.zeros(u.shape[:-1] + (u.shape[-1] + 1,))
    out[..., :-1] += u
    return out


def _dif_T_sign(u, hp):
    return -ORIG["dif_T"](u, hp)


def _interp_T_floor_only(u, xi, m):
    k0 = np.floor(xi).astype(np.int64)
    G = np.zeros(u.shape[:-1] + (m,))
    lead = np.indices(u.shape[:-1])
    ok = (k0 >= 0) & (k0 < m)
    idx = tuple(np.broadcast_to(ax[..., None], u.shape)[ok] for ax in lead) + (k0[ok],)
    np.add.at(G, idx, u[ok])
    return G


def _blur_unnormalised(b, sigma=1.0):
    offs = (-1, 0, 1)
    out = np.zeros_like(np.asarray(b, dtype=np.float64))
    for i in offs:
        for j in offs:
            for k in offs:
                wt = math.exp(-(i * i + j * j + k * k) / (2.0 * sigma * sigma))
                out += wt * np.roll(b, shift=(-i, -j, -k), axis=(0, 1, 2))
    return out


def _blur_no_wrap(b, sigma=1.0):
    # zero padding instead of the periodic wrap-around
    b = np.asarray(b, dtype=np.float64)
    p = np.pad(b, 1)
    offs = (-1, 0, 1)
    w = {(i, j, k): math.exp(-(i * i + j * j + k * k) / (2.0 * sigma * sigma))
         for i in offs for j in offs for k in offs}
    tot = sum(w.values())
    out = np.zeros_like(b)
    n0, n1, n2 = b.shape
    for (i, j, k), wt in w.items():
        out += (wt / tot) * p[1 + i:1 + i + n0, 1 + j:1 + j + n1, 1 + k:1 + k + n2]
    return out


def _ot_half_instead_of_quarter(*a, **k):
    res = ORIG["ot_init"](*a, **k)
    res.b0 = 2.0 * res.b0
    return res


def _ot_roles_swapped(*a, **k):
    res = ORIG["ot_init"](*a, **k)
    res.b0 = -res.b0
    return res


def _ot_guard_off(*a, **k):
    k["guard"] = False
    return ORIG["ot_init"](*a, **k)


def _gn_accepts_every_finite_trial(*a, **k):
    k["armijo_c"] = -1e300
    return ORIG["gauss_newton_cols"](*a, **k)


def _two_loop_unit_h0(g, pairs):
    # H0 = I instead of (s^T y / y^T y) I of the newest pair
    q = g.copy()
    alphas = []
    for s_, y, rho in reversed(pairs):
        a = rho * float(np.sum(s_ * q))
        alphas.append(a)
        q = q - a * y
    r = q
    for (s_, y, rho), a in zip(pairs, reversed(alphas)):
        r = r + (a - rho * float(np.sum(y * r))) * s_
    return r


def _two_loop_pairs_in_wrong_order(g, pairs):
    return ORIG_LB["two_loop"](g, list(reversed(pairs)))


def _push_opposite_polarity(bcol, x, hp, sign, ov=None):
    return ORIG_LSQ["push"](bcol, x, hp, -sign)


def _z_update_without_wrap(v, rho, alpha, hc):
    # the cross-axis eigenvalues of the Neumann (DCT) problem instead of the periodic one
    na, nb = v.shape[0], v.shape[1]
    la = (2.0 - 2.0 * np.cos(np.pi * np.arange(na) / na)) / hc[0] ** 2
    lb = (2.0 - 2.0 * np.cos(np.pi * np.arange(nb) / nb)) / hc[1] ** 2
    lam = la[:, None, None] + lb[None, :, None]
    vh = np.fft.fft2(rho * v, axes=(0, 1))
    return np.real(np.fft.ifft2(vh / (alpha * lam + rho), axes=(0, 1)))


def _tri_matvec_lower_band_shifted(diag, off, v):
    out = diag * v
    out[..., :-1] += off[..., :-1] * v[..., 1:]
    out[..., 1:] += off[..., 1:] * v[..., :-1]
    return out


def _pyramid_spacing_kept(Ip, Im, h, levels):
    return [(P, M, tuple(float(x) for x in h)) for P, M, _ in ORIG["pyramid"](Ip, Im, h, levels)]


def _prolong_skipped(bc, fine_shape, pe):
    # the coarse field resampled by nearest coarse index only (no interpolation)
    out = np.asarray(bc, dtype=np.float64)
    for ax in range(3):
        n_f = int(fine_shape[ax]) + (1 if ax == pe else 0)
        idx = np.minimum(np.arange(n_f) // 2, out.shape[ax] - 1)
        out = np.take(out, idx, axis=ax)
    return out


from oracle import admm as _admm   # noqa: E402
from oracle import lbfgs as _lb    # noqa: E402
from oracle import lsq as _lsq     # noqa: E402

ORIG["ot_init"] = rgp.ot_init
ORIG["gauss_newton_cols"] = rgp.gauss_newton_cols
ORIG["pyramid"] = rgp.pyramid
ORIG_LB = {"two_loop": _lb.two_loop}
ORIG_LSQ = {"push": _lsq.push}

# name -> (patches, pins); a pin is a zero-argument callable.  Patches name attributes of
# oracle.rgp, or (module, attribute) for the other oracle modules.
MUTATIONS = {
    "transform without the Jacobian modulation (1 +- Db)": (
        {"transform_cols": _transform_unmodulated},
        [pins.test_mass_smooth_field_second_order, lambda: pins.test_loops_match_vectorised(7),
         pins.test_gradient_matches_central_differences]),
    "displacement sign of the sample positions flipped": (
        {"_positions": _positions_flipped},
        [lambda: pins.test_loops_match_vectorised(7), lambda: pins.test_mass_constant_shift(2.0),
         pins.test_gradient_matches_central_differences]),
    "left-sided image slope at knots": (
        {"interp_lin": _interp_left_sided},
        [pins.test_knot_rule_is_right_sided, pins.test_zero_field_is_identity]),
    "barrier phi without its denominator": (
        {"phi": _phi_no_denominator}, [pins.test_phi_closed_forms]),
    "phi' of the numerator only": (
        {"dphi": _dphi_numerator_only}, [pins.test_phi_closed_forms]),
    "zero-padded (Dirichlet) Laplacian": (
        {"laplacian": _laplacian_zero_padded},
        [pins.test_laplacian_closed_forms, pins.test_gradient_matches_central_differences]),
    "smoothness term over two axes only": (
        {"smooth_sq": _smooth_sq_two_axes},
        [pins.test_laplacian_closed_forms, pins.test_gradient_matches_central_differences]),
    "Gauss-Newton operator without alpha L": (
        {"gn_matvec_cols": _gn_matvec_no_smoothness},
        [pins.test_gn_operator_dense_4x5x6_with_pe_first,
         pins.test_pcg_equals_direct_solve_and_orthogonality]),
    "Jacobi diagonal without the Laplacian's": (
        {"gn_diag_cols": _gn_diag_no_smoothness},
        [pins.test_gn_operator_dense_4x5x6_with_pe_first]),
    "CG without the Jacobi preconditioner": (
        {"pcg": _pcg_unpreconditioned},
        [pins.test_pcg_equals_direct_solve_and_orthogonality]),
    "inclusive CDF (C_k = sum over j <= k)": (
        {"nodal_cdf": _nodal_cdf_inclusive},
        [pins.test_ot_identity_and_antisymmetry, lambda: pins.test_ot_known_integer_shift(2),
         pins.test_ot_inverse_matches_library_interp_and_min_rule]),
    "CDF inverse without the linear spline": (
        {"cdf_inverse_index": _cdf_inverse_no_spline},
        [pins.test_ot_gaussians_closed_form,
         pins.test_ot_inverse_matches_library_interp_and_min_rule]),
    "positivity shift ignoring negative intensities": (
        {"ot_shift": _ot_shift_ignores_negatives},
        [pins.test_ot_shift_with_negative_intensities,
         pins.test_ot_of_images_with_negative_values_is_that_of_the_shifted_images]),
    "restriction sums instead of averaging": (
        {"restrict_image": _restrict_sum}, [pins.test_restrict_invariants]),
    "restriction adjoint without the block counts": (
        {"restrict_image_T": _restrict_T_unscaled},
        [lambda: pins.test_restrict_adjoint_identity_and_dense_matrix((5, 7, 3))]),
    "prolongation extrapolating linearly at the outer half cells": (
        {"_prolong_weights_cells": _prolong_cells_extrapolated},
        [lambda: pins.test_prolong_outer_half_cells_are_constant(1)]),
    "prolongation of the node axis at cell positions": (
        {"_prolong_weights_nodes": _prolong_nodes_at_cell_positions},
        [lambda: pins.test_prolong_reproduces_linear_fields(1)]),
    "adjoint of the node average scattering to one node": (
        {"avg_T": _avg_T_one_sided}, [pins.test_residual_jacobian_fd_and_adjoint]),
    "adjoint of the node difference with the wrong sign": (
        {"dif_T": _dif_T_sign}, [pins.test_residual_jacobian_fd_and_adjoint]),
    "interpolation adjoint dropping the upper tap": (
        {"interp_lin_T": _interp_T_floor_only}, [pins.test_interpolation_adjoint_identity]),
    "OT blur weights not normalised": (
        {"gaussian_blur3": _blur_unnormalised},
        [pins.test_blur_keeps_constants_and_the_total_and_is_separable]),
    "OT blur without the periodic wrap-around": (
        {"gaussian_blur3": _blur_no_wrap},
        [pins.test_blur_of_a_corner_delta_gives_the_wrapped_gaussian_weights]),
    "OT field with 1/2 instead of 1/4": (
        {"ot_init": _ot_half_instead_of_quarter},
        [lambda: pins.test_ot_known_integer_shift(2), pins.test_ot_gaussians_closed_form]),
    "OT maps of the two images swapped (sign of b0)": (
        {"ot_init": _ot_roles_swapped},
        [lambda: pins.test_ot_known_integer_shift(2), pins.test_ot_gaussians_closed_form]),
    "OT guard left out": (
        {"ot_init": _ot_guard_off}, [pins.test_ot_guard_clips_and_reintegrates]),
    "Armijo test that accepts every finite trial": (
        {"gauss_newton_cols": _gn_accepts_every_finite_trial},
        [pins.test_armijo_rejects_a_finite_increase_and_takes_the_largest_halving,
         pins.test_gauss_newton_stops_with_b_unchanged_when_no_trial_is_accepted]),
    "coarse levels keep the fine spacing": (
        {"pyramid": _pyramid_spacing_kept},
        [pins.test_two_level_ot_of_a_shifted_bump_keeps_physical_units]),
    "prolongation by nearest coarse value": (
        {"prolong_field": _prolong_skipped},
        [lambda: pins.test_prolong_reproduces_linear_fields(1),
         pins.test_two_level_ot_of_a_shifted_bump_keeps_physical_units]),
    "L-BFGS with H0 = I": (
        {(_lb, "two_loop"): _two_loop_unit_h0},
        [pins.test_lbfgs_two_loop_equals_dense_bfgs_updates]),
    "L-BFGS pairs applied newest first": (
        {(_lb, "two_loop"): _two_loop_pairs_in_wrong_order},
        [pins.test_lbfgs_two_loop_equals_dense_bfgs_updates]),
    "least-squares push-forward with the other polarity": (
        {(_lsq, "push"): _push_opposite_polarity},
        [pins.test_lsq_push_forward_is_the_distortion_model,
         pins.test_lsq_recovers_the_true_image_from_a_noise_free_pair]),
    "ADMM z-update with Neumann instead of periodic eigenvalues": (
        {(_admm, "z_update"): _z_update_without_wrap},
        [pins.test_admm_z_update_equals_dense_solve_of_the_periodic_problem]),
    "ADMM block PCG with the lower band shifted by one": (
        {(_admm, "tri_matvec"): _tri_matvec_lower_band_shifted},
        [pins.test_admm_block_pcg_per_column_and_dense_solves]),
}


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_fails_a_pin(name, monkeypatch):
    patches, checks = MUTATIONS[name]
    for attr, fn in patches.items():
        mod, name_ = (rgp, attr) if isinstance(attr, str) else attr
        monkeypatch.setattr(mod, name_, fn)
    failed = []
    for check in checks:
        try:
            with np.errstate(all="ignore"):
                check()
        except (AssertionError, FloatingPointError, ValueError, IndexError):
            failed.append(getattr(check, "__name__", "pin"))
    assert failed, f"no pin fails with the planted mistake: {name}"
