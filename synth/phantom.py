"""Seeded blob phantoms, smooth staggered field maps and push-forward distortion.

Recipe (all in float64, then cast by the caller):

* ``numpy.random.default_rng(seed)`` draws, in this order, the blob centres, blob widths and
  blob amplitudes.  Centres are uniform inside an ellipsoid whose semi-axes are 0.35 of the
  volume extent, centred in the volume, which leaves a near-empty background like a head
  inside its field of view.
* The field map b is a sum of signed Gaussian lobes evaluated on the staggered grid (cell
  centres across the phase-encoding axis, nodes along it), rescaled so ``max|b|`` equals the
  requested displacement.  Lobes are drawn from the substream ``default_rng([seed, 1, attempt])``
  and redrawn (next attempt) until ``max|d b / d v| <= 0.6``.
* The distorted pair is the mass-conserving push-forward of the phantom along the phase-encoding
  axis under x -> x + b(x) (``I_plus``) and x -> x - b(x) (``I_minus``): the mass of every true
  cell is spread uniformly over its deformed cell and integrated over the regular output cells
  (the push-forward simulation of Sec. 3.1).  Mass leaving the field of view is lost.
* Noise (substream ``default_rng([seed, 2])``) is added after the distortion: Gaussian, or Rician
  ``|I + n1 + i n2|``.
* ``scale`` multiplies the finished images (phantom and noise alike).

Spacing is h = (1, 1, 1) at the finest level, so b is measured in voxels.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "WORKLOADS",
    "SCHEDULES",
    "Pair",
    "make_pair",
    "make_workload",
    "make_batch",
    "make_batch_pair",
    "blob_phantom",
    "smooth_field",
    "push_forward",
    "restrict_shape",
]

# Workload definitions (shapes, phase-encoding axis, phantom and field statistics).
WORKLOADS = {
    # 32x32x24, PE along dim 1, FP64: the small parity case.
    "c1": dict(shape=(32, 32, 24), pe=1, n_blobs=20, blob_sigma=(2.0, 6.0), blob_amp=(0.2, 1.0),
               n_lobes=4, lobe_tau=(6.0, 10.0), bmax=3.0, noise="gauss", noise_sigma=0.01,
               seed=0),
    # 144x168x111, PE along dim 1 (AP), FP32: the 3T-brain-shaped headline workload.
    "c2": dict(shape=(144, 168, 111), pe=1, n_blobs=200, blob_sigma=(2.0, 8.0),
               blob_amp=(0.2, 1.0), n_lobes=5, lobe_tau=(12.0, 24.0), bmax=8.0,
               noise="rician", noise_sigma=0.02, seed=1),
    # 200x200x132, PE along dim 0 (LR), FP32: the 7T-brain-shaped workload with two frontal lobes.
    "c3": dict(shape=(200, 200, 132), pe=0, n_blobs=400, blob_sigma=(2.0, 8.0),
               blob_amp=(0.2, 1.0), lobes=((0.35, 0.8, 0.4), (0.65, 0.8, 0.4)), lobe_tau=(20.0, 20.0),
               bmax=12.0, noise="rician", noise_sigma=0.03, seed=2),
}

# Solver schedules that go with the workloads (levels, GN iterations per level, PCG steps).
SCHEDULES = {
    "c1": dict(levels=1, gn_iters=5, pcg_iters=10),
    "c2": dict(levels=3, gn_iters=10, pcg_iters=20),
    "c3": dict(levels=4, gn_iters=10, pcg_iters=20),
    "c5": dict(levels=3, gn_iters=10, pcg_iters=20),
}


@dataclasses.dataclass
class Pair:
    """One synthetic opposite-polarity pair (float64 arrays, caller layout [m0][m1][m2])."""

    I_plus: np.ndarray
    I_minus: np.ndarray
    I_true: np.ndarray
    b_true: np.ndarray  # staggered: m[pe] + 1 nodes along pe
    pe: int
    h: tuple
    seed: int
    scale: float = 1.0

    @property
    def shape(self):
        return self.I_plus.shape


def restrict_shape(shape: Sequence[int]) -> tuple:
    """Cell counts of the next coarser level: ceil(m / 2) on every axis."""
    return tuple((int(m) + 1) // 2 for m in shape)


def _ellipsoid_points(rng, n, shape, frac=0.35):
    """n points uniform in the centred ellipsoid with semi-axes frac * extent (cell units)."""
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = rng.uniform(size=(n, 1)) ** (1.0 / 3.0)
    ext = np.asarray(shape, dtype=np.float64)
    return ext / 2.0 + d * rad * frac * ext


def _axis_coords(n, h, nodes):
    """Physical coordinates of the samples along one axis: cell centres or nodes."""
    k = np.arange(n, dtype=np.float64)
    return k * h if nodes else (k + 0.5) * h


def _gauss_sum(shape, coords_nodes, h, centres, widths, amps, window=5.0):
    """Sum of isotropic Gaussians on a tensor grid, each truncated to +-window*width."""
    out = np.zeros(shape, dtype=np.float64)
    axes = [_axis_coords(shape[d], h[d], coords_nodes[d]) for d in range(3)]
    for c, s, a in zip(centres, widths, amps):
        sl = []
        fac = []
        for d in range(3):
            x = axes[d]
            lo = np.searchsorted(x, c[d] - window * s, side="left")
            hi = np.searchsorted(x, c[d] + window * s, side="right")
            sl.append(slice(lo, hi))
            fac.append(np.exp(-((x[lo:hi] - c[d]) ** 2) / (2.0 * s * s)))
        if any(f.size == 0 for f in fac):
            continue
        out[sl[0], sl[1], sl[2]] += a * (fac[0][:, None, None] * fac[1][None, :, None]
                                         * fac[2][None, None, :])
    return out


def blob_phantom(shape, h, centres, sigmas, amps):
    """Phantom I = sum_i a_i exp(-|x - mu_i|^2 / (2 sigma_i^2)) at cell centres."""
    return _gauss_sum(tuple(shape), (False, False, False), h, centres, sigmas, amps)


def smooth_field(shape, pe, h, centres, taus, amps):
    """Field map on the staggered grid: nodes along ``pe`` (m+1 of them), centres elsewhere."""
    nshape = list(shape)
    nshape[pe] += 1
    nodes = tuple(d == pe for d in range(3))
    return _gauss_sum(tuple(nshape), nodes, h, centres, taus, amps, window=6.0)


def _slope_along(b, pe, h):
    return np.diff(b, axis=pe) / h[pe]


def push_forward(I, b, pe, h, sign):
    """Mass-conserving push-forward of ``I`` along ``pe`` under x -> x + sign * b(x).

    Cell j of a column carries mass I_j h; its edges (nodes X_j, X_{j+1}) move to
    y_k = X_k + sign * b_k.  The mass is spread uniformly over [y_j, y_{j+1}] and integrated over
    the regular output cells.  ``1 + sign * d b / d v > 0`` is required (y strictly increasing).
    """
    hp = float(h[pe])
    Ic = np.moveaxis(np.asarray(I, dtype=np.float64), pe, -1)
    bc = np.moveaxis(np.asarray(b, dtype=np.float64), pe, -1)
    m = Ic.shape[-1]
    X = np.arange(m + 1, dtype=np.float64) * hp
    y = X + sign * bc  # [..., m+1]
    if np.any(np.diff(y, axis=-1) <= 0):
        raise ValueError("push_forward: deformation is not monotone (|db/dv| >= 1)")
    mass = np.concatenate([np.zeros(Ic.shape[:-1] + (1,)), np.cumsum(Ic * hp, axis=-1)], axis=-1)
    flat_y = y.reshape(-1, m + 1)
    flat_m = mass.reshape(-1, m + 1)
    out = np.empty((flat_y.shape[0], m), dtype=np.float64)
    for c in range(flat_y.shape[0]):
        M = np.interp(X, flat_y[c], flat_m[c], left=0.0, right=flat_m[c, -1])
        out[c] = np.diff(M) / hp
    out = out.reshape(Ic.shape)
    return np.moveaxis(out, -1, pe)


def make_pair(shape, pe, *, seed, n_blobs, blob_sigma, blob_amp, bmax, lobe_tau,
              n_lobes=None, lobes=None, noise="gauss", noise_sigma=0.0, scale=1.0,
              h=(1.0, 1.0, 1.0), max_slope=0.6, max_attempts=64) -> Pair:
    """Draw one seeded pair following the recipe in the module docstring."""
    shape = tuple(int(s) for s in shape)
    h = tuple(float(x) for x in h)
    rng = np.random.default_rng(seed)
    centres = _ellipsoid_points(rng, n_blobs, shape) * np.asarray(h)
    sigmas = rng.uniform(blob_sigma[0], blob_sigma[1], size=n_blobs)
    amps = rng.uniform(blob_amp[0], blob_amp[1], size=n_blobs)
    I_true = blob_phantom(shape, h, centres, sigmas, amps)

    b = None
    for attempt in range(max_attempts):
        frng = np.random.default_rng([seed, 1, attempt])
        if lobes is not None:
            lc = np.asarray(lobes, dtype=np.float64) * np.asarray(shape) * np.asarray(h)
            taus = frng.uniform(lobe_tau[0], lobe_tau[1], size=len(lc))
            sgn = np.ones(len(lc))
            mag = np.ones(len(lc))
        else:
            lc = _ellipsoid_points(frng, n_lobes, shape) * np.asarray(h)
            taus = frng.uniform(lobe_tau[0], lobe_tau[1], size=n_lobes)
            sgn = np.where(frng.uniform(size=n_lobes) < 0.5, -1.0, 1.0)
            mag = frng.uniform(0.5, 1.0, size=n_lobes)
        cand = smooth_field(shape, pe, h, lc, taus, sgn * mag)
        peak = np.max(np.abs(cand))
        if peak <= 0:
            continue
        cand *= bmax / peak
        if np.max(np.abs(_slope_along(cand, pe, h))) <= max_slope:
            b = cand
            break
    if b is None:
        raise RuntimeError("make_pair: no admissible field map within max_attempts")

    I_plus = push_forward(I_true, b, pe, h, +1.0)
    I_minus = push_forward(I_true, b, pe, h, -1.0)
    nrng = np.random.default_rng([seed, 2])
    if noise_sigma > 0:
        if noise == "gauss":
            I_plus = I_plus + nrng.normal(0.0, noise_sigma, size=shape)
            I_minus = I_minus + nrng.normal(0.0, noise_sigma, size=shape)
        elif noise == "rician":
            n1, n2 = nrng.normal(0.0, noise_sigma, size=(2,) + shape)
            I_plus = np.hypot(I_plus + n1, n2)
            n1, n2 = nrng.normal(0.0, noise_sigma, size=(2,) + shape)
            I_minus = np.hypot(I_minus + n1, n2)
        else:
            raise ValueError(f"unknown noise model {noise!r}")
    s = float(scale)
    return Pair(I_plus * s, I_minus * s, I_true * s, b, pe, h, seed, s)


def make_workload(name: str, *, seed: Optional[int] = None, scale: float = 1.0,
                  shape=None) -> Pair:
    """A pair from one of the named workloads (optionally overriding seed or shape)."""
    cfg = dict(WORKLOADS[name])
    if seed is not None:
        cfg["seed"] = seed
    if shape is not None:
        cfg["shape"] = tuple(shape)
    return make_pair(cfg.pop("shape"), cfg.pop("pe"), scale=scale, **cfg)


def batch_specs(n=32, first_seed=100):
    """Sizes, axes and displacements of the uneven batch (drawn from each pair's own seed)."""
    specs = []
    for i in range(n):
        seed = first_seed + i
        r = np.random.default_rng([seed, 7])
        d0, d1 = (int(x) for x in r.integers(96, 201, size=2))
        sl = int(r.integers(60, 133))
        pe = int(r.integers(0, 2))
        bmax = float(r.uniform(4.0, 12.0))
        specs.append(dict(shape=(d0, d1, sl), pe=pe, bmax=bmax, seed=seed))
    return specs


def _batch_pair(sp, scale, size_cap):
    shape = sp["shape"]
    if size_cap is not None:
        shape = tuple(min(int(s), int(size_cap)) for s in shape)
    return make_pair(shape, sp["pe"], seed=sp["seed"], n_blobs=200,
                     blob_sigma=(2.0, 8.0), blob_amp=(0.2, 1.0), bmax=sp["bmax"]
                     if size_cap is None else min(sp["bmax"], size_cap / 8.0),
                     n_lobes=5, lobe_tau=(12.0, 24.0) if size_cap is None else
                     (size_cap / 6.0, size_cap / 3.0), noise="rician",
                     noise_sigma=0.02, scale=scale)


def make_batch(n=32, first_seed=100, scale=1.0, size_cap=None):
    """The uneven batch: n pairs of different sizes and phase-encoding axes.

    ``size_cap`` (optional) shrinks every extent to at most that many cells, for quick tests.
    """
    return [_batch_pair(sp, scale, size_cap) for sp in batch_specs(n, first_seed)]


def make_batch_pair(index, n=32, first_seed=100, scale=1.0):
    """Pair ``index`` of ``make_batch(n, first_seed, scale)`` alone (the same arrays)."""
    return _batch_pair(batch_specs(n, first_seed)[index], scale, None)
