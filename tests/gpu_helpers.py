"""Shared helpers of the GPU parity tests (device transfer, tolerances, seeded fields)."""
import sys

import numpy as np
import torch

DEV = "cuda"

# Parity bars on the same seeded inputs (the oracle is fed the same rounded inputs):
J_RTOL = 1e-5        # objective, relative
VEC_RTOL = 1e-4      # gradient / Hessian-vector products / PCG solution, relative 2-norm
B0_ATOL = 1e-4       # OT-initialised field, voxels, max-abs
BFINAL_ATOL = 1e-2   # final field after the whole schedule, voxels, max-abs


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def to_dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device=DEV, dtype=dtype)


def to_host(t):
    return t.detach().to(torch.float64).cpu().numpy()


def rounded(x, dtype):
    """The values the device sees for an FP64 array stored as `dtype`, back in FP64."""
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).to(torch.float64).numpy()


def rel2(a, ref):
    a = np.asarray(a, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    return float(np.linalg.norm(a - ref) / max(np.linalg.norm(ref), 1e-300))


def smooth_field(shape, pe, seed, amp=2.0, max_slope=0.45):
    """A seeded smooth staggered field with |d b/d v| <= max_slope (voxel units)."""
    rng = np.random.default_rng(seed)
    nshape = list(shape)
    nshape[pe] += 1
    axes = [np.arange(n) / max(n - 1, 1) for n in nshape]
    X = np.meshgrid(*axes, indexing="ij")
    b = np.zeros(nshape)
    for _ in range(4):
        k = rng.uniform(0.5, 2.5, size=3)
        ph = rng.uniform(0, 2 * np.pi, size=3)
        b += rng.uniform(-1, 1) * np.sin(2 * np.pi * k[0] * X[0] + ph[0]) \
            * np.cos(2 * np.pi * k[1] * X[1] + ph[1]) * np.sin(np.pi * k[2] * X[2] + ph[2])
    b *= amp / max(np.max(np.abs(b)), 1e-12)
    sl = np.max(np.abs(np.diff(b, axis=pe)))
    if sl > max_slope:
        b *= max_slope / sl
    return b
