"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package holds no arithmetic of the correction method itself (no transform, objective,
Hessian, optimal-transport map or solver).  It only draws phantoms and field maps and simulates
the two opposite-polarity acquisitions with a mass-conserving push-forward, which is how the
paper builds its simulated data set (Sec. 3.1).
"""
from .phantom import (  # noqa: F401
    WORKLOADS,
    SCHEDULES,
    Pair,
    make_pair,
    make_workload,
    make_batch,
    make_batch_pair,
    blob_phantom,
    smooth_field,
    push_forward,
    restrict_shape,
)
