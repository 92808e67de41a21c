"""MI355X-native reversed-gradient-polarity distortion correction (hot path of PyHySCO).

The compute path is ``librgp.so`` (hand-written HIP kernels for gfx950 behind a C ABI declared in
``include/rgp.h``); ``paper_2403_10706_amd.rgp`` is its ctypes binding.  Importing this package
does not load the library; the first call does, and fails loudly if it has not been built.
"""
from . import rgp  # noqa: F401
from .rgp import (  # noqa: F401
    Options,
    apply_correction,
    correct,
    gn_hvp,
    loss_grad,
    ot_init,
    pcg_solve,
)
