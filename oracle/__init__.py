"""Plain FP64 CPU oracle of reversed-gradient-polarity distortion correction.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` use it.
It shares no code with the HIP library (no kernels, headers, helpers or constant tables); the
only thing both sides share is the seeded input generator in ``synth/``.

``oracle.rgp`` is the vectorised NumPy implementation, ``oracle.loops`` a plain-loop version
for tiny grids that is used to pin the vectorised one.
"""
from . import rgp  # noqa: F401
