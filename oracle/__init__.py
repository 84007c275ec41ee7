"""FP64 CPU oracle for the modal heat-current path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the package smoke check and
the benchmark's CPU-baseline leg, never by the library.  It shares no code
with the GPU path.
"""
from . import modal, fft_lattice, shc, directional, cross, virial  # noqa: F401
from .modal import *  # noqa: F401,F403
from .fft_lattice import binned_current_fft  # noqa: F401
from .shc import shc_correlation, shc_correlation_directional, shc_kappa, shc_spectrum, shc_weights  # noqa: F401
