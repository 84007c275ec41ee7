"""modalhc: MI355X-native modal heat-current library (HNEMA / GKMA).

Thin Python binding over the C ABI of ``libmodalhc.so`` (include/mhc.h).
This module only marshals arguments: every step of the computation runs in
the library's HIP kernels.  PyTorch is used, when present, only to pass
device pointers and the current HIP stream.  There is no fallback: if the
library is missing, every entry point raises.
"""
from ._lib import (  # noqa: F401
    HNEMA, GKMA, DIRECTIONAL, CROSS, PREC_FP32, PREC_BF16X3, PREC_FP8, PREC_FP8X3, SCHED_AUTO, SCHED_TILES, SCHED_STREAMK,
    SCHED_SPLIT, MhcError, ModalGroup, ModalHC, ModalSHC, ModalVirial, SHCGroup, TersoffParams, bins_uniform, library, library_path, status_string,
)
from .physics import gkma_kappa, hnema_kappa, shc_kappa, tersoff_si  # noqa: F401
