"""MI355X (gfx950) SPME stochastic-Lanczos MBD energy: HIP kernels behind a C ABI.

The compute path is libmbd.so (built by paper_2307_02278_amd.build). Importing
this package does not load it; the first call into the binding does, and it
raises ImportError when the library is not built. There is no CPU fallback.
"""
from ._lib import (  # noqa: F401
    C_ALL, C_DIAG, C_DIR, C_REC, C_SELF, MBD_E_ARG, MBD_E_CELL, MBD_E_GRID, MBD_E_HIP,
    MBD_E_NOCONV, MBD_E_NODEVICE, MBD_E_NONFINITE, MBD_E_NOT_POSDEF, MBD_E_OOM, MBD_E_STATE,
    MBD_OK, PREC_FP64, PREC_MIXED, REORTH_FULL, REORTH_LOCAL, REORTH_NONE, SHAPE_SOURCES,
    TUNE_GIVEN, TUNE_MEASURE, TUNE_OFF, MbdError, MbdShape,
)
from .api import DeviceSystem, MBDEnergy, Params, Plan, energy  # noqa: F401
