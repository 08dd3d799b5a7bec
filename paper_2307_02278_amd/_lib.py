"""ctypes binding of the C ABI in include/mbd.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmbd.so")
HOSTCHECK_PATH = os.path.join(HERE, "libmbd_hostcheck.so")

MBD_OK = 0
MBD_E_ARG, MBD_E_CELL, MBD_E_GRID, MBD_E_NOT_POSDEF, MBD_E_NONFINITE = -1, -2, -3, -4, -5
MBD_E_NODEVICE, MBD_E_HIP, MBD_E_OOM, MBD_E_STATE, MBD_E_NOCONV = -6, -7, -8, -9, -10
PREC_FP64, PREC_MIXED = 0, 1
REORTH_NONE, REORTH_LOCAL, REORTH_FULL = 0, 1, 2
C_DIAG, C_DIR, C_REC, C_SELF, C_ALL = 1, 2, 4, 8, 15
STAGES = ["pair", "spread", "fft_x", "fft_y", "fft_z_conv", "ifft_y", "ifft_x", "gather",
          "lanczos", "setup", "force", "adjoint"]


class MbdSystem(C.Structure):
    _fields_ = [
        ("n_atoms", C.c_int32),
        ("pos", C.c_void_p),
        ("cell", C.c_double * 9),
        ("alpha", C.c_void_p),
        ("omega", C.c_void_p),
        ("r_vdw", C.c_void_p),
    ]


class MbdShape(C.Structure):
    _fields_ = [
        ("pair_wg_per_cu", C.c_int32),
        ("pair_subsets", C.c_int32),
        ("grid_chunk", C.c_int32),
        ("overlap", C.c_int32),
        ("gather_waves", C.c_int32),
        ("spread_mode", C.c_int32),
        ("pair_mode", C.c_int32),
    ]


TUNE_OFF, TUNE_MEASURE, TUNE_GIVEN = 0, 1, 2
SHAPE_SOURCES = ["builtin", "measured", "cached", "given"]


class MbdParams(C.Structure):
    _fields_ = [
        ("damp_beta", C.c_double),
        ("damp_d", C.c_double),
        ("ewald_tau", C.c_double),
        ("real_cutoff", C.c_double),
        ("damp_tol", C.c_double),
        ("grid", C.c_int32 * 3),
        ("spline_order", C.c_int32),
        ("n_probes", C.c_int32),
        ("n_steps", C.c_int32),
        ("block", C.c_int32),
        ("seed", C.c_uint64),
        ("precision", C.c_int32),
        ("reorth", C.c_int32),
        ("want_forces", C.c_int32),
        ("deterministic", C.c_int32),
        ("replica_cutoff", C.c_double),
        ("graph", C.c_int32),
        ("krylov_block", C.c_int32),
        ("tune", C.c_int32),
        ("shape", MbdShape),
        ("tune_cache", C.c_char_p),
        ("store_grids", C.c_int32),
    ]


class MbdInfo(C.Structure):
    _fields_ = [
        ("tau", C.c_double),
        ("r_pair", C.c_double),
        ("grid", C.c_int32 * 3),
        ("spline_order", C.c_int32),
        ("cells", C.c_int32 * 3),
        ("block", C.c_int32),
        ("workspace_bytes", C.c_size_t),
        ("n_pairs", C.c_int64),
        ("shape", MbdShape),
        ("shape_source", C.c_int32),
        ("tune_ms", C.c_double),
    ]


class MbdScsParams(C.Structure):
    _fields_ = [
        ("n_freq", C.c_int32),
        ("freq_scale", C.c_double),
        ("tol", C.c_double),
        ("max_iter", C.c_int32),
    ]


class MbdScsInfo(C.Structure):
    _fields_ = [
        ("iterations", C.c_int32),
        ("max_rel_residual", C.c_double),
    ]


# (name, restype, argtypes) for every entry point declared in include/mbd.h
SIGNATURES = [
    ("mbd_plan_create", C.c_int32,
     [C.POINTER(C.c_void_p), C.POINTER(MbdSystem), C.c_int32, C.POINTER(MbdParams), C.c_void_p]),
    ("mbd_plan_info", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(MbdInfo)]),
    ("mbd_set_positions", C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
    ("mbd_execute", C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("mbd_check", C.c_int32, [C.c_void_p]),
    ("mbd_matvec", C.c_int32,
     [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_uint32]),
    ("mbd_get_tridiagonal", C.c_int32,
     [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
      C.POINTER(C.c_int32)]),
    ("mbd_get_quadrature", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_double)]),
    ("mbd_plan_destroy", C.c_int32, [C.c_void_p]),
    ("mbd_grid_supported", C.c_int32, [C.c_int32]),
    ("mbd_set_timing", C.c_int32, [C.c_void_p, C.c_int32]),
    ("mbd_get_stage_times", C.c_int32,
     [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    ("mbd_scs", C.c_int32,
     [C.c_void_p, C.c_int32, C.POINTER(MbdScsParams), C.c_void_p, C.c_void_p, C.c_void_p,
      C.c_void_p, C.POINTER(MbdScsInfo)]),
    ("mbd_scs_noalloc", C.c_int32,
     [C.c_void_p, C.c_int32, C.POINTER(MbdScsParams), C.c_void_p, C.c_void_p, C.c_void_p,
      C.c_void_p, C.POINTER(MbdScsInfo)]),
    ("mbd_status_string", C.c_char_p, [C.c_int32]),
    ("mbd_last_error", C.c_char_p, []),
]

HOSTCHECK_SIGNATURES = [
    ("mbdh_splitmix", C.c_uint64, [C.c_uint64, C.c_uint64]),
    ("mbdh_bspline", C.c_int32, [C.c_int32, C.c_double, C.POINTER(C.c_double),
                                 C.POINTER(C.c_double)]),
    ("mbdh_direct_kernel", None, [C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double,
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("mbdh_tridiag_quadrature", C.c_int32,
     [C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double),
      C.POINTER(C.c_double)]),
    ("mbdh_bspline2", C.c_int32, [C.c_int32, C.c_double, C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("mbdh_direct_kernel_grad", None, [C.c_double, C.c_double, C.c_double, C.c_double,
                                       C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("mbdh_tridiag_adjoint", C.c_int32,
     [C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double),
      C.POINTER(C.c_double)]),
    ("mbdh_gauss_legendre", None, [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("mbdh_scs_kernel", None, [C.c_double, C.c_double, C.c_double, C.c_double,
                               C.POINTER(C.c_double), C.POINTER(C.c_double)]),
]

_lib = None
_hostcheck = None


class MbdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mbd error {code}: {msg}")
        self.code = code


def _bind(path, sigs):
    if not os.path.exists(path):
        raise ImportError(
            f"{os.path.basename(path)} is not built; run paper_2307_02278_amd.build.build()")
    lib = C.CDLL(path)
    for name, res, args in sigs:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


def lib():
    """The loaded libmbd.so (raises ImportError when it is not built)."""
    global _lib
    if _lib is None:
        _lib = _bind(LIB_PATH, SIGNATURES)
    return _lib


def hostcheck():
    global _hostcheck
    if _hostcheck is None:
        _hostcheck = _bind(HOSTCHECK_PATH, HOSTCHECK_SIGNATURES)
    return _hostcheck


def check(code: int):
    if code != MBD_OK:
        L = lib()
        raise MbdError(code, f"{L.mbd_status_string(code).decode()}: "
                             f"{L.mbd_last_error().decode()}")
