"""ctypes view of include/floquet.h and the loader of libfloquet.so.

Only marshalling lives here: structures mirroring the C declarations, the
function prototypes, and status-to-exception translation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfloquet.so")

FQ_OK, FQ_ERR_ARG, FQ_ERR_NONFINITE, FQ_ERR_SPECTRUM, FQ_ERR_HIP, FQ_ERR_UNSUPPORTED, FQ_ERR_STATE = range(7)
STATUS_NAMES = {0: "FQ_OK", 1: "FQ_ERR_ARG", 2: "FQ_ERR_NONFINITE", 3: "FQ_ERR_SPECTRUM",
                4: "FQ_ERR_HIP", 5: "FQ_ERR_UNSUPPORTED", 6: "FQ_ERR_STATE"}
FQ_DENSE, FQ_TRIDIAG, FQ_DENSE_EIGEN = 0, 1, 2
FQ_C128, FQ_C64 = 0, 1
FQ_MAGNUS4, FQ_MAGNUS6, FQ_CF4 = 0, 1, 2
SCHEMES = {"magnus4": FQ_MAGNUS4, "magnus6": FQ_MAGNUS6, "cf4": FQ_CF4}
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
#: kernel kinds timed in profile mode (fq_report.ms_kernel indices)
K_FIRST, K_FIRST_LAST, K_MID, K_LAST, K_HEFF, K_TRIDIAG, K_SLOTS = 0, 1, 2, 3, 4, 5, 16
K_ADJ_FWD, K_ADJ_REV = 6, 7
#: split-BF16 builds time their products by term format (fq_term_format + K_TERM_FP64)
K_TERM_FP64, K_TERM_F64ACC, K_TERM_X3, K_TERM_X2, K_TERM_X1, K_CONVERT = 8, 9, 10, 11, 12, 13
K_CHAIN = 14
TERM_SLOTS = 16
#: fq_term_format values
TERM_FORMATS = {"fp64": 0, "bf16x3_f64acc": 1, "bf16x3": 2, "bf16x2": 3, "bf16x1": 4, "fp32": 5}
TERM_FORMAT_NAMES = {v: k for k, v in TERM_FORMATS.items()}

#: every entry point include/floquet.h declares
EXPORTS = (
    "fq_node_times", "fq_node_times_magnus6", "fq_bessel_weights", "fq_choose_order", "fq_tridiag_extremes",
    "fq_hermitian_cover", "fq_workspace_bytes", "fq_create", "fq_destroy", "fq_set_drive",
    "fq_get_report",
    "floquet_build_UT", "floquet_propagate", "floquet_period_average", "floquet_grad",
    "floquet_build_UT_static", "fq_last_error",
)


class FqSystem(ctypes.Structure):
    _fields_ = [("n", c_int64), ("layout", c_int32), ("n_drive", c_int32),
                ("h0", c_void_p), ("hmod", c_void_p),
                ("h0_diag", c_void_p), ("h0_off", c_void_p), ("hmod_diag", c_void_p),
                ("hmods", POINTER(c_void_p))]


class FqParams(ctypes.Structure):
    _fields_ = [("T", c_double), ("M", c_int32), ("L", c_int32),
                ("f_nodes", POINTER(c_double)),
                ("e_min", c_double), ("e_max", c_double), ("tol", c_double),
                ("precision", c_int32), ("checkpoint_every", c_int32),
                ("profile", c_int32), ("reorthonormalize", c_int32),
                ("dtype", c_int32), ("scheme", c_int32),
                ("mixed_tol", c_double), ("term_formats", POINTER(c_int32)),
                ("n_term_formats", c_int32), ("grad_pair_sums", c_int32)]


class FqReport(ctypes.Structure):
    _fields_ = [("L", c_int32), ("M", c_int32), ("R", c_double), ("dE", c_double),
                ("beta", c_double), ("e_min", c_double), ("e_max", c_double),
                ("unitarity_max", c_double), ("unitarity_fro", c_double),
                ("unitarity_max_after", c_double), ("unitarity_fro_after", c_double),
                ("ms_build", c_double), ("ms_kernel", c_double * K_SLOTS),
                ("n_kernel", c_int32 * K_SLOTS), ("term_format", c_int32 * TERM_SLOTS),
                ("mixed_err_est", c_double), ("diverged", c_int32)]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if name in ("ms_kernel", "n_kernel", "term_format") else v
        return out


class FloquetError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libfloquet.so (built in-tree). Raises if it is missing: there is no
    fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1508_07621_amd.build` "
                           "(or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    st = c_int32
    L.fq_node_times.argtypes = [c_double, c_int32, POINTER(c_double)]
    L.fq_node_times_magnus6.argtypes = [c_double, c_int32, POINTER(c_double)]
    L.fq_bessel_weights.argtypes = [c_double, c_int32, POINTER(c_double)]
    L.fq_choose_order.argtypes = [c_double, c_double, POINTER(c_int32)]
    L.fq_tridiag_extremes.argtypes = [c_int64, POINTER(c_double), POINTER(c_double),
                                      POINTER(c_double), POINTER(c_double)]
    L.fq_hermitian_cover.argtypes = [c_int64, c_void_p, POINTER(c_double), POINTER(c_double)]
    L.fq_workspace_bytes.argtypes = [POINTER(FqSystem), POINTER(FqParams), POINTER(c_size_t)]
    L.fq_create.argtypes = [POINTER(c_void_p), POINTER(FqSystem), POINTER(FqParams), c_void_p,
                            c_size_t, c_void_p]
    L.fq_destroy.argtypes = [c_void_p]
    L.fq_set_drive.argtypes = [c_void_p, POINTER(c_double)]
    L.fq_get_report.argtypes = [c_void_p, POINTER(FqReport)]
    L.floquet_build_UT.argtypes = [c_void_p, c_void_p, POINTER(FqReport)]
    L.floquet_propagate.argtypes = [c_void_p, c_void_p, c_int64, c_int32, c_int32, c_void_p,
                                    c_void_p, c_int32]
    L.floquet_period_average.argtypes = [c_void_p, c_void_p, c_int64, POINTER(c_double),
                                         POINTER(c_double)]
    L.floquet_grad.argtypes = [c_void_p, c_void_p, POINTER(c_double)]
    L.floquet_build_UT_static.argtypes = [POINTER(FqSystem), POINTER(FqParams), c_void_p, c_void_p,
                                          POINTER(FqReport)]
    for name in EXPORTS:
        if name != "fq_last_error":
            getattr(L, name).restype = st
    L.fq_last_error.argtypes = []
    L.fq_last_error.restype = c_char_p
    _lib = L
    return L


def check(status: int) -> None:
    if status != FQ_OK:
        msg = lib().fq_last_error().decode(errors="replace")
        raise FloquetError(status, msg)


def dptr(a) -> ctypes.POINTER(c_double):
    """Pointer to a C-contiguous float64 NumPy array."""
    return a.ctypes.data_as(POINTER(c_double))
