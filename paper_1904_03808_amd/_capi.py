"""ctypes declarations of the libqsmg C ABI (include/qsmg.h).

Argument marshalling only: every computation happens in the HIP library.
Importing this module loads the shared library and fails loudly if it has not
been built.
"""
from __future__ import annotations

import ctypes as C
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libqsmg.so")

QS_OK = 0
QS_ERR_ARG = -1
QS_ERR_SHAPE = -2
QS_ERR_HIP = -3
QS_ERR_NOT_CONVERGED = -4
QS_ERR_NONFINITE = -5
QS_ERR_WORKSPACE = -6
QS_FP64 = 0
QS_FP32_IR = 1
QS_HIST = 64
QS_NOALLOC_SCRATCH_BYTES = 96 * 1024 * 1024


class QSParams(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("h", C.c_double),
                ("lam", C.c_double), ("mu", C.c_double), ("min_coarse_nz", C.c_int),
                ("n_pre", C.c_int), ("n_post", C.c_int), ("precision", C.c_int),
                ("colour_order", C.c_int * 8)]


class QSSolveInfo(C.Structure):
    _fields_ = [("cycles", C.c_int), ("levels", C.c_int), ("rel_res", C.c_double),
                ("rel_res_hist", C.c_double * QS_HIST)]


class QSStzParams(C.Structure):
    _fields_ = [("s_y", C.c_double), ("tau0", C.c_double), ("beta", C.c_double),
                ("delta_over_T", C.c_double), ("c0", C.c_double), ("chi_inf", C.c_double),
                ("dt", C.c_double), ("l_diff", C.c_double), ("n_sub", C.c_int),
                ("advect", C.c_int), ("chi_wall", C.c_int)]


class QSError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s (%d) [%s]" % (where, lib().qs_status_string(status).decode(),
                                               status, lib().qs_last_error().decode()))


_P = C.c_void_p
_D = C.c_double
_I = C.c_int
# name -> argtypes (all return qs_status as int, except qs_status_string)
SIGNATURES = {
    "qs_workspace_bytes": [C.POINTER(QSParams), C.POINTER(C.c_size_t)],
    "qs_level_dims": [C.POINTER(QSParams), _I, C.POINTER(_I), C.POINTER(_I), C.POINTER(_I),
                      C.POINTER(_I)],
    "qs_setup": [C.POINTER(QSParams), _P, C.c_size_t, _P, C.POINTER(_P)],
    "qs_destroy": [_P],
    "qs_apply": [_P, _P, _P],
    "qs_mg_solve": [_P, _P, _P, _D, _I, C.POINTER(QSSolveInfo)],
    "qs_stz_step": [_P, C.POINTER(QSStzParams), _P, _P, _P, _P, _P],
    "qs_rhs": [_P, _P, _D, _P],
    "qs_stress_update": [_P, _P, _P, _D, _P],
    "qs_step_scratch_bytes": [_P, C.POINTER(C.c_size_t)],
    "qs_projection_step": [_P, C.POINTER(QSStzParams), _D, _P, _P, _P, _P, _D, _I,
                           C.POINTER(QSSolveInfo)],
    "qs_projection_step_noalloc": [_P, C.POINTER(QSStzParams), _D, _P, _P, _P, _D, _I,
                                   C.POINTER(QSSolveInfo)],
    "qs_projection_step_walls": [_P, C.POINTER(QSStzParams), _P, _P, _P, _P, _P, _P, _D, _I,
                                 C.POINTER(QSSolveInfo)],
    "qs_explicit_step": [_P, C.POINTER(QSStzParams), _D, _D, _D, _P, _P, _P, _P],
    "qs_stz_step_vjp": [_P, C.POINTER(QSStzParams), _P, _P, _P, _P, _P, _P, _P, _P, _P],
    "qs_rhs_vjp": [_P, _P, _D, _P],
    "qs_stress_update_vjp": [_P, _P, _D, _P],
    "qs_level_colour_pass": [_P, _I, _P, _P, _I],
    "qs_level_residual": [_P, _I, _P, _P, _P],
    "qs_level_restrict": [_P, _I, _P, _P],
    "qs_level_prolong_add": [_P, _I, _P, _P],
    "qs_coarse_solve": [_P, _P, _P],
    "qs_level_stencil": [_P, _I, _P],
    "qs_smooth": [_P, _I, _P, _P, _I],
}

_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime (same soname); loading it first makes
        # the library bind to that runtime, the one that owns the tensors.
        import torch  # noqa: F401
        if not os.path.exists(_LIB_PATH):
            raise ImportError("libqsmg.so is not built (run __graft_entry__.build() or "
                              "python paper_1904_03808_amd/build.py): %s" % _LIB_PATH)
        L = C.CDLL(_LIB_PATH)
        L.qs_status_string.restype = C.c_char_p
        L.qs_status_string.argtypes = [_I]
        L.qs_last_error.restype = C.c_char_p
        L.qs_last_error.argtypes = []
        for name, args in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _I
        _lib = L
    return _lib


def check(status: int, where: str, allow=(QS_OK,)) -> int:
    if status not in allow:
        raise QSError(status, where)
    return status
