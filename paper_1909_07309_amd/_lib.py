"""ctypes declarations of libstig's C ABI (include/stig.h).

Loading fails loudly: there is no CPU fallback for any entry point.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstig.so")

STATUS = {0: "ok", 1: "not converged", -1: "invalid argument", -2: "out of device memory",
          -3: "HIP runtime error", -4: "breakdown", -5: "non-finite value", -6: "plan not set up"}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}


class StigError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libstig: {STATUS.get(code, code)} ({code}): {msg}")
        self.code = code


class StigInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("relres_true", C.c_double),
                ("relres_est", C.c_double), ("t_solve_ms", C.c_double)]


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_vp = C.c_void_p

# name -> (restype, argtypes)
SIGNATURES = {
    "stig_plan_create": (C.c_int, [C.POINTER(_vp), C.c_int, _ip, C.c_int, C.c_int, C.c_int, _vp]),
    "stig_plan_destroy": (None, [_vp]),
    "stig_set_stream": (C.c_int, [_vp, _vp]),
    "stig_set_option": (C.c_int, [_vp, C.c_int, C.c_int]),
    "stig_setup_1d_pencils": (C.c_int, [_vp, C.POINTER(_dp), C.POINTER(_dp), _dp, _dp,
                                        C.c_double, C.c_double]),
    "stig_set_diag_scaling": (C.c_int, [_vp, _vp]),
    "stig_set_A_csr": (C.c_int, [_vp, _vp, _vp, _vp, C.c_int64]),
    "stig_set_spatial_factors": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "stig_apply_Pinv": (C.c_int, [_vp, _vp, _vp, C.c_int, C.c_int, C.c_int]),
    "stig_apply_Pinv_noalloc": (C.c_int, [_vp, _vp, _vp, C.c_int, C.c_int, C.c_int]),
    "stig_matvec_A": (C.c_int, [_vp, _vp, _vp, C.c_int, C.c_int]),
    "stig_apply_mass": (C.c_int, [_vp, _vp, _vp, C.c_int]),
    "stig_lift_adjoint": (C.c_int, [_vp, _dp, _dp, _vp, _vp, C.c_int]),
    "stig_lift_apply": (C.c_int, [_vp, _dp, _dp, _vp, _vp, _vp, C.c_int]),
    "stig_workspace_bytes": (C.c_size_t, [_vp, C.c_int, C.c_int, C.c_int, C.c_int]),
    "stig_set_workspace": (C.c_int, [_vp, _vp, C.c_size_t]),
    "stig_gmres_solve": (C.c_int, [_vp, _vp, _vp, C.c_int, C.c_int, C.c_double, C.c_int,
                                   C.c_int, C.c_int, C.c_int, C.POINTER(StigInfo)]),
    "stig_plan_device_bytes": (C.c_size_t, [_vp]),
    "stig_profile_enable": (C.c_int, [_vp, C.c_int]),
    "stig_profile_reset": (C.c_int, [_vp]),
    "stig_profile_get": (C.c_int, [_vp, C.c_int, _dp, _dp, C.POINTER(C.c_longlong)]),
    "stig_set_diag_scaling_kron": (C.c_int, [_vp, _dp, _dp]),
    "stig_assemble_2d": (C.c_int, [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _vp, _vp, _dp, _dp,
                                   C.POINTER(C.c_int64)]),
    "stig_separate_2d": (C.c_int, [C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp]),
    "stig_assemble_3d": (C.c_int, [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _dp, _vp, _vp, _dp,
                                   _dp, C.POINTER(C.c_int64)]),
    "stig_separate_3d": (C.c_int, [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                   _dp, _dp, _dp]),
    "stig_kron_csr_rowptr": (C.c_int, [C.c_int, C.c_int, C.c_int64, _vp, _vp]),
    "stig_kron_csr_fill": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _dp, _dp]),
    "stig_quadrature": (C.c_int, [C.c_int, C.c_int, C.c_double, _dp, _dp]),
    "stig_assemble_1d": (C.c_int, [C.c_int, C.c_int, C.c_double, C.c_int, _dp, C.c_int, _dp]),
    "stig_load_1d": (C.c_int, [C.c_int, C.c_int, C.c_double, _dp, C.c_int, _dp]),
    "stig_sym_eig": (C.c_int, [C.c_int, _dp, _dp, _dp, _dp]),
    "stig_split_eig": (C.c_int, [C.c_int, _dp, _dp, _dp, _dp]),
    "stig_time_arrowhead": (C.c_int, [C.c_int, _dp, _dp, _dp, _dp, _ip]),
    "stig_status_string": (C.c_char_p, [C.c_int]),
    "stig_last_error": (C.c_char_p, []),
}

_lib = None


def lib():
    """The loaded libstig (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code, allow_warning=False):
    if code == 0 or (allow_warning and code > 0):
        return code
    msg = lib().stig_last_error().decode(errors="replace")
    raise StigError(code, msg)


def dptr(a):
    """ctypes double* of a C-contiguous float64 numpy array."""
    return a.ctypes.data_as(_dp)
