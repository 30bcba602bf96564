"""ctypes loader for libdelimit.so.  Marshalling only: every step of the
layers runs in the library's HIP kernels.  Importing this module does not
touch the GPU; loading fails loudly when the library is not built."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdelimit.so")

DLM_OK, DLM_EINVAL, DLM_ESINGULAR, DLM_ENOMEM, DLM_EDEVICE, DLM_EWORKSPACE = range(6)
DLM_FP32, DLM_BF16 = 0, 1
DLM_LSC_RESAMPLE, DLM_LSC_FOLDED = 0, 1
DLM_RELU_OUT, DLM_RELU_IN = 1, 2
DLM_IO_IN_BF16, DLM_IO_OUT_BF16 = 1, 2

_p = C.c_void_p
_dp = C.POINTER(C.c_double)
_i64 = C.c_int64
_int = C.c_int
_dbl = C.c_double
_st = C.c_int  # dlm_status

# name -> (restype, argtypes)
SIGNATURES = {
    "dlm_status_str": (C.c_char_p, [_int]),
    "dlm_last_error": (C.c_char_p, []),
    "dlm_version": (_int, []),
    "dlm_sh_basis": (_st, [_int, _dp, _i64, _dp]),
    "dlm_sh_fit_matrix": (_st, [_int, _dp, _i64, _dbl, _dp]),
    "dlm_lsc_kernel_points": (_st, [_dp, _i64, C.POINTER(_int), _int, _dbl, _dp]),
    "dlm_sh_plan_create": (_st, [_dp, _dp, _i64, _int, _dbl, _dbl, _dbl, C.POINTER(_p)]),
    "dlm_sh_plan_info": (_st, [_p, C.POINTER(_int), C.POINTER(_int), C.POINTER(_i64)]),
    "dlm_sh_plan_shell": (_st, [_p, _int, C.POINTER(_i64), C.POINTER(_dbl), C.POINTER(_i64)]),
    "dlm_sh_plan_matrices": (_st, [_p, _int, _dp, _dp]),
    "dlm_sh_plan_fit_status": (_st, [_p]),
    "dlm_sh_plan_update_gradients": (_st, [_p, _dp, _p]),
    "dlm_sh_plan_destroy": (None, [_p]),
    "dlm_signal2sh_fwd": (_st, [_p, _p, _p, _i64, _int, _p]),
    "dlm_signal2sh_bwd": (_st, [_p, _p, _p, _i64, _int, _p]),
    "dlm_sh2signal_fwd": (_st, [_p, _p, _p, _i64, _int, _p]),
    "dlm_sh2signal_bwd": (_st, [_p, _p, _p, _i64, _int, _p]),
    "dlm_lsc_plan_create": (_st, [_dp, _i64, _int, _int, C.POINTER(_int), _int, _dbl, _dbl, C.POINTER(_p)]),
    "dlm_lsc_plan_info": (_st, [_p, C.POINTER(_int), C.POINTER(_int), C.POINTER(_int), C.POINTER(_i64)]),
    "dlm_lsc_plan_tables": (_st, [_p, _dp, _dp, _dp]),
    "dlm_lsc_plan_destroy": (None, [_p]),
    "dlm_lsc_workspace_bytes": (_st, [_p, _int, _int, _i64, _int, _int, C.POINTER(C.c_size_t)]),
    "dlm_lsc_fwd": (_st, [_p, _p, _int, _p, _p, _int, _p, _i64, _int, _int, _p, C.c_size_t, _int, _p]),
    "dlm_lsc_bwd": (_st, [_p, _p, _int, _p, _int, _p, _p, _p, _p, _p, _i64, _int, _int, _p, C.c_size_t, _int, _p]),
    "dlm_lsc_fwd_io": (_st, [_p, _p, _int, _p, _p, _int, _p, _i64, _int, _int, _p, _int, _p, C.c_size_t, _int, _p]),
    "dlm_lsc_bwd_io": (_st, [_p, _p, _int, _p, _int, _p, _p, _p, _p, _p, _i64, _int, _int, _p, _int, _p, C.c_size_t,
                             _int, _p]),
    "dlm_mse_workspace_bytes": (C.c_size_t, [_i64]),
    "dlm_mse_fwd_bwd": (_st, [_p, _p, _i64, _p, _p, _p, C.c_size_t, _p]),
    "dlm_adam_step": (_st, [_p, _p, _p, _p, _i64, C.c_float, C.c_float, C.c_float, C.c_float, _i64, _p]),
    "dlm_signal2sh_raw_workspace_bytes": (C.c_size_t, [_i64]),
    "dlm_signal2sh_fwd_raw": (_st, [_p, _p, _p, _i64, _p, C.c_size_t, _int, _p]),
    "dlm_relmse_fwd_bwd": (_st, [_p, _p, _i64, C.c_float, _p, _p, _p, C.c_size_t, _p]),
    "dlm_sh2signal_mse_supported": (_int, [_p]),
    "dlm_sh2signal_mse_workspace_bytes": (C.c_size_t, [_p, _i64]),
    "dlm_sh2signal_mse_fwd_bwd": (_st, [_p, _p, _p, _i64, _p, _p, _p, _p, C.c_size_t, _int, _p]),
    "dlm_sh2signal_mse_static_scratch_bytes": (C.c_size_t, []),
    "dlm_sh2signal_mse_fwd_bwd_noalloc": (_st, [_p, _p, _p, _i64, _p, _p, _p, _int, _p]),
    "dlm_peak_copy": (_st, [_p, _p, C.c_size_t, _p]),
    "dlm_peak_mfma_out_floats": (C.c_size_t, [_int]),
    "dlm_peak_mfma_flops": (_dbl, [_int, _int, _int]),
    "dlm_peak_mfma": (_st, [_int, _int, _int, _p, _p]),
    "dlm_timing_enable": (_st, [_int]),
    "dlm_timing_reset": (_st, []),
    "dlm_timing_count": (_int, []),
    "dlm_timing_entry": (_st, [_int, C.c_char_p, C.c_size_t, C.POINTER(_dbl), C.POINTER(_i64), C.POINTER(_dbl),
                               C.POINTER(_dbl)]),
}

_lib = None


class DelimitError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def lib() -> C.CDLL:
    """Load libdelimit.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1808_01517_amd.build` "
                               "(or __graft_entry__.build()); there is no fallback path")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != DLM_OK:
        msg = lib().dlm_last_error().decode()
        raise DelimitError(status, msg or lib().dlm_status_str(status).decode())


def dptr(a):
    """ctypes double* of a C-contiguous float64 numpy array."""
    return a.ctypes.data_as(_dp)
