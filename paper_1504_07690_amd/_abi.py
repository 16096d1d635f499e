"""ctypes declarations of the libssm C ABI (include/ssm.h).

Marshalling only: every function here forwards to the library of the same name.
Importing this module loads libssm.so from the package directory and raises
ImportError if it is missing; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libssm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libssm.so not built at {LIB_PATH}; run python -m paper_1504_07690_amd.build")
lib = C.CDLL(LIB_PATH)

# status codes
SSM_OK, SSM_ERR_ARG, SSM_ERR_WORKSPACE, SSM_ERR_HIP, SSM_ERR_BOUNDS, SSM_ERR_NONFINITE, SSM_ERR_STATE, \
    SSM_ERR_UNSUPPORTED = range(8)
# precisions
SSM_FP64, SSM_FP32, SSM_FP32_BF16SWEEP, SSM_FP32_BF16X3 = 0, 1, 2, 3


class ssm_csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p),
                ("values", C.c_void_p)]


class ssm_params(C.Structure):
    _fields_ = [("lo", C.c_double), ("hi", C.c_double), ("sigma", C.c_double), ("tau", C.c_double),
                ("range_slack", C.c_double), ("nv", C.c_int32), ("degree", C.c_int32), ("nt", C.c_int32),
                ("precision", C.c_int32), ("seed", C.c_uint64), ("ckpt_every", C.c_int32), ("dgc", C.c_int32),
                ("method", C.c_int32), ("nv_hybrid", C.c_int32), ("floor_scale", C.c_double),
                ("plan_batch", C.c_int32), ("plan_chunk", C.c_int32), ("lattice", C.c_int32 * 3)]


class ssm_stats(C.Structure):
    _fields_ = [("ms_total", C.c_double), ("ms_recurrence", C.c_double), ("ms_sweep", C.c_double),
                ("ms_gram", C.c_double), ("ms_geneig", C.c_double), ("spmm_launches", C.c_int64),
                ("sweep_launches", C.c_int64), ("passes", C.c_int32), ("chunk", C.c_int32),
                ("batch", C.c_int32), ("gram_segments", C.c_int32), ("split_k3", C.c_int32),
                ("box_stencil", C.c_int32)]


class ssm_backward_stats(C.Structure):
    _fields_ = [("ms_total", C.c_double), ("ms_geneig", C.c_double), ("ms_zbar", C.c_double),
                ("ms_ybar", C.c_double), ("ms_recompute", C.c_double), ("ms_reverse", C.c_double),
                ("segments", C.c_int32), ("recomputed", C.c_int32), ("ms_forward", C.c_double),
                ("passes", C.c_int32), ("levels", C.c_int32)]


class ssm_views(C.Structure):
    _fields_ = [("w", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("k_w", C.c_void_p),
                ("k_z", C.c_void_p), ("coeff", C.c_void_p), ("chunk", C.c_int32), ("batch", C.c_int32),
                ("first_point_of_last_batch", C.c_int32), ("elem_bytes", C.c_int32),
                ("moments", C.c_void_p), ("coeff_sq", C.c_void_p), ("s_floor", C.c_void_p)]


SCALAR_FN = C.CFUNCTYPE(C.c_double, C.c_double, C.c_void_p)

_P = C.c_void_p
_SIGS = {
    "ssm_last_error": (C.c_char_p, []),
    "ssm_status_str": (C.c_char_p, [C.c_int]),
    "ssm_workspace_size": (C.c_int, [C.POINTER(ssm_csr), C.POINTER(ssm_params), C.c_size_t,
                                     C.POINTER(C.c_size_t)]),
    "ssm_create": (C.c_int, [C.POINTER(ssm_csr), C.POINTER(ssm_params), C.POINTER(C.c_double), _P, _P,
                             C.c_size_t, _P, C.POINTER(_P)]),
    "ssm_dos": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "ssm_trace": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "ssm_dgc": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "ssm_get_stats": (C.c_int, [_P, C.POINTER(ssm_stats)]),
    "ssm_get_views": (C.c_int, [_P, C.POINTER(ssm_views)]),
    "ssm_destroy": (C.c_int, [_P]),
    "ssm_backward_workspace_size": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "ssm_backward": (C.c_int, [_P, C.POINTER(C.c_double), _P, _P, C.c_size_t]),
    "ssm_get_backward_stats": (C.c_int, [_P, C.POINTER(ssm_backward_stats)]),
    "ssm_trace_weights": (C.c_int, [C.c_double, C.c_double, C.c_int32, C.c_int64, C.c_double, C.c_double,
                                    C.c_double, SCALAR_FN, _P, C.POINTER(C.c_double)]),
    "ssm_trace_weights_exp": (C.c_int, [C.c_double, C.c_double, C.c_int32, C.c_int64, C.c_double, C.c_double,
                                        C.c_double, C.POINTER(C.c_double)]),
    "ssm_coefficients": (C.c_int, [C.c_double, C.c_double, C.c_double, C.c_int64, _P, C.c_int32, C.c_int32,
                                   _P, _P, _P]),
    "ssm_gaussian_block": (C.c_int, [C.c_uint64, C.c_int64, C.c_int32, C.c_int32, _P, _P]),
    "ssm_chebyshev": (C.c_int, [C.POINTER(ssm_csr), C.c_double, C.c_double, C.c_int32, C.c_int32, C.c_int32,
                                _P, _P, _P]),
    "ssm_sweep": (C.c_int, [C.c_int32, C.c_int64, C.c_int32, C.c_int32, _P, C.c_int64, _P, _P, C.c_int32, _P]),
    "ssm_split_coefficients": (C.c_int, [_P, C.c_int64, C.c_int32, C.c_int32, _P, _P, C.c_int64, _P]),
    "ssm_sweep_split": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, _P, _P, C.c_int64, _P, _P, C.c_int32, C.c_int32,
                                 _P]),
    "ssm_gram": (C.c_int, [C.c_int32, C.c_int64, C.c_int32, C.c_int32, _P, _P, _P, _P, C.c_int32, _P, _P]),
    "ssm_gram_noalloc": (C.c_int, [C.c_int32, C.c_int64, C.c_int32, C.c_int32, _P, _P, _P, _P, C.c_int32, _P]),
    "ssm_geneig_trace": (C.c_int, [C.c_int32, C.c_int32, _P, _P, C.c_double, C.c_double, C.c_double, _P, _P,
                                   _P, _P]),
    "ssm_geneig_trace_scratch_doubles": (C.c_int64, [C.c_int32, C.c_int32]),
}

for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


class SSMError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib.ssm_last_error().decode()
        super().__init__(f"{where}: {lib.ssm_status_str(status).decode()} ({status}): {msg}")


def check(status: int, where: str) -> None:
    if status != SSM_OK:
        raise SSMError(status, where)
