"""ctypes binding of libfraclap.so (declarations in include/fraclap.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Importing this module raises if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(HERE, "libfraclap.so")

FL_OK, FL_EINVAL, FL_ENOMEM, FL_EHIP, FL_ENOTSPD, FL_ENOCONV, FL_ESTATE, FL_EIO = 0, -1, -2, -3, -4, -5, -6, -7
FL_ELEM_P1, FL_ELEM_Q1 = 3, 4
FL_FP64, FL_MIXED = 0, 1
FL_MIXED_FP32_BAND = 1
STAGES = ["potrf", "sygst", "sy2sb", "sb2st", "stedc", "q2", "q1", "trsm", "refine"]
FL_NSTAGES = len(STAGES)

STATUS_NAMES = {FL_OK: "FL_OK", FL_EINVAL: "FL_EINVAL", FL_ENOMEM: "FL_ENOMEM", FL_EHIP: "FL_EHIP",
                FL_ENOTSPD: "FL_ENOTSPD", FL_ENOCONV: "FL_ENOCONV", FL_ESTATE: "FL_ESTATE", FL_EIO: "FL_EIO"}
FL_TUNE_F64, FL_TUNE_F32, FL_TUNE_SCALED = 0, 1, 2
FL_GV_AUTO, FL_GV_SQUARE16, FL_GV_SQUARE32, FL_GV_THIN = 0, 1, 2, 3

# Every symbol the header declares (checked by the CPU test-suite).
EXPORTS = [
    "fl_ctx_create", "fl_ctx_set_stream", "fl_ctx_destroy", "fl_last_error",
    "fl_assemble", "fl_assemble_sparse", "fl_op_from_dense", "fl_op_n", "fl_op_matrices", "fl_op_destroy",
    "fl_eigensolve", "fl_eigensolve_batched", "fl_eigensolve_batched_begin", "fl_eigensolve_batched_wait",
    "fl_eigenpairs", "fl_op_set_eigenpairs",
    "fl_op_save", "fl_op_load", "fl_op_info", "fl_inertia_count", "fl_eigensolve_interval",
    "fl_apply_fractional", "fl_apply_fractional_noalloc", "fl_grad_apply", "fl_apply_graph", "fl_apply_diffusion", "fl_grad_diffusion",
    "fl_gemm_tune", "fl_gemm_tuning_set", "fl_gemm_tuning_count", "fl_gemm_tuning_get", "fl_gemm_tuning_clear",
    "fl_dgemm", "fl_dpotrf", "fl_dsygst", "fl_dstedc", "fl_dsytrd_2stage", "fl_dsyevd",
    "fl_kernel_timing", "fl_kernel_time", "fl_measure_peaks",
]


class FlEigOpts(ctypes.Structure):
    _fields_ = [("band", ctypes.c_int32), ("leaf", ctypes.c_int32),
                ("refine_max_iters", ctypes.c_int32), ("refine_tol", ctypes.c_double),
                ("mixed_flags", ctypes.c_int32)]


class FlEigInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("index", ctypes.c_int64), ("refine_iters", ctypes.c_int32),
                ("refine_resid", ctypes.c_double), ("stage_ms", ctypes.c_double * FL_NSTAGES),
                ("total_ms", ctypes.c_double), ("flops_nominal", ctypes.c_double)]

    def as_dict(self):
        return {"status": self.status, "index": self.index, "refine_iters": self.refine_iters,
                "refine_resid": self.refine_resid, "total_ms": self.total_ms,
                "flops_nominal": self.flops_nominal,
                "stage_ms": {s: self.stage_ms[i] for i, s in enumerate(STAGES)}}


class FlSliceInfo(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64), ("slices", ctypes.c_int64), ("max_load", ctypes.c_int64),
                ("partition_rounds", ctypes.c_int64), ("iterations", ctypes.c_int64),
                ("max_residual", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class FlGemmChoice(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("ta", ctypes.c_int32), ("tb", ctypes.c_int32),
                ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("k", ctypes.c_int64),
                ("variant", ctypes.c_int32), ("split", ctypes.c_int32), ("group", ctypes.c_int32),
                ("ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class FraclapError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path: str = SO_PATH):
    """Load the HIP library (raises ImportError when it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_1911_11906_amd.build`")
    L = ctypes.CDLL(path)
    P, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "fl_ctx_create": ([i32, P, pp], i32),
        "fl_ctx_set_stream": ([P, P], i32),
        "fl_ctx_destroy": ([P], None),
        "fl_last_error": ([P], ctypes.c_char_p),
        "fl_assemble": ([P, i32, i64, P, i64, P, P, pp, ctypes.POINTER(i64), P], i32),
        "fl_assemble_sparse": ([P, i32, i64, P, i64, P, P, pp, ctypes.POINTER(i64), P], i32),
        "fl_op_from_dense": ([P, i64, P, P, i64, i32, pp], i32),
        "fl_op_n": ([P], i64),
        "fl_op_matrices": ([P, P, P, i64, i32], i32),
        "fl_op_destroy": ([P], None),
        "fl_eigensolve": ([P, i32, ctypes.POINTER(FlEigOpts), ctypes.POINTER(FlEigInfo)], i32),
        "fl_eigensolve_batched": ([P, i64, P, i32, P], i32),
        "fl_eigensolve_batched_begin": ([P, i64, P, i32, P], i32),
        "fl_eigensolve_batched_wait": ([P, P], i32),
        "fl_eigenpairs": ([P, P, P, i64, i32], i32),
        "fl_op_set_eigenpairs": ([P, P, P, i64, i32], i32),
        "fl_inertia_count": ([P, i64, P, P, ctypes.POINTER(i64)], i32),
        "fl_eigensolve_interval": ([P, dbl, dbl, i64, dbl, i64, P, P, i64, ctypes.POINTER(FlSliceInfo)], i32),
        "fl_op_save": ([P, ctypes.c_char_p], i32),
        "fl_op_load": ([P, ctypes.c_char_p, pp], i32),
        "fl_op_info": ([P, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                        ctypes.POINTER(dbl)], i32),
        "fl_apply_fractional": ([P, i64, P, i64, i64, P, i32, P, i64], i32),
        "fl_grad_apply": ([P, i64, P, i64, P, P, i64, P, i64, P], i32),
        "fl_apply_graph": ([P, i64, P, i64, i64, P, i32, P, i64], i32),
        "fl_apply_fractional_noalloc": ([P, i64, P, i64, i64, P, i32, P, i64], i32),
        "fl_apply_diffusion": ([P, i64, P, i64, i64, P, P, P, i32, P, i64], i32),
        "fl_grad_diffusion": ([P, i64, P, i64, P, P, P, P, i64, P, i64, P, P, P], i32),
        "fl_gemm_tune": ([P, i32, i32, i32, i64, i64, i64, i32, ctypes.POINTER(FlGemmChoice)], i32),
        "fl_gemm_tuning_set": ([ctypes.POINTER(FlGemmChoice)], i32),
        "fl_gemm_tuning_count": ([], i64),
        "fl_gemm_tuning_get": ([i64, ctypes.POINTER(FlGemmChoice)], i32),
        "fl_gemm_tuning_clear": ([], None),
        "fl_dgemm": ([P, i32, i32, i64, i64, i64, dbl, P, i64, P, i64, dbl, P, i64], i32),
        "fl_dpotrf": ([P, i64, P, i64, ctypes.POINTER(i64)], i32),
        "fl_dsygst": ([P, i64, P, i64, P, i64], i32),
        "fl_dstedc": ([P, i64, P, P, P, i64], i32),
        "fl_dsytrd_2stage": ([P, i64, P, i64, i32, P, P, P, i64], i32),
        "fl_dsyevd": ([P, i64, P, i64, i32, P, P, i64], i32),
        "fl_kernel_timing": ([i32], i32),
        "fl_kernel_time": ([ctypes.c_char_p, ctypes.POINTER(i64), ctypes.POINTER(dbl)], i32),
        "fl_measure_peaks": ([P, ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(dbl), i64], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L
