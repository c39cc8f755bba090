"""ctypes declarations of the C ABI in include/sketchycgal.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsketchycgal.so")

SCG_OK, SCG_EINVAL, SCG_ENOMEM, SCG_EHIP, SCG_ENUMERIC, SCG_ESTATE = range(6)
SCG_FP64, SCG_FP32_STREAM = 0, 1


class scg_params(C.Structure):
    _fields_ = [
        ("R", C.c_int32), ("T", C.c_int32), ("beta0", C.c_double), ("K", C.c_double),
        ("alpha", C.c_double), ("seed", C.c_uint64), ("q_mode", C.c_int32), ("q_fixed", C.c_int32),
        ("scale", C.c_int32), ("trace_correct", C.c_int32), ("reorth", C.c_int32),
        ("precision", C.c_int32), ("instance", C.c_int32), ("matrix_format", C.c_int32),
        ("autotune", C.c_int32), ("segments", C.c_int32), ("spmv_lanes", C.c_int32), ("spmv_grid", C.c_int32),
        ("basis_mode", C.c_int32), ("omega_mode", C.c_int32), ("trace_mode", C.c_int32),
        ("constraint_set", C.c_int32), ("batch_kernel", C.c_int32),
    ]


class scg_iter_log(C.Structure):
    _fields_ = [
        ("t", C.c_int32), ("q", C.c_int32), ("k", C.c_int32), ("flags", C.c_int32),
        ("xi", C.c_double), ("cv", C.c_double), ("p", C.c_double), ("infeas", C.c_double),
        ("gamma", C.c_double), ("gap", C.c_double), ("stop_obj", C.c_double), ("stop_feas", C.c_double),
        ("resid", C.c_double), ("beta", C.c_double), ("eta", C.c_double),
    ]


class scg_summary(C.Structure):
    _fields_ = [
        ("t_done", C.c_int32), ("status_flags", C.c_int32), ("objective", C.c_double),
        ("infeasibility", C.c_double), ("p_scaled", C.c_double), ("tau_scaled", C.c_double),
        ("c_F", C.c_double), ("alpha", C.c_double), ("alpha_scaled", C.c_double),
        ("spmv_lanes", C.c_int32), ("spmv_segments", C.c_int32), ("matrix_format", C.c_int32), ("spmv_grid", C.c_int32),
        ("batch_kernel", C.c_int32),
    ]


class scg_pr_params(C.Structure):
    _fields_ = [
        ("R", C.c_int32), ("T", C.c_int32), ("beta0", C.c_double), ("K", C.c_double),
        ("alpha", C.c_double), ("seed", C.c_uint64), ("q_mode", C.c_int32), ("q_fixed", C.c_int32),
        ("scale", C.c_int32), ("trace_correct", C.c_int32), ("instance", C.c_int32),
        ("mask_groups", C.c_int32), ("tile_cols", C.c_int32), ("mask_format", C.c_int32),
        ("autotune", C.c_int32),
    ]


class scg_pr_info(C.Structure):
    _fields_ = [
        ("t_done", C.c_int32), ("status_flags", C.c_int32), ("objective", C.c_double),
        ("infeasibility", C.c_double), ("p_scaled", C.c_double), ("tau_scaled", C.c_double),
        ("alpha", C.c_double), ("alpha_scaled", C.c_double), ("c_F", C.c_double), ("op_norm", C.c_double),
        ("n1", C.c_int32), ("n2", C.c_int32), ("tile_cols", C.c_int32), ("row_tile", C.c_int32),
        ("mask_groups", C.c_int32), ("mask_codes", C.c_int32),
    ]


EXPORTS = [
    "scg_default_params", "scg_workspace_size", "sketchycgal_init", "sketchycgal_step",
    "sketchycgal_reconstruct", "sketchycgal_log", "sketchycgal_summary", "sketchycgal_get_state",
    "sketchycgal_set_state", "sketchycgal_lanczos_coeffs", "sketchycgal_apply", "sketchycgal_time_spmv",
    "sketchycgal_destroy", "scg_status_string", "sketchycgal_round", "sketchycgal_set_constraints",
    "sketchycgal_set_ball",
    "scg_batch_workspace_size", "sketchycgal_batch_init", "sketchycgal_batch_step", "sketchycgal_batch_log",
    "sketchycgal_batch_summary", "sketchycgal_batch_get_state", "sketchycgal_batch_set_state", "sketchycgal_batch_reconstruct",
    "sketchycgal_batch_destroy", "sketchycgal_batch_round", "sketchycgal_batch_set_beta0",
    "scg_round_csr",
    "scg_pr_default_params", "scg_pr_workspace_size", "scg_pr_init", "scg_pr_step", "scg_pr_apply",
    "scg_pr_measure", "scg_pr_log", "scg_pr_summary", "scg_pr_get_state", "scg_pr_set_state",
    "scg_pr_reconstruct", "scg_pr_round", "scg_pr_destroy", "scg_pr_time_apply",
]

_lib = None


def load() -> C.CDLL:
    """Load the built HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1912_02949_amd/build.py "
                          "(the library has no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    lib.scg_default_params.argtypes = [P(scg_params)]
    lib.scg_default_params.restype = None
    lib.scg_workspace_size.argtypes = [P(scg_params), i64, i64, P(sz)]
    lib.sketchycgal_init.argtypes = [P(vp), P(scg_params), i64, i64, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.sketchycgal_step.argtypes = [vp, i32]
    lib.sketchycgal_reconstruct.argtypes = [vp, vp, vp, vp]
    lib.sketchycgal_log.argtypes = [vp, P(scg_iter_log), i32, P(i32)]
    lib.sketchycgal_summary.argtypes = [vp, P(scg_summary)]
    lib.sketchycgal_get_state.argtypes = [vp, P(i32), vp, vp, vp, P(C.c_double), P(C.c_double)]
    lib.sketchycgal_set_state.argtypes = [vp, i32, vp, vp, vp, C.c_double, C.c_double]
    lib.sketchycgal_lanczos_coeffs.argtypes = [vp, P(C.c_double), P(C.c_double), i32, P(i32), P(C.c_double)]
    lib.sketchycgal_apply.argtypes = [vp, vp, vp]
    lib.sketchycgal_time_spmv.argtypes = [vp, i32, P(C.c_double)]
    lib.sketchycgal_destroy.argtypes = [vp]
    lib.sketchycgal_destroy.restype = None
    lib.scg_batch_workspace_size.argtypes = [P(scg_params), i32, vp, i64, P(sz)]
    lib.sketchycgal_batch_init.argtypes = [P(vp), P(scg_params), i32, vp, i64, vp, vp, vp, vp, vp, sz, vp]
    lib.sketchycgal_batch_step.argtypes = [vp, i32]
    lib.sketchycgal_batch_set_beta0.argtypes = [vp, vp]
    lib.sketchycgal_batch_log.argtypes = [vp, i32, P(scg_iter_log), i32, P(i32)]
    lib.sketchycgal_batch_summary.argtypes = [vp, i32, P(scg_summary)]
    lib.sketchycgal_batch_get_state.argtypes = [vp, i32, P(i32), vp, vp, vp, P(C.c_double), P(C.c_double)]
    lib.sketchycgal_batch_set_state.argtypes = [vp, i32, i32, vp, vp, vp, C.c_double, C.c_double]
    lib.sketchycgal_batch_reconstruct.argtypes = [vp, i32, vp, vp, vp]
    lib.sketchycgal_round.argtypes = [vp, vp, vp, P(C.c_double), P(i32)]
    lib.sketchycgal_set_constraints.argtypes = [vp, vp, vp]
    lib.sketchycgal_set_ball.argtypes = [vp, C.c_double]
    lib.sketchycgal_batch_round.argtypes = [vp, i32, vp, vp, P(C.c_double), P(i32)]
    lib.scg_round_csr.argtypes = [i64, i64, vp, vp, vp, i32, vp, vp, P(C.c_double), P(i32), vp]
    lib.sketchycgal_batch_destroy.argtypes = [vp]
    lib.sketchycgal_batch_destroy.restype = None
    lib.scg_pr_default_params.argtypes = [P(scg_pr_params)]
    lib.scg_pr_default_params.restype = None
    lib.scg_pr_workspace_size.argtypes = [P(scg_pr_params), i64, i32, P(sz)]
    lib.scg_pr_init.argtypes = [P(vp), P(scg_pr_params), i64, i32, vp, vp, vp, vp, sz, vp]
    lib.scg_pr_step.argtypes = [vp, i32]
    lib.scg_pr_apply.argtypes = [vp, vp, vp, vp]
    lib.scg_pr_measure.argtypes = [vp, vp, vp]
    lib.scg_pr_log.argtypes = [vp, P(scg_iter_log), i32, P(i32)]
    lib.scg_pr_summary.argtypes = [vp, P(scg_pr_info), i32]
    lib.scg_pr_get_state.argtypes = [vp, P(i32), vp, vp, vp, P(C.c_double), P(C.c_double)]
    lib.scg_pr_set_state.argtypes = [vp, i32, vp, vp, vp, C.c_double, C.c_double]
    lib.scg_pr_reconstruct.argtypes = [vp, vp, vp, vp]
    lib.scg_pr_round.argtypes = [vp, vp, vp, vp, vp, P(C.c_double)]
    lib.scg_pr_destroy.argtypes = [vp]
    lib.scg_pr_time_apply.argtypes = [vp, i32, P(C.c_double)]
    lib.scg_status_string.argtypes = [C.c_int]
    lib.scg_status_string.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("scg_default_params", "sketchycgal_destroy", "scg_status_string", "scg_pr_default_params"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


class SCGError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = load().scg_status_string(status).decode()
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


def check(status: int, where: str):
    if status != SCG_OK:
        raise SCGError(status, where)
