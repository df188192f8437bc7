"""ctypes view of libskls.so (declarations in include/skls.h)."""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libskls.so")

F64, F32, BF16 = 0, 1, 2
DENSE, CSR = 0, 1
SKETCH_AUTO, SKETCH_ATOMIC, SKETCH_SORTED, SKETCH_BINNED = 0, 1, 2, 3

STATUS = {
    0: "SKLS_OK",
    1: "SKLS_ERR_ARG",
    2: "SKLS_ERR_SHAPE",
    3: "SKLS_ERR_DTYPE",
    4: "SKLS_ERR_RANK",
    5: "SKLS_ERR_NOCONV",
    6: "SKLS_ERR_WORKSPACE",
    7: "SKLS_ERR_DEVICE",
    8: "SKLS_ERR_NOTIMPL",
}


class SklsMatrix(ctypes.Structure):
    _fields_ = [
        ("layout", c_int32),
        ("dtype", c_int32),
        ("n", c_int64),
        ("d", c_int64),
        ("ld", c_int64),
        ("nnz", c_int64),
        ("row_ptr", c_void_p),
        ("row_ptr_64", c_int32),
        ("reserved", c_int32),
        ("col_idx", c_void_p),
        ("val", c_void_p),
    ]


class SklsSketchPlanDesc(ctypes.Structure):
    _fields_ = [
        ("n", c_int64),
        ("d", c_int64),
        ("t", c_int64),
        ("row_start", c_int64),
        ("seed", c_uint64),
        ("layout", c_int32),
        ("row_ptr_64", c_int32),
        ("variant", c_int32),
        ("out_dtype", c_int32),
        ("bytes", c_int64),
        ("reserved", c_int64 * 2),
    ]


class SklsLstsqOpts(ctypes.Structure):
    _fields_ = [
        ("t", c_int64),
        ("seed", c_uint64),
        ("delta", c_double),
        ("sigma_lb", c_double),
        ("max_iter", c_int32),
        ("precision", c_int32),
        ("sketch_only", c_int32),
        ("variant", c_int32),
        ("w", c_void_p),
        ("x0", c_void_p),
        ("max_retries", c_int32),
        ("second_stage", c_int32),
    ]


class SklsLstsqInfo(ctypes.Structure):
    _fields_ = [
        ("iterations", c_int32),
        ("refinements", c_int32),
        ("certified", c_int32),
        ("retries", c_int32),
        ("resid_norm", c_double),
        ("grad_norm", c_double),
        ("ratio_bound", c_double),
        ("ms_sketch", c_double),
        ("ms_qr", c_double),
        ("ms_iter", c_double),
    ]


class SklsLowRankOpts(ctypes.Structure):
    _fields_ = [
        ("k", c_int64),
        ("t_r", c_int64),
        ("t_s", c_int64),
        ("seed", c_uint64),
        ("eps", c_double),
        ("k_g", c_int32),
        ("oversample", c_int32),
        ("max_iter", c_int32),
        ("tol", c_double),
        ("reserved", c_int32 * 4),
    ]


class SklsLowRankInfo(ctypes.Structure):
    _fields_ = [
        ("t_r", c_int64),
        ("t_s", c_int64),
        ("rows_sampled", c_int64),
        ("nnz_sampled", c_int64),
        ("iterations", c_int32),
        ("converged", c_int32),
        ("resid_fro", c_double),
        ("fro_norm", c_double),
        ("ms_sketch", ctypes.c_float),
        ("ms_sample", ctypes.c_float),
        ("ms_topk", ctypes.c_float),
        ("ms_factors", ctypes.c_float),
        ("reserved", c_int32 * 4),
    ]


class SklsMultiOpts(ctypes.Structure):
    _fields_ = [
        ("t", c_int64),
        ("t_s", c_int64),
        ("seed", c_uint64),
        ("k_g", c_int32),
        ("reserved", c_int32 * 5),
    ]


class SklsMultiInfo(ctypes.Structure):
    _fields_ = [
        ("rows_sampled", c_int64),
        ("resid_fro", c_double),
        ("b_fro", c_double),
        ("ms_scores", ctypes.c_float),
        ("ms_solve", ctypes.c_float),
        ("reserved", c_int32 * 4),
    ]


class SklsLpOpts(ctypes.Structure):
    _fields_ = [
        ("p", c_double),
        ("q", c_int64),
        ("v", c_int64),
        ("a", c_int32),
        ("k_g", c_int32),
        ("w", c_int64),
        ("s1", c_double),
        ("s2", c_double),
        ("seed", c_uint64),
        ("max_iter", c_int32),
        ("reserved0", c_int32),
        ("tol", c_double),
        ("reserved", c_int64 * 4),
    ]


class SklsLpInfo(ctypes.Structure):
    _fields_ = [
        ("rows_stage1", c_int64),
        ("rows_stage2", c_int64),
        ("iters_stage1", c_int32),
        ("iters_stage2", c_int32),
        ("converged", c_int32),
        ("reserved0", c_int32),
        ("obj_stage1", c_double),
        ("obj", c_double),
        ("coreset_obj", c_double),
        ("ms_condition", ctypes.c_float),
        ("ms_stage1", ctypes.c_float),
        ("ms_stage2", ctypes.c_float),
        ("reserved1", c_int32),
        ("reserved", c_int64 * 4),
    ]


# name -> (restype, argtypes); every symbol declared in include/skls.h
SIGNATURES = {
    "skls_status_str": (c_char_p, [c_int32]),
    "skls_last_error": (c_char_p, []),
    "skls_version": (c_char_p, []),
    "skls_hash": (c_int32, [c_int64, c_int64, c_uint64, c_int64, c_void_p, c_void_p, c_void_p]),
    "skls_sketch_workspace": (c_int32, [POINTER(SklsMatrix), c_int64, c_int32, POINTER(c_size_t)]),
    "skls_sketch": (c_int32, [POINTER(SklsMatrix), c_void_p, c_int32, c_int64, c_uint64, c_void_p, c_int32,
                              c_void_p, c_void_p, c_int32, c_void_p, c_size_t, c_void_p]),
    "skls_sketch_rows": (c_int32, [POINTER(SklsMatrix), c_int64, c_void_p, c_int32, c_int64, c_uint64, c_void_p,
                                   c_int32, c_void_p, c_void_p, c_int32, c_void_p, c_size_t, c_void_p]),
    "skls_sketch_plan_workspace": (c_int32, [POINTER(SklsMatrix), c_int64, c_int32, c_int32, POINTER(c_size_t)]),
    "skls_sketch_plan": (c_int32, [POINTER(SklsMatrix), c_int64, c_int64, c_uint64, c_int32, c_int32, c_void_p,
                                   c_size_t, POINTER(SklsSketchPlanDesc), c_void_p]),
    "skls_sketch_planned": (c_int32, [POINTER(SklsMatrix), c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                                      POINTER(SklsSketchPlanDesc), c_void_p, c_size_t, c_void_p]),
    "skls_sketch_noalloc": (c_int32, [POINTER(SklsMatrix), c_void_p, c_int32, c_int64, c_uint64, c_void_p, c_int32,
                                      c_void_p, c_void_p, c_int32, c_void_p]),
    "skls_sketch_general_workspace": (c_int32, [POINTER(SklsMatrix), c_int64, c_int64, c_int32, POINTER(c_size_t)]),
    "skls_sketch_general": (c_int32, [POINTER(SklsMatrix), c_void_p, c_int32, c_int64, c_int64, c_int32, c_uint64,
                                      c_int32, c_void_p, c_void_p, c_int32, c_void_p, c_size_t, c_void_p]),
    "skls_qr_r_workspace": (c_int32, [c_int64, c_int64, POINTER(c_size_t)]),
    "skls_qr_r": (c_int32, [c_void_p, c_int32, c_int64, c_int64, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "skls_lstsq_workspace": (c_int32, [POINTER(SklsMatrix), POINTER(SklsLstsqOpts), POINTER(c_size_t)]),
    "skls_lstsq": (c_int32, [POINTER(SklsMatrix), c_void_p, POINTER(SklsLstsqOpts), c_void_p,
                             POINTER(SklsLstsqInfo), c_void_p, c_size_t, c_void_p]),
    "skls_second_stage_workspace": (c_int32, [c_int64, c_int64, c_int64, POINTER(c_size_t)]),
    "skls_second_stage": (c_int32, [c_void_p, c_void_p, c_int32, c_int64, c_int64, c_int64, c_uint64, c_void_p,
                                    c_void_p, c_void_p, c_size_t, c_void_p]),
    "skls_leverage_workspace": (c_int32, [POINTER(SklsMatrix), c_int64, c_int32, POINTER(c_size_t)]),
    "skls_leverage_scores": (c_int32, [POINTER(SklsMatrix), c_int64, c_uint64, c_int32, c_void_p, c_void_p,
                                       c_void_p, c_size_t, c_void_p]),
    "skls_leverage_from_r_workspace": (c_int32, [POINTER(SklsMatrix), c_int32, POINTER(c_size_t)]),
    "skls_leverage_scores_from_r": (c_int32, [POINTER(SklsMatrix), c_void_p, c_int32, c_void_p, c_uint64, c_void_p,
                                              c_void_p, c_size_t, c_void_p]),
    "skls_gram_workspace": (c_int32, [POINTER(SklsMatrix), POINTER(c_size_t)]),
    "skls_gram": (c_int32, [POINTER(SklsMatrix), c_void_p, c_void_p, c_size_t, c_void_p]),
    "skls_learned_workspace": (c_int32, [POINTER(SklsMatrix), c_int64, POINTER(c_size_t)]),
    "skls_learned_grad": (c_int32, [POINTER(SklsMatrix), c_void_p, c_int64, c_uint64, c_void_p, c_float, c_int32,
                                    c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "skls_learned_grad_planned": (c_int32, [POINTER(SklsMatrix), c_void_p, POINTER(SklsSketchPlanDesc), c_void_p,
                                            c_size_t, c_void_p, c_float, c_int32, c_void_p, c_void_p, c_void_p,
                                            c_size_t, c_void_p]),
    "skls_learned_batch_workspace": (c_int32, [POINTER(SklsMatrix), c_int64, POINTER(c_size_t)]),
    "skls_learned_grad_batch": (c_int32, [c_int32, POINTER(SklsMatrix), POINTER(c_void_p), POINTER(c_float),
                                          POINTER(SklsSketchPlanDesc), c_void_p, c_size_t, c_void_p, c_int32,
                                          c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "skls_adam_step": (c_int32, [c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_float, c_float,
                                 c_float, c_float, c_void_p]),
    "skls_profile_enable": (c_int32, [c_int32]),
    "skls_profile_count": (c_int32, []),
    "skls_profile_get": (c_int32, [c_int32, POINTER(c_char_p), POINTER(c_int64), POINTER(c_double)]),
    "skls_multi_lstsq_workspace": (c_int32, [POINTER(SklsMatrix), c_int64, POINTER(SklsMultiOpts), POINTER(c_size_t)]),
    "skls_multi_lstsq": (c_int32, [POINTER(SklsMatrix), c_void_p, c_int64, POINTER(SklsMultiOpts), c_void_p, c_void_p,
                                   c_void_p, POINTER(SklsMultiInfo), c_void_p, c_size_t, c_void_p]),
    "skls_lp_regression_workspace": (c_int32, [POINTER(SklsMatrix), POINTER(SklsLpOpts), POINTER(c_size_t)]),
    "skls_lp_regression": (c_int32, [POINTER(SklsMatrix), c_void_p, POINTER(SklsLpOpts), c_void_p, c_void_p,
                                     c_void_p, c_void_p, c_void_p, c_void_p, POINTER(SklsLpInfo), c_void_p,
                                     c_size_t, c_void_p]),
    "skls_low_rank_workspace": (c_int32, [POINTER(SklsMatrix), POINTER(SklsLowRankOpts), POINTER(c_size_t)]),
    "skls_low_rank": (c_int32, [POINTER(SklsMatrix), POINTER(SklsLowRankOpts), c_void_p, c_void_p, c_void_p,
                                POINTER(SklsLowRankInfo), c_void_p, c_size_t, c_void_p]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libskls.so and declare every entry point; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build the HIP library first "
            "(python paper_1207_6365_amd/build.py)"
        )
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class SklsError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {message}")


def check(status: int) -> None:
    if status != 0:
        msg = load().skls_last_error()
        raise SklsError(status, msg.decode() if msg else "")

