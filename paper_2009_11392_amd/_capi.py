"""ctypes declarations of the libgn C ABI (include/gn.h).  Marshalling only."""
from __future__ import annotations

import ctypes
import os

from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgn.so")

GN_OK, GN_ERR_ARG, GN_ERR_SHAPE, GN_ERR_DTYPE, GN_ERR_ALIGN = 0, 1, 2, 3, 4
GN_ERR_WORKSPACE, GN_ERR_HIP, GN_ERR_NUMERIC, GN_ERR_UNSUPPORTED = 5, 6, 7, 8
GN_SKETCH_GAUSSIAN, GN_SKETCH_SRHT, GN_SKETCH_USER = 0, 1, 2
GN_MODE_F64, GN_MODE_F32, GN_MODE_BF16_BS, GN_MODE_F16_BS = 0, 1, 2, 3
GN_BATCH_PASS, GN_BATCH_CORE, GN_BATCH_ALL = 1, 2, 3
GN_DT_F64, GN_DT_F32, GN_DT_BF16, GN_DT_F16 = 0, 1, 2, 3
(GN_OP_SKETCH, GN_OP_CORE, GN_OP_FACTORS, GN_OP_APPLY, GN_OP_RESIDUAL, GN_OP_SRHT,
 GN_OP_BACKWARD, GN_OP_MATERIALIZE, GN_OP_UPDATE, GN_OP_CHECK) = range(10)
(GN_CORE_QR, GN_CORE_SVD, GN_CORE_LIFT_SVD, GN_CORE_LIFT_RRQR, GN_CORE_LIFT_DIAG) = range(5)

EXPORTED = (
    "gn_workspace_size", "gn_generate_gaussian", "gn_srht_generate", "gn_sketch_prepare",
    "gn_sketch_pass", "gn_sketch", "gn_core", "gn_core_check",
    "gn_factors", "gn_apply", "gn_backward", "gn_sketch_extend", "gn_sketch_append",
    "gn_sketch_update", "gn_residual", "gn_residual_noalloc", "gn_quantize_bf16_bs",
    "gn_quantize_f16_bs",
    "gn_batch_workspace_size", "gn_batch_prepare", "gn_batch_solve", "gn_status_string",
    "gn_version",
)


class GnProblem(ctypes.Structure):
    _fields_ = [("m", c_int64), ("n", c_int64), ("r", c_int64), ("l", c_int64),
                ("kind_x", c_int32), ("kind_y", c_int32), ("seed", c_uint64),
                ("mode", c_int32), ("core_method", c_int32),
                ("eps", c_double), ("nu_x", c_double), ("nu_y", c_double)]


class GnCoreOut(ctypes.Structure):
    _fields_ = [("k", c_void_p), ("status", c_void_p), ("Q1", c_void_p), ("R", c_void_p),
                ("Q2", c_void_p), ("R2", c_void_p)]


class GnBatchProblem(ctypes.Structure):
    _fields_ = [("m", c_int64), ("n", c_int64), ("r", c_int64), ("l", c_int64),
                ("seed", c_uint64), ("eps", c_double), ("A", c_void_p), ("lda", c_int64),
                ("AX", c_void_p), ("ldax", c_int64), ("YtA", c_void_p), ("ldya", c_int64),
                ("core", GnCoreOut)]


class GnBatchPlan(ctypes.Structure):
    _fields_ = [("count", c_int32), ("n_pass_items", c_int32), ("n_core_items", c_int32),
                ("grid", c_int32), ("max_m", c_int64), ("max_n", c_int64), ("max_r", c_int64),
                ("max_rl", c_int64), ("ws_bytes", c_size_t), ("off_desc", c_size_t),
                ("off_items", c_size_t), ("off_qr", c_size_t), ("off_qr2", c_size_t),
                ("off_trunc", c_size_t), ("off_widen", c_size_t), ("pass_flops", c_double),
                ("pass_bytes", c_double), ("tile_policy", c_int32 * 4),
                ("pass_threads", c_int32)]


class GNError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {msg} (status {code})")
        self.code = code


_lib = None


def lib(path: str = LIB_PATH):
    """Load libgn.so (fails loudly if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"libgn.so not found at {path}: build it with `python -m paper_2009_11392_amd.build` "
            "(hipcc, gfx950). There is no fallback path.")
    L = ctypes.CDLL(path)
    P = POINTER(GnProblem)
    L.gn_workspace_size.argtypes = [P, c_int32, c_int64, POINTER(c_size_t)]
    L.gn_generate_gaussian.argtypes = [c_uint64, c_int32, c_int64, c_int64, c_int64, c_int64,
                                       c_int32, c_int32, c_void_p, c_int64, c_void_p]
    L.gn_srht_generate.argtypes = [c_uint64, c_int64, c_int64, c_void_p, c_void_p, c_void_p,
                                   c_size_t, c_void_p]
    L.gn_sketch.argtypes = [P, c_void_p, c_int64, c_void_p, c_void_p, c_int64, c_void_p, c_int64,
                            c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_void_p,
                            c_size_t, c_void_p]
    L.gn_sketch_prepare.argtypes = [P, c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_void_p,
                                    c_void_p, c_size_t, c_void_p]
    L.gn_sketch_pass.argtypes = [P, c_void_p, c_int64, c_void_p, c_void_p, c_int64, c_void_p,
                                 c_int64, c_void_p, c_size_t, c_void_p]
    L.gn_core.argtypes = [P, c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                          POINTER(GnCoreOut), c_void_p, c_size_t, c_void_p]
    L.gn_core_check.argtypes = [P, POINTER(GnCoreOut), c_double, c_int32, c_int32, c_void_p,
                                c_void_p, c_size_t, c_void_p]
    L.gn_factors.argtypes = [P, c_void_p, c_int64, c_void_p, c_int64, POINTER(GnCoreOut), c_void_p,
                             c_int64, c_void_p, c_int64, c_void_p, c_size_t, c_void_p]
    L.gn_apply.argtypes = [P, c_int32, c_void_p, c_int64, c_void_p, c_int64, POINTER(GnCoreOut),
                           c_void_p, c_int64, c_int64, c_void_p, c_int64, c_void_p, c_size_t,
                           c_void_p]
    L.gn_backward.argtypes = [P, c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                              c_void_p, c_int64, POINTER(GnCoreOut), c_void_p, c_int64, c_void_p,
                              c_size_t, c_void_p]
    L.gn_sketch_extend.argtypes = [P, P, c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                                   c_void_p, c_size_t, c_void_p]
    L.gn_sketch_append.argtypes = [P, c_int32, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                                   c_void_p, c_int64, c_void_p, c_size_t, c_void_p]
    L.gn_sketch_update.argtypes = [P, c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                                   c_void_p, c_size_t, c_void_p]
    BP = POINTER(GnBatchProblem)
    L.gn_batch_workspace_size.argtypes = [BP, c_int32, POINTER(c_size_t)]
    L.gn_batch_prepare.argtypes = [BP, c_int32, c_void_p, POINTER(GnBatchPlan), c_void_p, c_size_t,
                                   c_void_p]
    L.gn_batch_solve.argtypes = [POINTER(GnBatchPlan), c_int32, c_void_p, c_size_t, c_void_p]
    L.gn_residual.argtypes = [c_int64, c_int64, c_int64, c_void_p, c_int64, c_int32, c_void_p,
                              c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_void_p, c_size_t,
                              c_void_p]
    L.gn_residual_noalloc.argtypes = [c_int64, c_int64, c_int64, c_void_p, c_int64, c_int32,
                                      c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_void_p,
                                      c_void_p]
    L.gn_quantize_bf16_bs.argtypes = [c_int64, c_int64, c_void_p, c_int64, c_int32, c_void_p,
                                      c_int64, c_void_p, c_void_p]
    L.gn_quantize_f16_bs.argtypes = [c_int64, c_int64, c_void_p, c_int64, c_int32, c_void_p,
                                     c_int64, c_void_p, c_void_p]
    for name in EXPORTED[:-2]:
        getattr(L, name).restype = c_int32
    L.gn_status_string.argtypes = [c_int32]
    L.gn_status_string.restype = c_char_p
    L.gn_version.argtypes = []
    L.gn_version.restype = c_char_p
    _lib = L
    return L


def check(code: int, where: str):
    if code != GN_OK:
        msg = lib().gn_status_string(code).decode()
        raise GNError(code, where, msg)
