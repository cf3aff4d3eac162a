"""ctypes binding of the C ABI in include/rk.h (argument marshalling only).

Every step of the solver runs in the HIP library ``librk.so``; this module
only converts Python/torch arguments to pointers and structs.  Importing it
raises if the library has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (load torch's HIP runtime before the library)

HERE = os.path.dirname(os.path.abspath(__file__))
# RK_LIB_PATH selects another build of the same library (tuning experiments)
LIB_PATH = os.environ.get("RK_LIB_PATH", os.path.join(HERE, "librk.so"))

RK_OK, RK_EINVAL, RK_EWORKSPACE, RK_EHIP, RK_ENOCONV = 0, -1, -2, -3, -4
RK_FP64, RK_FP32 = 0, 1
RK_PREC_FP64, RK_PREC_MIXED = 0, 1
RK_BATCHED, RK_PER_STAGE = 0, 1
RK_METHOD_CROUT, RK_METHOD_COMPLEX = 0, 1
RK_OP_CALA, RK_OP_STAGE, RK_OP_BLOCKS, RK_OP_K, RK_OP_M, RK_OP_CBLOCKS = 0, 1, 2, 3, 4, 5
RK_MAX_Q, RK_MAX_DEGREE, RK_MAX_LEVELS = 9, 6, 16
RK_MAX_DEFORM = 0.1
RK_STATIC_SCRATCH_BYTES = 64 << 20

EXPORTS = ["rk_default_options", "rk_workspace_bytes", "rk_create", "rk_destroy", "rk_info",
           "rk_step", "rk_step_batch", "rk_apply_operator", "rk_vcycle", "rk_apply_preconditioner",
           "rk_deformed_geometry_bytes", "rk_deformed_geometry", "rk_deformed_apply", "rk_last_error",
           "rk_apply_operator_static", "rk_apply_operator_batch"]


class rk_mesh(C.Structure):
    _fields_ = [("n_cells", C.c_int32), ("length", C.c_double)]

    def __init__(self, n_cells=0, length=1.0):
        super().__init__(n_cells, length)


class rk_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("mode", C.c_int32), ("rtol", C.c_double),
                ("max_iter", C.c_int32), ("restart", C.c_int32), ("cheb_degree", C.c_int32),
                ("coarse_cheb_degree", C.c_int32), ("cheb_range", C.c_double),
                ("eig_safety", C.c_double), ("eig_iterations", C.c_int32),
                ("eig_max", C.POINTER(C.c_double)), ("timing", C.c_int32), ("method", C.c_int32),
                ("deform", C.c_double), ("autotune", C.c_int32), ("deform_mg", C.c_int32),
                ("vc_streams", C.c_int32), ("z_chunk", C.c_int32), ("tile_shape", C.c_int32),
                ("tail_nodes", C.c_int32)]


class rk_stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("vcycles", C.c_int32), ("rel_residual", C.c_double),
                ("t_rhs", C.c_double), ("t_vmult", C.c_double), ("t_basis", C.c_double),
                ("t_blocks", C.c_double), ("t_rest", C.c_double),
                ("block_iterations", C.c_int32 * RK_MAX_Q)]


class rk_info_t(C.Structure):
    _fields_ = [("N", C.c_int32), ("n_cells", C.c_int32), ("degree", C.c_int32), ("Q", C.c_int32),
                ("n_levels", C.c_int32), ("level_cells", C.c_int32 * RK_MAX_LEVELS),
                ("tau", C.c_double), ("h", C.c_double),
                ("A", C.c_double * 81), ("b", C.c_double * 9), ("c", C.c_double * 9),
                ("Ainv", C.c_double * 81), ("L", C.c_double * 81), ("S", C.c_double * 81),
                ("Sinv", C.c_double * 81), ("lambda_", C.c_double * 9),
                ("eig_max", C.c_double * RK_MAX_LEVELS), ("nodes", C.c_double * (RK_MAX_DEGREE + 1)),
                ("n_blocks", C.c_int32), ("n_pairs", C.c_int32),
                ("clam_re", C.c_double * RK_MAX_Q), ("clam_im", C.c_double * RK_MAX_Q),
                ("T", C.c_double * 81), ("U", C.c_double * 81),
                ("level_cz", C.c_int32 * RK_MAX_LEVELS), ("krylov_cz", C.c_int32),
                ("level_ts", C.c_int32 * RK_MAX_LEVELS), ("level_cz_store", C.c_int32 * RK_MAX_LEVELS),
                ("level_ts_store", C.c_int32 * RK_MAX_LEVELS), ("tail_level", C.c_int32)]


def load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2209_06700_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    lib.rk_default_options.argtypes = [C.POINTER(rk_options)]
    lib.rk_default_options.restype = None
    lib.rk_workspace_bytes.argtypes = [C.POINTER(rk_mesh), C.c_int, C.c_int, C.POINTER(rk_options),
                                       C.POINTER(C.c_size_t)]
    lib.rk_create.argtypes = [C.POINTER(rk_mesh), C.c_int, C.c_int, C.c_double, C.POINTER(rk_options),
                              vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.rk_destroy.argtypes = [vp]
    lib.rk_info.argtypes = [vp, C.POINTER(rk_info_t)]
    lib.rk_step.argtypes = [vp, C.c_double, vp, vp, C.POINTER(C.c_double), C.POINTER(rk_stats)]
    lib.rk_step_batch.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(C.c_double), C.POINTER(vp), C.POINTER(vp),
                                  C.POINTER(C.c_double), C.POINTER(rk_stats), C.POINTER(C.c_int), C.c_int]
    lib.rk_apply_operator.argtypes = [vp, C.c_int, C.c_int, vp, vp]
    lib.rk_vcycle.argtypes = [vp, C.c_int, vp, vp]
    lib.rk_apply_preconditioner.argtypes = [vp, vp, vp]
    lib.rk_deformed_geometry_bytes.argtypes = [C.POINTER(rk_mesh), C.c_int, C.c_int, C.POINTER(C.c_size_t)]
    lib.rk_deformed_geometry.argtypes = [C.POINTER(rk_mesh), C.c_int, C.c_double, C.c_int, vp, vp]
    lib.rk_deformed_apply.argtypes = [C.POINTER(rk_mesh), C.c_int, C.c_int, C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.c_int, vp, vp, vp, vp]
    lib.rk_apply_operator_static.argtypes = [C.POINTER(rk_mesh), C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                             vp, vp, vp]
    lib.rk_apply_operator_batch.argtypes = [C.POINTER(vp), C.c_int, C.c_int, C.c_int, C.POINTER(vp), C.POINTER(vp),
                                            vp]
    lib.rk_last_error.argtypes = [vp]
    lib.rk_last_error.restype = C.c_char_p
    for name in ("rk_workspace_bytes", "rk_create", "rk_destroy", "rk_info", "rk_step", "rk_step_batch",
                 "rk_apply_operator", "rk_vcycle", "rk_apply_preconditioner", "rk_deformed_geometry_bytes",
                 "rk_deformed_geometry", "rk_deformed_apply", "rk_apply_operator_static",
                 "rk_apply_operator_batch"):
        getattr(lib, name).restype = C.c_int
    return lib


LIB = load()
