"""ctypes declarations of libngd's C ABI (include/ngd.h). Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libngd.so")

NGD_OK, NGD_ERR_INVALID, NGD_ERR_OOM, NGD_ERR_NOT_PD, NGD_ERR_BREAKDOWN, NGD_ERR_NOT_CONVERGED, NGD_ERR_HIP = range(7)
NGD_F64, NGD_F32, NGD_BF16 = 0, 1, 2
NGD_PDE_POISSON, NGD_PDE_HEAT, NGD_PDE_NAVIER_STOKES = 0, 1, 2
NGD_NOALLOC_SCRATCH_BYTES = 40 * 1024 * 1024

STATUS_NAMES = {0: "NGD_OK", 1: "NGD_ERR_INVALID", 2: "NGD_ERR_OOM", 3: "NGD_ERR_NOT_PD", 4: "NGD_ERR_BREAKDOWN",
                5: "NGD_ERR_NOT_CONVERGED", 6: "NGD_ERR_HIP"}


class ProblemDesc(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("widths", C.POINTER(C.c_int32)), ("pde", C.c_int32),
                ("dtype", C.c_int32), ("n_rows", C.c_int64), ("X", C.c_void_p), ("w", C.c_void_p),
                ("f", C.c_void_p), ("g", C.c_void_p), ("row_kind", C.c_void_p), ("max_ell", C.c_int32),
                ("viscosity", C.c_double)]


class Operator(C.Structure):
    _fields_ = [("theta", C.c_void_p), ("J", C.c_void_p), ("ldJ", C.c_int64)]


class NystromInfo(C.Structure):
    _fields_ = [("nu", C.c_double), ("lam1", C.c_double), ("lam_ell", C.c_double), ("rank_z", C.c_int32),
                ("rank", C.c_int32)]


class Precond(C.Structure):
    _fields_ = [("U", C.c_void_p), ("ldU", C.c_int64), ("lam_hat", C.c_void_p), ("ell", C.c_int64)]


class PcgInfo(C.Structure):
    _fields_ = [("iters", C.c_int64), ("rel_res", C.c_double), ("converged", C.c_int32), ("breakdown", C.c_int32)]


# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "ngd_problem_create": (C.c_int, [C.POINTER(ProblemDesc), C.POINTER(C.c_void_p)]),
    "ngd_problem_destroy": (C.c_int, [C.c_void_p]),
    "ngd_num_params": (C.c_int64, [C.c_void_p]),
    "ngd_recommended_ld": (C.c_int64, [C.c_void_p]),
    "ngd_workspace_bytes": (C.c_int64, [C.c_void_p]),
    "ngd_last_error": (C.c_char_p, []),
    "ngd_residual_jacobian": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                        C.c_void_p, C.c_void_p]),
    "ngd_gramian_matvec": (C.c_int, [C.c_void_p, C.POINTER(Operator), C.c_void_p, C.c_int64, C.c_int64, C.c_double,
                                     C.c_void_p, C.c_int64, C.c_void_p]),
    "ngd_gramian_matvec_noalloc": (C.c_int, [C.c_int32, C.c_void_p, C.c_int64, C.c_int64, C.c_int64, C.c_void_p,
                                             C.c_double, C.c_void_p, C.c_void_p]),
    "ngd_jvp": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_int64,
                          C.c_void_p]),
    "ngd_vjp": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "ngd_gaussian_omega": (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint64, C.c_int64, C.c_void_p, C.c_int64,
                                     C.c_void_p]),
    "ngd_nystrom_sketch": (C.c_int, [C.c_void_p, C.POINTER(Operator), C.c_int64, C.c_uint64, C.c_uint64, C.c_void_p,
                                     C.c_int64, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p,
                                     C.POINTER(NystromInfo), C.c_void_p]),
    "ngd_pcg_solve": (C.c_int, [C.c_void_p, C.POINTER(Operator), C.c_void_p, C.c_double, C.POINTER(Precond),
                                C.c_double, C.c_int64, C.c_void_p, C.POINTER(PcgInfo), C.c_void_p]),
    "ngd_pcg_solve_damped": (C.c_int, [C.c_void_p, C.POINTER(Operator), C.c_void_p, C.c_double, C.c_double,
                                       C.c_void_p, C.POINTER(Precond), C.c_double, C.c_int64, C.c_void_p,
                                       C.POINTER(PcgInfo), C.POINTER(C.c_double), C.c_void_p]),
    "ngd_power_lambda_max": (C.c_int, [C.c_void_p, C.POINTER(Operator), C.c_void_p, C.c_int32,
                                       C.POINTER(C.c_double), C.c_void_p, C.c_void_p]),
    "ngd_damping": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_void_p,
                              C.POINTER(C.c_double), C.c_void_p]),
    "ngd_next_rank": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_int64, C.c_int64, C.c_int64,
                                C.POINTER(C.c_int64), C.c_void_p]),
    "ngd_lm_damping": (C.c_int, [C.c_void_p, C.POINTER(Operator), C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                                 C.c_double, C.c_double, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.c_void_p]),
    "ngd_line_search": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_int32,
                                  C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p]),
    "ngd_nystrom_sketch_columns": (C.c_int, [C.c_void_p, C.POINTER(Operator), C.c_int64, C.c_void_p, C.c_int32,
                                             C.c_void_p, C.c_int64, C.c_void_p, C.POINTER(NystromInfo), C.c_void_p]),
    "ngd_gramian_diagonal": (C.c_int, [C.c_void_p, C.POINTER(Operator), C.c_void_p, C.c_void_p]),
    "ngd_sample_pivots": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_uint64, C.c_uint64, C.c_uint32, C.c_int32,
                                    C.c_void_p, C.c_void_p, C.c_void_p]),
    "ngd_direct_solve": (C.c_int, [C.c_void_p, C.POINTER(Operator), C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]),
    "ngd_rpcholesky": (C.c_int, [C.c_void_p, C.POINTER(Operator), C.c_void_p, C.c_int64, C.c_int32, C.c_uint64,
                                 C.c_uint64, C.c_double, C.c_void_p, C.c_int64, C.POINTER(C.c_int64),
                                 C.POINTER(C.c_double), C.c_void_p]),
    "ngd_rpchol_precond": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p,
                                     C.c_void_p]),
    "ngd_rpchol_precond_woodbury": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_double, C.c_void_p,
                                              C.c_int64, C.c_void_p, C.c_void_p]),
    "ngd_solution_error": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p]),
    "ngd_batch_create": (C.c_int, [C.POINTER(ProblemDesc), C.c_int32, C.POINTER(C.c_void_p)]),
    "ngd_batch_destroy": (C.c_int, [C.c_void_p]),
    "ngd_batch_size": (C.c_int32, [C.c_void_p]),
    "ngd_batch_problem": (C.c_void_p, [C.c_void_p, C.c_int32]),
    "ngd_batch_residual_jacobian": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                              C.POINTER(C.c_void_p), C.POINTER(C.c_int64), C.POINTER(C.c_void_p),
                                              C.POINTER(C.c_void_p), C.c_void_p]),
    "ngd_batch_pcg_solve": (C.c_int, [C.c_void_p, C.POINTER(Operator), C.POINTER(C.c_void_p), C.POINTER(C.c_double),
                                      C.POINTER(Precond), C.c_double, C.c_int64, C.POINTER(C.c_void_p),
                                      C.POINTER(PcgInfo), C.c_void_p]),
    "ngd_batch_pcg_solve_damped": (C.c_int, [C.c_void_p, C.POINTER(Operator), C.POINTER(C.c_void_p), C.c_double,
                                             C.c_double, C.POINTER(C.c_void_p), C.POINTER(Precond), C.c_double,
                                             C.c_int64, C.POINTER(C.c_void_p), C.POINTER(PcgInfo),
                                             C.POINTER(C.c_double), C.c_void_p]),
    "ngd_batch_nystrom_sketch": (C.c_int, [C.c_void_p, C.POINTER(Operator), C.POINTER(C.c_int64), C.c_uint64,
                                           C.c_uint64, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                           C.POINTER(C.c_void_p), C.c_void_p]),
    "ngd_batch_matvec_time": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.c_void_p]),
    "ngd_batch_line_search": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                        C.POINTER(C.c_void_p), C.POINTER(C.c_double), C.c_double, C.c_int32,
                                        C.POINTER(C.c_void_p), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.c_void_p]),
    "ngd_timing_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "ngd_timing_enable_mask": (C.c_int, [C.c_void_p, C.c_uint32]),
    "ngd_timing_read": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
}

TIMERS = {"matvec_rows": 0, "residual_jacobian": 1, "sketch_z": 2, "sketch_w": 3, "core": 4, "precond": 5,
          "sketch_prep": 6}

_lib = None


class NgdError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load(path: str = LIB_PATH):
    """Load libngd.so and declare its signatures. Raises if the library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2505_11638_amd.build` "
                          "(the GPU path has no fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, where: str, allow=()):
    if status != NGD_OK and status not in allow:
        raise NgdError(status, where, load().ngd_last_error().decode())
    return status
