"""ctypes binding of libsttsv.so (the C ABI in include/sttsv.h).

Argument marshalling only: every step of STTSV and of the solver runs in the
HIP library.  There is no CPU fallback -- if the library is missing the
import of any entry point raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsttsv.so")

STTSV_OK = 0
STTSV_EINVAL = -1
STTSV_ENOMEM = -2
STTSV_EDISCONNECTED = -3
STTSV_ENOTCONV = -4
STTSV_ENUMERIC = -5
STTSV_EHIP = -6
STTSV_ENOTSUP = -7
STTSV_MAX_ORDER = 64
MPNN_NPARAM = 17665
MPNN_HIDDEN = 64
FLAG_GENERIC_ONLY = 1
FLAG_ONE_STREAM = 2
FLAG_PREFIX_REUSE = 4

PREC = {"fp64": 0, "fp32": 1}
SCHEDULE = {"fp64": 0, "fp32_fp64": 1}

Q_PERM, Q_MEM, Q_BUCKET_K, Q_BUCKET_M, Q_TPTR, Q_TSLOT, Q_WEIGHTS, Q_SCALE_EXP, Q_BUCKET_R, Q_BUCKET_RUNS, \
    Q_CONTRIB, Q_BUCKET_LANES, Q_CCSS_LEVEL_N, Q_CCSS_VERT, Q_CCSS_PARENT, Q_CCSS_LEAF, Q_BUCKET_STACK = range(17)

# every symbol the header declares
EXPORTS = ["sttsv_plan", "sttsv_apply", "sttsv_apply_prec", "sttsv_apply_timed", "sttsv_apply_naive",
           "sttsv_contract", "sttsv_contract_noalloc", "zeigvec_sshopm", "sttsv_ccss_build", "sttsv_apply_ccss",
           "sttsv_cp_objective_grad", "sym_cp_descent",
           "heigvec_solve", "heigvec_solve_ex", "sttsv_plan_batch", "heigvec_solve_batch",
           "sttsv_plan_graph_info", "sttsv_plan_autotune",
           "sttsv_mpnn_graph", "sttsv_mpnn_graph_destroy", "sttsv_mpnn_create", "sttsv_mpnn_destroy",
           "sttsv_mpnn_params", "sttsv_mpnn_forward", "sttsv_mpnn_loss_grad", "sttsv_mpnn_adam",
           "sttsv_mpnn_warm_start", "sttsv_mpnn_query",
           "sttsv_plan_get_info", "sttsv_plan_query", "sttsv_plan_destroy", "sttsv_strerror"]


class SttsvOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("edge_weights", ctypes.c_void_p)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("shift", ctypes.c_double), ("switch_tol", ctypes.c_double)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("iters_fp32", ctypes.c_int32),
                ("iters_fp64", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("lambda_min", ctypes.c_double), ("lambda_max", ctypes.c_double),
                ("criterion", ctypes.c_double)]


class ZeigInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("lambda_", ctypes.c_double), ("residual", ctypes.c_double)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("nnz", ctypes.c_int64), ("n", ctypes.c_int32),
                ("r", ctypes.c_int32), ("nbuckets", ctypes.c_int32), ("connected", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64), ("graphs", ctypes.c_int32), ("lanes", ctypes.c_int32)]


class CcssInfo(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("nodes", ctypes.c_int64), ("roots", ctypes.c_int64),
                ("convolutions", ctypes.c_int64), ("leaves", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("build_ms", ctypes.c_double)]


class CpInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("halvings", ctypes.c_int32), ("f0", ctypes.c_double),
                ("f", ctypes.c_double), ("norm2", ctypes.c_double)]


CP_MAX_R = 32


class GraphDesc(ctypes.Structure):
    _fields_ = [("eptr", ctypes.c_void_p), ("eidx", ctypes.c_void_p), ("m", ctypes.c_int64),
                ("n", ctypes.c_int32), ("r", ctypes.c_int32), ("w", ctypes.c_void_p)]


class GraphInfo(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int32), ("r", ctypes.c_int32),
                ("voff", ctypes.c_int32), ("connected", ctypes.c_int32)]


class SttsvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


_lib = None


def load(path=None):
    """Load libsttsv.so (built in-tree by ``paper_2311_08595_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError("libsttsv.so not built: run python -m paper_2311_08595_amd.build "
                           "(no CPU fallback exists)")
    # torch first: the library must bind to the HIP runtime torch loads (torch
    # ships its own; loaded before it, the library would pull in another one,
    # which torch would then share)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.sttsv_plan.argtypes = [P, P, i64, i32, i32, ctypes.POINTER(SttsvOpts), ctypes.POINTER(P)]
    lib.sttsv_apply.argtypes = [P, P, P]
    lib.sttsv_apply_prec.argtypes = [P, P, P, i32]
    lib.sttsv_apply_naive.argtypes = [P, P, P]
    lib.sttsv_contract.argtypes = [P, P, P, P]
    lib.sttsv_contract_noalloc.argtypes = [P, P, P, P]
    lib.sttsv_ccss_build.argtypes = [P, ctypes.POINTER(CcssInfo)]
    lib.sttsv_apply_ccss.argtypes = [P, P, P]
    lib.sttsv_cp_objective_grad.argtypes = [P, i32, P, P, P, P, P]
    lib.sym_cp_descent.argtypes = [P, i32, P, P, i32, f64, ctypes.POINTER(CpInfo)]
    lib.zeigvec_sshopm.argtypes = [P, P, ctypes.c_double, ctypes.c_double, i32, P, P]
    lib.sttsv_apply_timed.argtypes = [P, P, P, i32, i32, P, P, P, P, P]
    lib.heigvec_solve.argtypes = [P, P, f64, P, ctypes.POINTER(SolveInfo)]
    lib.heigvec_solve_ex.argtypes = [P, P, f64, ctypes.POINTER(SolveOpts), P, ctypes.POINTER(SolveInfo)]
    f32 = ctypes.c_float
    lib.sttsv_mpnn_graph.argtypes = [P, P, i64, i32, i32, ctypes.POINTER(P)]
    lib.sttsv_mpnn_graph_destroy.argtypes = [P]
    lib.sttsv_mpnn_create.argtypes = [P, ctypes.POINTER(P)]
    lib.sttsv_mpnn_destroy.argtypes = [P]
    lib.sttsv_mpnn_params.argtypes = [P, P, P]
    lib.sttsv_mpnn_forward.argtypes = [P, P, P]
    lib.sttsv_mpnn_loss_grad.argtypes = [P, P, P, ctypes.POINTER(f32)]
    lib.sttsv_mpnn_adam.argtypes = [P, f32, f32, f32, f32]
    lib.sttsv_mpnn_warm_start.argtypes = [P, P, P]
    lib.sttsv_mpnn_query.argtypes = [P, P, i32, P, i64]
    lib.sttsv_plan_autotune.argtypes = [P, P, i32, ctypes.c_char_p, ctypes.POINTER(i32)]
    lib.sttsv_plan_batch.argtypes = [i32, P, ctypes.POINTER(SttsvOpts), ctypes.POINTER(P)]
    lib.heigvec_solve_batch.argtypes = [P, P, f64, ctypes.POINTER(SolveOpts), P, P]
    lib.sttsv_plan_graph_info.argtypes = [P, i32, ctypes.POINTER(GraphInfo)]
    lib.sttsv_plan_get_info.argtypes = [P, ctypes.POINTER(PlanInfo)]
    lib.sttsv_plan_query.argtypes = [P, i32, P, i64]
    lib.sttsv_plan_destroy.argtypes = [P]
    lib.sttsv_strerror.argtypes = [ctypes.c_int]
    lib.sttsv_strerror.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "sttsv_strerror":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def check(code):
    if code != STTSV_OK:
        raise SttsvError(code, load().sttsv_strerror(code).decode())
    return code
