"""ctypes binding of libkct.so (the C ABI in include/kct.h).

Argument marshalling only: every step of the reconstruction runs in the HIP
kernels behind these symbols.  Loading fails loudly if the library has not
been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkct.so")

# kct_status
KCT_OK = 0
STATUS_NAMES = {0: "KCT_OK", 1: "KCT_E_INVALID_ARG", 2: "KCT_E_GEOMETRY", 3: "KCT_E_DTYPE", 4: "KCT_E_OOM",
                5: "KCT_E_BUDGET", 6: "KCT_E_DEVICE", 7: "KCT_E_NONFINITE", 8: "KCT_E_STATE"}
# kct_dtype
KCT_F32, KCT_BF16, KCT_F16 = 0, 1, 2
# kct_solver
(KCT_CGLS, KCT_LSQR, KCT_LSMR, KCT_HYBRID_LSQR, KCT_IRN_TV_CGLS, KCT_AB_GMRES, KCT_BA_GMRES, KCT_SIRT,
 KCT_OS_SART, KCT_HYBRID_FLSQR_TV) = range(10)
# kct_backprojector
KCT_BP_MATCHED, KCT_BP_INTERP = 0, 1
# flags
KCT_FLAG_STOP_ON_RESIDUAL_INCREASE = 1
KCT_FLAG_EXPLICIT_RESIDUAL = 2
KCT_FLAG_X0_GIVEN = 4
KCT_HIST_COLS = 5
# kct_lambda_rule
KCT_LAMBDA_FIXED, KCT_LAMBDA_GCV, KCT_LAMBDA_DP = 0, 1, 2

EXPORTED = [
    "kct_plan_create", "kct_plan_destroy", "kct_plan_reserve", "kct_plan_check", "kct_plan_device_bytes",
    "kct_forward", "kct_forward_noalloc", "kct_backproject",
    "kct_backproject_interp",
    "kct_solve_workspace_bytes", "kct_solve", "kct_state_create", "kct_state_step", "kct_state_progress",
    "kct_state_resume",
    "kct_state_destroy", "kct_status_str", "kct_last_error", "kct_version",
]


class KctGeometry(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("vx", ctypes.c_double), ("vy", ctypes.c_double), ("vz", ctypes.c_double),
        ("ox", ctypes.c_double), ("oy", ctypes.c_double), ("oz", ctypes.c_double),
        ("nu", ctypes.c_int32), ("nv", ctypes.c_int32),
        ("du", ctypes.c_double), ("dv", ctypes.c_double),
        ("dso", ctypes.c_double), ("dsd", ctypes.c_double),
        ("n_angles", ctypes.c_int32),
        ("angles", ctypes.POINTER(ctypes.c_double)),
    ]


class KctSolveParams(ctypes.Structure):
    _fields_ = [
        ("solver", ctypes.c_int32), ("n_iter", ctypes.c_int32), ("lam", ctypes.c_double),
        ("tv_outer", ctypes.c_int32), ("tv_inner", ctypes.c_int32), ("tv_eps", ctypes.c_double),
        ("vec_dtype", ctypes.c_int32), ("lambda_rule", ctypes.c_int32), ("noise_level", ctypes.c_double),
        ("backprojector", ctypes.c_int32), ("n_subsets", ctypes.c_int32),
        ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32),
    ]


class KctError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{where}: {self.name}: {detail}")


_lib = None


def load(path: str = LIB_PATH):
    """Load libkct.so (once) and declare every exported signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2211_14212_amd.build` "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P, vp, i32, sz = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    st = ctypes.c_int
    sig = {
        "kct_plan_create": ([P(KctGeometry), ctypes.c_int, P(vp)], st),
        "kct_plan_destroy": ([vp], st),
        "kct_plan_reserve": ([vp, i32], st),
        "kct_plan_check": ([vp, vp], st),
        "kct_plan_device_bytes": ([vp, P(sz)], st),
        "kct_forward": ([vp, vp, i32, vp, i32, vp], st),
        "kct_forward_noalloc": ([vp, vp, i32, vp, i32, vp], st),
        "kct_backproject": ([vp, vp, i32, vp, i32, vp], st),
        "kct_backproject_interp": ([vp, vp, i32, vp, i32, vp], st),
        "kct_solve_workspace_bytes": ([vp, P(KctSolveParams), P(sz)], st),
        "kct_solve": ([vp, P(KctSolveParams), vp, vp, vp, sz, vp, vp], st),
        "kct_state_create": ([vp, P(KctSolveParams), vp, vp, vp, sz, vp, vp, P(vp)], st),
        "kct_state_step": ([vp, i32], st),
        "kct_state_progress": ([vp, P(i32), P(i32)], st),
        "kct_state_resume": ([vp, P(KctSolveParams), vp, vp, vp, sz, vp, vp, i32, P(vp)], st),
        "kct_state_destroy": ([vp], st),
        "kct_status_str": ([st], ctypes.c_char_p),
        "kct_last_error": ([], ctypes.c_char_p),
        "kct_version": ([], ctypes.c_char_p),
        "kct_debug_bwd_shape": ([vp, P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_int)], None),
        "kct_debug_fwd_shape_geom": ([P(KctGeometry), P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_int),
                                      P(ctypes.c_int)], ctypes.c_int),
        "kct_debug_bwd_shape_geom": ([P(KctGeometry), P(ctypes.c_int), P(ctypes.c_int), P(ctypes.c_int),
                                      P(ctypes.c_int)], ctypes.c_int),
        "kct_debug_bwd_mode_geom": ([P(KctGeometry), P(ctypes.c_int), P(ctypes.c_int)], ctypes.c_int),
        "kct_debug_bwd_mode": ([vp, P(ctypes.c_int), P(ctypes.c_int)], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def check(status: int, where: str):
    if status != KCT_OK:
        detail = load().kct_last_error().decode(errors="replace")
        raise KctError(status, where, detail)
