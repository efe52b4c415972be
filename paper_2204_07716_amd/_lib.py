"""ctypes binding of the C ABI declared in include/fkr.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfkr.so")

FKR_OK, FKR_WARN_ILLPOSED = 0, 1
FKR_E_ARG, FKR_E_DOMAIN, FKR_E_WORKSPACE = -1, -2, -3
FKR_E_DEVICE, FKR_E_UNSUPPORTED, FKR_E_STATE = -4, -5, -6
FKR_F32, FKR_F64 = 0, 1
FKR_KERNEL_ES, FKR_KERNEL_GAUSS = 0, 1
FKR_VAR_LOG, FKR_VAR_DIRECT = 0, 1
FKR_TP_SAME, FKR_TP_F32, FKR_TP_F64 = 0, 1, 2
FKR_SIG_SCALAR, FKR_SIG_GRID = 0, 1
FKR_REG = {"gauss": 0, "box": 1, "triangle": 2, "epanechnikov": 3, "biweight": 4, "triweight": 5}
FKR_MAX_H = 64
FKR_RESOLVE = 1e-3
FKR_STATIC_WORKSPACE_BYTES = 64 << 20

I64x3 = ctypes.c_int64 * 3
F64x3 = ctypes.c_double * 3


class PlanDesc(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("order", ctypes.c_int), ("M", I64x3), ("lo", F64x3),
                ("hi", F64x3), ("h_min", F64x3), ("h_max", F64x3), ("eps", ctypes.c_double),
                ("precision", ctypes.c_int), ("spread_kernel", ctypes.c_int),
                ("sigma", ctypes.c_double), ("n_max", ctypes.c_int64),
                ("max_weights", ctypes.c_int), ("max_h", ctypes.c_int),
                ("transform_precision", ctypes.c_int), ("reg_kernel", ctypes.c_int)]


class Geometry(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("order", ctypes.c_int), ("n_s", ctypes.c_int),
                ("n_t", ctypes.c_int), ("M", I64x3), ("L", I64x3), ("K", I64x3), ("Mr", I64x3),
                ("tile", I64x3), ("delta", F64x3), ("period", F64x3), ("w", ctypes.c_int),
                ("kparam", ctypes.c_double), ("n_tiles", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_size_t)]


class Diag(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("out_of_domain", ctypes.c_int64),
                ("ill_posed", ctypes.c_int64), ("n_jobs", ctypes.c_int64),
                ("max_tile_count", ctypes.c_int64)]


EXPORTS = ["fkr_plan_create", "fkr_plan_destroy", "fkr_plan_geometry", "fkr_workspace_size",
           "fkr_set_workspace", "fkr_set_points", "fkr_spectrum", "fkr_moments", "fkr_fit", "fkr_fit_noalloc",
           "fkr_interp", "fkr_dof", "fkr_cv", "fkr_gcv", "fkr_variance", "fkr_variance_full", "fkr_interval", "fkr_interval_full", "fkr_gcv_grad", "fkr_gcv_grad_full", "fkr_fit_full", "fkr_cv_full", "fkr_moments_full", "fkr_spline",
           "fkr_predict", "fkr_get_diagnostics",
           "fkr_status_string", "fkr_hlist", "fkr_select_bandwidth", "fkr_profile_enable",
           "fkr_profile_read", "fkr_batch_create", "fkr_batch_destroy", "fkr_batch_workspace_size",
           "fkr_batch_set_workspace", "fkr_batch_cv", "fkr_batch_tune", "fkr_batch_config"]

STAGES = ["sort", "weights", "spread", "fold", "fft_fwd", "expand", "fft_inv", "solve", "reduce"]

_lib = None


class FkrError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = load().fkr_status_string(status).decode() if _lib is not None else str(status)
        super().__init__(f"{where}: {msg} ({status})")


def load() -> ctypes.CDLL:
    """Load libfkr.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                          "(run __graft_entry__.build() or python paper_2204_07716_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, I64, D, U64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
    pD = ctypes.POINTER(ctypes.c_double)
    sig = {
        "fkr_plan_create": ([ctypes.POINTER(PlanDesc), ctypes.POINTER(P)], I),
        "fkr_plan_destroy": ([P], None),
        "fkr_plan_geometry": ([P, ctypes.POINTER(Geometry)], I),
        "fkr_workspace_size": ([P, ctypes.POINTER(ctypes.c_size_t)], I),
        "fkr_set_workspace": ([P, P, ctypes.c_size_t], I),
        "fkr_set_points": ([P, I64, P, I, P], I),
        "fkr_spectrum": ([P, I, P, I, P, P], I),
        "fkr_moments": ([P, I, pD, I, P, I, P, P, P], I),
        "fkr_fit": ([P, I, pD, I, I, P, I, P, P, P], I),
        "fkr_fit_noalloc": ([P, I64, P, I, I, pD, I, I, P, I, P, P, P], I),
        "fkr_interp": ([P, I, P, I64, P, I, P, P], I),
        "fkr_dof": ([P, I, pD, I, U64, P, I, P, P, P], I),
        "fkr_cv": ([P, I, pD, I, I, P, I, I, U64, P, P, P, P, P, P, P], I),
        "fkr_gcv": ([P, I, pD, I, I, P, I, I, P, P, P, P, P, P], I),
        "fkr_variance": ([P, pD, I, P, I, P, I, P, P, P, P], I),
        "fkr_variance_full": ([P, pD, I, P, I, P, I, P, P, P, P], I),
        "fkr_interval": ([P, pD, I, D, P, P, D, P, P, P, P], I),
        "fkr_interval_full": ([P, pD, I, D, P, P, D, P, P, P, P], I),
        "fkr_spline": ([P, I, P, P, P], I),
        "fkr_fit_full": ([P, I, pD, I, I, P, I, P, P, P], I),
        "fkr_cv_full": ([P, I, pD, I, I, P, I, I, U64, P, P, P, P, P, P, P], I),
        "fkr_moments_full": ([P, I, pD, I, P, I, P, P, P], I),
        "fkr_gcv_grad": ([P, pD, I, P, I, I, U64, P, P, P, P, P], I),
        "fkr_gcv_grad_full": ([P, pD, I, P, I, I, U64, P, P, P, P, P], I),
        "fkr_predict": ([P, I, P, I64, P, I, P, P], I),
        "fkr_get_diagnostics": ([P, ctypes.POINTER(Diag)], I),
        "fkr_status_string": ([I], ctypes.c_char_p),
        "fkr_hlist": ([I, D, D, I, pD], I),
        "fkr_select_bandwidth": ([I, pD, D, ctypes.POINTER(I)], I),
        "fkr_profile_enable": ([P, I], I),
        "fkr_profile_read": ([P, I, pD, ctypes.POINTER(I64)], I),
        "fkr_batch_create": ([ctypes.POINTER(PlanDesc), I, ctypes.POINTER(P)], I),
        "fkr_batch_destroy": ([P], None),
        "fkr_batch_workspace_size": ([P, ctypes.POINTER(ctypes.c_size_t)], I),
        "fkr_batch_set_workspace": ([P, P, ctypes.c_size_t], I),
        "fkr_batch_cv": ([P, I, P, P, I, I, pD, I, I, P, I, I, U64, P, P, P, P, P, P], I),
        "fkr_batch_tune": ([P, I, P, P, I, I, pD, I, I, P, I, I, U64, I, ctypes.POINTER(I),
                            ctypes.POINTER(I64), pD, P], I),
        "fkr_batch_config": ([P, I, I64], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _ = D
    _lib = lib
    return lib


def check(status: int, where: str, allow=(FKR_OK,)) -> int:
    if status not in allow:
        raise FkrError(status, where)
    return status
