"""ctypes declarations of libens.so (include/ens.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libens.so")

ENS_OK, ENS_EINVAL, ENS_ENOMEM, ENS_EDEVICE, ENS_EUNSUPPORTED = 0, -1, -2, -3, -4
SYSTEMS = {"linear": 0, "lorenz": 1, "robertson": 2, "gbm4": 3, "orego": 4, "hires": 5,
           "pollu": 6, "crn": 7}
ALGS = {"tsit5": 1, "rodas4": 2, "em": 3, "ros23": 4, "siea": 5, "rodas5p": 6}
OPTS = {"precision": 1, "form": 2, "block": 3, "dt": 4, "seed": 5, "h0": 6,
        "maxiters": 7, "tspan_broadcast": 8, "refill": 9, "grid": 10, "tpl": 11,
        "mlp_tile": 12, "save_mode": 13, "stage_saves": 14, "autotune_cached": 15}
PTRS = {"status": 1, "stats": 2}
MAX_TRAJ = (1 << 32) - (1 << 11)  # ENS_MAX_TRAJ
STATIC_MAX_QUERIES = 1 << 20      # ENS_STATIC_MAX_QUERIES

# Every symbol include/ens.h declares.
EXPORTS = ("ens_create", "ens_destroy", "ens_last_error", "ens_set_option",
           "ens_get_option", "ens_set_ptr", "ens_system_dims", "ens_solve",
           "ens_autotune", "ens_set_autotune_file", "ens_solve_mixed", "ens_philox_fill", "ens_surrogate_create", "ens_surrogate_destroy",
           "ens_surrogate_copy", "ens_surrogate_get_step", "ens_surrogate_set_step",
           "ens_surrogate_fit_norm", "ens_surrogate_train_step", "ens_surrogate_train",
           "ens_surrogate_predict", "ens_surrogate_solve", "ens_surrogate_save",
           "ens_surrogate_load", "ens_surrogate_solve_static")
SURR_BUFFERS = {"master": 1, "weights_bf16": 2, "grad": 3, "adam_m": 4, "adam_v": 5, "norm": 6}
SURR_NPARAM = 145200
SURR_MAX_BATCH = 1 << 28  # ENS_SURR_MAX_BATCH


class EnsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"ens error {code}: {msg}")
        self.code = code


class Group(ctypes.Structure):
    """struct ens_group of include/ens.h."""
    _fields_ = [("system_id", ctypes.c_int), ("tspan_broadcast", ctypes.c_int),
                ("n_traj", ctypes.c_int64), ("params", ctypes.c_void_p),
                ("u0", ctypes.c_void_p), ("tspan", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("stats", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libens.so.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2304_06835_amd.build` "
            "(the HIP library is the only implementation)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl, c_int = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    L.ens_create.argtypes = [ctypes.POINTER(vp), c_int]
    L.ens_destroy.argtypes = [vp]
    L.ens_last_error.argtypes = [vp]
    L.ens_last_error.restype = ctypes.c_char_p
    L.ens_set_option.argtypes = [vp, c_int, dbl]
    L.ens_get_option.argtypes = [vp, c_int, dp]
    L.ens_set_ptr.argtypes = [vp, c_int, vp]
    L.ens_system_dims.argtypes = [c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]
    L.ens_solve.argtypes = [vp, c_int, i64, vp, vp, vp, c_int, dbl, dbl, dp, c_int, vp, vp]
    L.ens_autotune.argtypes = [vp, c_int, i64, vp, vp, vp, c_int, dbl, dbl, dp, c_int, vp, vp,
                               dp]
    L.ens_set_autotune_file.argtypes = [vp, ctypes.c_char_p]
    L.ens_solve_mixed.argtypes = [vp, c_int, ctypes.POINTER(Group), c_int, dbl, dbl, dp, c_int,
                                  vp]
    L.ens_philox_fill.argtypes = [vp, ctypes.c_uint64, i64, ctypes.c_uint32, vp, vp]
    u64 = ctypes.c_uint64
    L.ens_surrogate_create.argtypes = [vp, u64, ctypes.POINTER(vp)]
    L.ens_surrogate_destroy.argtypes = [vp]
    L.ens_surrogate_copy.argtypes = [vp, vp, c_int, vp, c_int, vp]
    L.ens_surrogate_save.argtypes = [vp, vp, ctypes.c_char_p]
    L.ens_surrogate_load.argtypes = [vp, vp, ctypes.c_char_p]
    L.ens_surrogate_get_step.argtypes = [vp, ctypes.POINTER(i64)]
    L.ens_surrogate_set_step.argtypes = [vp, i64]
    L.ens_surrogate_fit_norm.argtypes = [vp, vp, vp, vp, vp, i64, vp]
    L.ens_surrogate_train_step.argtypes = [vp, vp, vp, vp, vp, i64, i64, i64, u64, u64, dbl, vp,
                                           vp]
    L.ens_surrogate_train.argtypes = [vp, vp, vp, vp, vp, i64, c_int, i64, dbl, dbl, u64, vp, vp]
    L.ens_surrogate_predict.argtypes = [vp, vp, vp, vp, i64, vp, vp]
    L.ens_surrogate_solve.argtypes = [vp, vp, vp, vp, vp, dbl, dbl, dp, c_int, i64, dbl, dbl, u64,
                                      vp, vp, vp, vp]
    L.ens_surrogate_solve_static.argtypes = L.ens_surrogate_solve.argtypes
    for name in EXPORTS:
        getattr(L, name).restype = getattr(L, name).restype or c_int
    L.ens_last_error.restype = ctypes.c_char_p
    _lib = L
    return L
