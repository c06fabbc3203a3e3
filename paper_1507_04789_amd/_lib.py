"""ctypes declarations of the C ABI in include/mra.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmra.so")

MRA_OK, MRA_EINVAL, MRA_ENOTPD, MRA_ENOMEM, MRA_EHIP, MRA_ESTATE = 0, -1, -2, -3, -4, -5
MRA_COV_EXPONENTIAL, MRA_COV_MATERN32 = 0, 1
MRA_SYNC, MRA_PLAIN, MRA_GRAPH, MRA_NO_GRAD, MRA_CHECKPOINT, MRA_JOINT = 1, 2, 4, 8, 16, 32
SIM_MAX_DRAWS = 64   # MRA_SIM_MAX_DRAWS

# every symbol the header declares
SYMBOLS = ["mra_build", "mra_requirements", "mra_get_info", "mra_get_geometry", "mra_bind", "mra_loglik",
           "mra_loglik_grad", "mra_loglik_grad_data", "mra_predict", "mra_last_failure", "mra_profile", "mra_profile_read",
           "mra_status_string", "mra_destroy", "mra_autotune", "mra_get_tuning", "mra_set_tuning",
           "mra_loglik_grad_noalloc", "mra_gls", "mra_predict_cov", "mra_simulate"]
NOALLOC_MAX_BYTES = 256 << 20   # MRA_NOALLOC_MAX_BYTES


class Config(C.Structure):
    _fields_ = [("d", C.c_int32), ("M", C.c_int32), ("J", C.c_int32), ("r", C.c_int32),
                ("lo", C.c_double * 2), ("hi", C.c_double * 2), ("cov", C.c_int32),
                ("max_theta", C.c_int32), ("flags", C.c_uint32), ("chunks", C.c_int32),
                ("J_level", C.c_int32 * 12), ("r_level", C.c_int32 * 12), ("adaptive", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_pred", C.c_int64), ("n_rows_pad", C.c_int64), ("n_leaves", C.c_int64),
                ("n_regions", C.c_int64), ("max_leaf", C.c_int64), ("flops_loglik", C.c_double),
                ("flops_grad", C.c_double), ("flops_predict", C.c_double), ("n_sim_normals", C.c_int64)]


class PhaseStat(C.Structure):
    _fields_ = [("name", C.c_char * 24), ("level", C.c_int32), ("groups", C.c_int64), ("launches", C.c_int64),
                ("total_ms", C.c_double), ("flops", C.c_double)]


class MRAError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        super().__init__("%s: %s (%d)%s" % (where, _status_string(status), status, detail))


_lib = None


def lib() -> C.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmra.so is not built: run `python -m paper_1507_04789_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    L.mra_build.argtypes = [C.POINTER(Config), vp, i64, vp, i64, vp, C.POINTER(vp)]
    L.mra_requirements.argtypes = [vp, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]
    L.mra_get_info.argtypes = [vp, C.POINTER(Info)]
    L.mra_get_geometry.argtypes = [vp, vp, vp, vp]
    L.mra_bind.argtypes = [vp, vp, C.c_size_t, vp, C.c_size_t, vp]
    L.mra_loglik.argtypes = [vp, vp, vp, i32, vp, vp]
    L.mra_loglik_grad.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    L.mra_loglik_grad_data.argtypes = [vp, vp, i64, vp, i32, vp, vp, vp, vp]
    L.mra_loglik_grad_noalloc.argtypes = [vp, vp, vp, i32, vp, vp, vp]
    L.mra_gls.argtypes = [vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
    L.mra_predict_cov.argtypes = [vp, vp, vp, vp, vp, vp]
    L.mra_simulate.argtypes = [vp, vp, vp, vp, i64, i32, vp, vp]
    L.mra_predict.argtypes = [vp, vp, vp, vp, vp, vp]
    L.mra_last_failure.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i64), vp]
    L.mra_profile.argtypes = [vp, i32]
    L.mra_profile_read.argtypes = [vp, C.POINTER(PhaseStat), i32, C.POINTER(i32), vp]
    L.mra_status_string.argtypes = [i32]
    L.mra_status_string.restype = C.c_char_p
    L.mra_autotune.argtypes = [vp, vp, vp, i32, vp, vp, i32, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t), vp]
    L.mra_get_tuning.argtypes = [vp, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]
    L.mra_set_tuning.argtypes = [vp, C.c_char_p]
    L.mra_destroy.argtypes = [vp]
    L.mra_destroy.restype = None
    for name in SYMBOLS:
        if name not in ("mra_status_string", "mra_destroy"):
            getattr(L, name).restype = i32
    _lib = L
    return L


def _status_string(s: int) -> str:
    try:
        return lib().mra_status_string(s).decode()
    except Exception:  # pragma: no cover
        return "status"


def check(status: int, where: str, detail: str = "") -> None:
    if status != MRA_OK:
        raise MRAError(status, where, detail)
