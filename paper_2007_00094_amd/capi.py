"""ctypes binding of the C-ABI declared in include/idp.h (same names).

Argument marshalling only: every step of the method runs in the HIP
library.  Loading fails loudly when libidp.so has not been built; there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libidp.so")

IDP_OK = 0
IDP_WARN_CFL = 1
IDP_EINVAL = -1
IDP_EMESH = -2
IDP_ENOMEM = -3
IDP_EHIP = -4
IDP_ESTATE = -5
IDP_EDT = -6
IDP_ENOTSUP = -7
IDP_EWAIT = -8
IDP_ESCRATCH = -9
IDP_FLAG_ASYNC = 1
IDP_FLAG_NO_STAGING = 2
IDP_FLAG_RENUMBER = 4
IDP_FLAG_SPLIT_P = 8
IDP_SCHED_LAUNCHES = 1
IDP_SCHED_PERSISTENT = 2

IDP_DBG_D = 0
IDP_DBG_ALPHA = 1
IDP_DBG_R = 2
IDP_DBG_UL = 3
IDP_DBG_BOUNDS = 4
IDP_DBG_L1 = 5
IDP_DBG_L2 = 6
IDP_DBG_UPASS = 7
IDP_DBG_TAUI = 8
IDP_DBG_P = 9
IDP_DBG_L1RAW = 10
IDP_DBG_L2RAW = 11


class idp_params(C.Structure):
    _fields_ = [("dim", C.c_int), ("gamma", C.c_double), ("cfl", C.c_double),
                ("limiter_passes", C.c_int), ("newton_max_iter", C.c_int),
                ("newton_tol", C.c_double), ("relax_bounds", C.c_int),
                ("flags", C.c_int), ("sell_sigma", C.c_int)]


class idp_schedule(C.Structure):
    _fields_ = [("kind", C.c_int), ("tile", C.c_int)]


_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)
_u8p = C.POINTER(C.c_uint8)
_vp = C.c_void_p

# name -> (restype, argtypes)
SIGNATURES = {
    "idp_default_params": (C.c_int, [C.POINTER(idp_params), C.c_int]),
    "idp_create": (C.c_int, [C.POINTER(_vp), C.POINTER(idp_params), C.c_int64, _dp,
                             C.c_int64, _i64p, _u8p, _vp]),
    "idp_max_dt": (C.c_int, [_vp, _vp, _dp]),
    "idp_step": (C.c_int, [_vp, _vp, C.c_double, _dp]),
    "idp_euler_stage": (C.c_int, [_vp, _vp, C.c_double, _vp]),
    "idp_get_status": (C.c_int, [_vp]),
    "idp_info": (C.c_int, [_vp, _i64p, _i64p, C.POINTER(C.c_size_t)]),
    "idp_export_matrices": (C.c_int, [_vp, _i64p, _i32p, _dp, _dp, _dp]),
    "idp_debug_export": (C.c_int, [_vp, C.c_int, _dp]),
    "idp_set_timing": (C.c_int, [_vp, C.c_int]),
    "idp_kernel_times": (C.c_int, [_vp, C.c_int, C.POINTER(C.c_char_p), _dp, _i64p]),
    "idp_device_math": (C.c_int, [_vp, C.c_int, C.c_int64, _vp, _vp, _vp]),
    "idp_create_batch": (C.c_int, [C.POINTER(_vp), C.POINTER(idp_params), C.c_int, _i64p,
                                   C.POINTER(_dp), _i64p, C.POINTER(_i64p), C.POINTER(_u8p),
                                   _vp]),
    "idp_batch_info": (C.c_int, [_vp, C.POINTER(C.c_int), _i64p]),
    "idp_batch_steps": (C.c_int, [_vp, _vp, C.c_int, _dp, _dp, C.POINTER(idp_schedule)]),
    "idp_batch_steps_noalloc": (C.c_int, [_vp, _vp, C.c_int, _dp, _dp]),
    "idp_batch_max_dt": (C.c_int, [_vp, _vp, _dp]),
    "idp_batch_tune": (C.c_int, [_vp, _vp, C.c_int, C.POINTER(idp_schedule), _dp,
                                 C.POINTER(C.c_int)]),
    "idp_euler_stage_vjp": (C.c_int, [_vp, _vp, C.c_double, _vp, _vp]),
    "idp_step_vjp": (C.c_int, [_vp, _vp, C.c_double, _vp, _vp]),
    "idp_forward_checkpoints": (C.c_int, [_vp, _vp, C.c_int, _dp, C.c_int]),
    "idp_trace_decisions": (C.c_int, [_vp, _vp, C.c_int, _dp, _vp, C.c_int64, _i64p]),
    "idp_adjoint_checkpoints": (C.c_int, [_vp, C.c_int, _dp, C.c_int, _vp, _vp]),
    "idp_debug_adjoint": (C.c_int, [_vp, C.c_int, _dp]),
    "idp_strerror": (C.c_char_p, [C.c_int]),
    "idp_destroy": (None, [_vp]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().idp_strerror(int(code)).decode()


class IdpError(RuntimeError):
    def __init__(self, where: str, code: int):
        super().__init__(f"{where}: {strerror(code)} ({code})")
        self.code = code


def check(where: str, code: int) -> int:
    if code < 0:
        raise IdpError(where, code)
    return code
