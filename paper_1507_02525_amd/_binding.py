"""ctypes binding of the C ABI in include/mrdft.h and include/mrdft_tune.h
(argument marshalling only).

Every computation runs in the HIP library ``libmrdft.so``; there is no CPU or
PyTorch fallback.  If the library is missing or cannot be loaded, importing a
compute entry point raises ``RuntimeError``.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrdft.so")

MRDFT_OK = 0
MRDFT_E_INVALID_ARG = 1
MRDFT_E_UNSUPPORTED = 2
MRDFT_E_ALLOC = 3
MRDFT_E_HIP = 4
MRDFT_C64 = 0
MRDFT_R32 = 1
MRDFT_MAX_ORDER = 28
MRDFT_FLAG_NONE = 0
MRDFT_FLAG_TUNE = 1
MRDFT_FLAG_GRAPH = 2
MRDFT_FLAG_HALF = 4
ORDERS = ("tiles_first", "rows_first", "interleaved", "blocks")
MRDFT_SCHED_SERIAL = 0x100
MRDFT_SCHED_AFTER = 0x200
KERNEL_KINDS = ("tile_fwd", "pass_fwd", "tile_adj", "pass_adj", "fused_fwd", "loss")

# Every symbol the header declares, with (restype, argtypes).
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i64p = ctypes.POINTER(ctypes.c_int64)
SIGNATURES = {
    "mrdft_plan_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, _i64, _i64p, ctypes.c_int,
                                         ctypes.c_uint, _vp]),
    "mrdft_plan_create_levels": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, _i64, _i64p, ctypes.c_int,
                                                ctypes.c_uint, ctypes.c_int, ctypes.c_int, _vp]),
    "mrdft_plan_output_offsets": (ctypes.c_int, [_vp, _i64p]),
    "mrdft_plan_sizes": (ctypes.c_int, [_vp, _i64p, _i64p]),
    "mrdft_plan_schedule": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_int)]),
    "mrdft_plan_set_schedule": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]),
    "mrdft_forward": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "mrdft_adjoint": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "mrdft_spectral_loss_fwd": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "mrdft_spectral_loss_bwd": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mrdft_spectral_loss_fwd_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "mrdft_plan_set_profiling": (ctypes.c_int, [_vp, ctypes.c_int]),
    "mrdft_plan_read_profile": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), _i64p]),
    "mrdft_plan_destroy": (ctypes.c_int, [_vp]),
    "mrdft_plan2d_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int, _i64, ctypes.c_int, _vp]),
    "mrdft_plan2d_sizes": (ctypes.c_int, [_vp, _i64p, _i64p]),
    "mrdft_forward2d": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "mrdft_adjoint2d": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "mrdft_plan2d_destroy": (ctypes.c_int, [_vp]),
    "mrdft_last_error": (ctypes.c_char_p, []),
    "mrdft_live_device_allocations": (ctypes.c_int64, []),
    "mrdft_tune_cache_lookup": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int),
                                               ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                               ctypes.POINTER(ctypes.c_int)]),
    "mrdft_tune_cache_store": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_char_p, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_int, ctypes.c_int]),
}

_lib = None


class MrdftError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("mrdft error %d: %s" % (status, msg))
        self.status = status


def lib():
    """Load libmrdft.so (once).  Raises RuntimeError if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmrdft.so is not built (run __graft_entry__.build() or "
                               "python paper_1507_02525_amd/build.py); there is no fallback")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(status: int):
    if status != MRDFT_OK:
        msg = lib().mrdft_last_error()
        raise MrdftError(status, msg.decode() if msg else "")


def last_error() -> str:
    msg = lib().mrdft_last_error()
    return msg.decode() if msg else ""
