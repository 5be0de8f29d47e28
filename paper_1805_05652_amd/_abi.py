"""ctypes declarations of the tfstat C ABI (include/tfstat.h).

Argument marshalling only: every step of the map runs in libtfstat.so.  The
library must have been built (``python -m paper_1805_05652_amd.build`` or
``__graft_entry__.build()``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

from .build import library_path

OK = 0
E_INVAL, E_GRID, E_NOMEM, E_DEVICE, E_BUSY, E_NOTFOUND, E_CANCELLED = -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {
    0: "OK", -1: "E_INVAL", -2: "E_GRID", -3: "E_NOMEM", -4: "E_DEVICE", -5: "E_BUSY",
    -6: "E_NOTFOUND", -7: "E_CANCELLED",
}

WIN_RECT, WIN_EXP, WIN_SHAPE = 0, 1, 2
PREC_FP64, PREC_FP32, PREC_BF16X3, PREC_RECUR64, PREC_F16X3 = 0, 1, 2, 3, 4

K_UPLOAD, K_WEIGHTS, K_EXP, K_SCAN, K_RECT, K_MERGE, K_MFMA, K_ABC, K_RECUR = range(9)
KERNEL_NAMES = ["upload", "weights", "exp", "scan", "rect", "merge", "mfma", "abc", "recur"]


class Window(ctypes.Structure):
    _fields_ = [
        ("type", ctypes.c_int32),
        ("n_t0", ctypes.c_int32),
        ("n_tau", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("t0_min", ctypes.c_int64),
        ("dt0", ctypes.c_int64),
        ("tau_min", ctypes.c_int64),
        ("dtau", ctypes.c_int64),
        ("t0_list", ctypes.c_void_p),
        ("tau_list", ctypes.c_void_p),
        ("shape", ctypes.c_void_p),
        ("n_shape", ctypes.c_int32),
        ("support_num", ctypes.c_int32),
        ("support_den", ctypes.c_int32),
        ("reserved2", ctypes.c_int32),
    ]


class AtomsDesc(ctypes.Structure):
    _fields_ = [
        ("n_sft", ctypes.c_int32),
        ("n_bins", ctypes.c_int32),
        ("t_sft", ctypes.c_int64),
        ("timestamps", ctypes.c_void_p),
        ("a2", ctypes.c_void_p),
        ("b2", ctypes.c_void_p),
        ("ab", ctypes.c_void_p),
        ("fa", ctypes.c_void_p),
        ("fb", ctypes.c_void_p),
    ]


class BinResult(ctypes.Structure):
    _fields_ = [
        ("max2F", ctypes.c_double),
        ("logB", ctypes.c_double),
        ("t0", ctypes.c_int64),
        ("tau", ctypes.c_int64),
        ("m", ctypes.c_int32),
        ("n", ctypes.c_int32),
    ]


class BatchStats(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int32),
        ("groups", ctypes.c_int32),
        ("n_tiles", ctypes.c_int32),
        ("n_results", ctypes.c_int32),
        ("tune_ms", ctypes.c_double),
        ("last_ms", ctypes.c_double),
        ("last_fused_ms", ctypes.c_double),
        ("last_mfma_ms", ctypes.c_double),
    ]


BATCH_VARIANTS = ["fp64_r4", "fp32_r8", "fp32_r4_b2", "fp32_r4_b4", "mixed"]
BATCH_VARIANTS = BATCH_VARIANTS + [v + "_lowocc" for v in BATCH_VARIANTS]


# Every symbol the header declares, with (restype, argtypes).
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64
SIGNATURES = {
    "tfstat_ctx_create": (ctypes.c_int, [ctypes.c_int, _P, ctypes.c_size_t, _P, _P]),
    "tfstat_ctx_destroy": (ctypes.c_int, [_P]),
    "tfstat_atoms_upload": (ctypes.c_int, [_P, ctypes.POINTER(AtomsDesc), ctypes.POINTER(_U64)]),
    "tfstat_atoms_free": (ctypes.c_int, [_P, _U64]),
    "tfstat_atoms_info": (ctypes.c_int, [_P, _U64, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "tfstat_fmap": (ctypes.c_int, [_P, _U64, ctypes.POINTER(Window), _I32, _P,
                                   ctypes.POINTER(BinResult)]),
    "tfstat_logB": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, _P]),
    "tfstat_logB_noalloc": (ctypes.c_int, [_P, _P, _I32, _I32, _I32, _P]),
    "tfstat_window_odds": (ctypes.c_int, [_P, _U64, ctypes.POINTER(Window), ctypes.POINTER(Window), _I32,
                                          _P]),
    "tfstat_submit": (ctypes.c_int, [_P, _U64, ctypes.POINTER(Window), _I32, ctypes.POINTER(_U64)]),
    "tfstat_poll": (ctypes.c_int, [_P, _U64, ctypes.POINTER(BinResult), ctypes.POINTER(ctypes.c_int)]),
    "tfstat_cancel": (ctypes.c_int, [_P, _U64]),
    "tfstat_serve_config": (ctypes.c_int, [_P, _I32]),
    "tfstat_tiling_config": (ctypes.c_int, [_P, _I32, _I32]),
    "tfstat_batch_create": (ctypes.c_int, [_P, _I32, ctypes.POINTER(_U64), ctypes.POINTER(Window), _I32,
                                           _I32, ctypes.POINTER(_P)]),
    "tfstat_batch_run": (ctypes.c_int, [_P, _P, _I32, ctypes.POINTER(BinResult)]),
    "tfstat_batch_stats_read": (ctypes.c_int, [_P, ctypes.POINTER(BatchStats)]),
    "tfstat_batch_destroy": (ctypes.c_int, [_P, _P]),
    "tfstat_profile_enable": (ctypes.c_int, [_P, ctypes.c_int]),
    "tfstat_profile_read": (ctypes.c_int, [_P, _I32, ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_double)]),
    "tfstat_profile_reset": (ctypes.c_int, [_P]),
    "tfstat_last_error": (ctypes.c_char_p, []),
    "tfstat_version": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Loads libtfstat.so from the package directory; raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(
            "libtfstat.so is not built (expected at %s); run __graft_entry__.build() "
            "or python -m paper_1805_05652_amd.build" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class TfstatError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, str(code)), msg))
        self.code = code


def check(rc: int):
    if rc != OK:
        msg = load().tfstat_last_error()
        raise TfstatError(rc, msg.decode() if msg else "")
    return rc
