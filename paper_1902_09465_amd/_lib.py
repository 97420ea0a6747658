"""ctypes binding of libknn (include/knn.h): argument marshalling only.

Every step of the search runs in libknn's HIP kernels; torch supplies device
memory and the stream handle.  Importing this module on a machine where
libknn.so has not been built raises ImportError -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libknn.so")

KNN_OK, KNN_PENDING = 0, 1
KNN_EINVAL, KNN_ENOMEM, KNN_EDEVICE, KNN_EBUSY, KNN_ENOTFOUND = -1, -2, -3, -4, -5
KNN_U8, KNN_F32 = 0, 1
KNN_DB_BORROW, KNN_DB_COPY, KNN_DB_L1 = 0, 1, 2
KNN_METRIC_L2, KNN_METRIC_L1 = 0, 1
KNN_MAX_KH = 2048
KNN_MAX_ROUNDS = 48


class Params(ctypes.Structure):
    """knn_params (include/knn.h)."""
    _fields_ = [("h", ctypes.c_int64), ("delta", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("alpha_kind", ctypes.c_int32),
                ("c_alpha", ctypes.c_double), ("b0", ctypes.c_int32),
                ("growth", ctypes.c_float), ("theta_exact", ctypes.c_float),
                ("c_exact", ctypes.c_int32), ("sampling", ctypes.c_int32)]


class Stats(ctypes.Structure):
    """knn_stats (include/knn.h), 24 bytes."""
    _fields_ = [("coord_evals", ctypes.c_int64), ("rounds", ctypes.c_int32),
                ("count", ctypes.c_int32), ("exact_points", ctypes.c_int64)]


assert ctypes.sizeof(Stats) == 24


class KnnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libknn error {code}: {msg}")
        self.code = code


_lib = None

# (name, restype, argtypes)
_P, _I64, _I32, _U64, _D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
EXPORTS = [
    ("knn_params_default", None, [ctypes.POINTER(Params)]),
    ("knn_last_error", ctypes.c_char_p, []),
    ("knn_version", ctypes.c_char_p, []),
    ("knn_db_create", ctypes.c_int, [_P, _I64, _I64, ctypes.c_int, _I32, ctypes.POINTER(_P)]),
    ("knn_db_destroy", ctypes.c_int, [_P]),
    ("knn_db_info", ctypes.c_int, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I32)]),
    ("knn_db_metric", ctypes.c_int, [_P, ctypes.POINTER(_I32)]),
    ("knn_schedule", ctypes.c_int, [ctypes.POINTER(Params), _I64, _I64, _P, _P, ctypes.POINTER(_I32)]),
    ("knn_adaptive", ctypes.c_int, [_P, _P, _I64, _P, ctypes.POINTER(Params), _I64, _P, _I64, _P, _P, _P]),
    ("knn_adaptive_state", ctypes.c_int, [_P, _P, _I64, _P, ctypes.POINTER(Params), _I64, _I64, _I32, _P, _P, _P,
                                          _P]),
    ("knn_naive", ctypes.c_int, [_P, _P, _I64, _I32, _P, _P, _P]),
    ("knn_naive_noalloc", ctypes.c_int, [_P, _P, _I64, _I32, _P, _P, _P]),
    ("knn_autotune", ctypes.c_int, [_P, _P, _I64, _I32, ctypes.POINTER(Params), _I32, _I32, ctypes.c_char_p,
                                    ctypes.c_size_t, _P]),
    ("knn_session_create", ctypes.c_int, [ctypes.c_size_t, ctypes.POINTER(_P)]),
    ("knn_session_add_db", ctypes.c_int, [_P, _P, ctypes.POINTER(_I32)]),
    ("knn_session_submit", ctypes.c_int, [_P, _I32, _P, _I32, ctypes.POINTER(Params), ctypes.POINTER(_U64)]),
    ("knn_session_poll", ctypes.c_int, [_P, _U64, _P, ctypes.POINTER(_I32), ctypes.POINTER(Stats)]),
    ("knn_session_destroy", ctypes.c_int, [_P]),
    ("knn_prof_enable", ctypes.c_int, [ctypes.c_int]),
    ("knn_prof_read", ctypes.c_int, [_I32, ctypes.POINTER(_D), ctypes.POINTER(_I64), ctypes.POINTER(_D)]),
    ("knn_prof_counters", ctypes.c_int, [_P]),
]


def lib():
    """Loads libknn.so (raises ImportError when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run paper_1902_09465_amd/build.py "
                              "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in EXPORTS:
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int) -> int:
    if rc < 0:
        raise KnnError(rc, lib().knn_last_error().decode())
    return rc


def default_params(**kw) -> Params:
    p = Params()
    lib().knn_params_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p
