"""CPU oracle for adaptive k-NN -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it.

Thin ctypes marshalling over ``liboracle.so`` (plain C, ``knn_oracle.c``),
which implements the paper's estimator, confidence widths, round schedule,
accept/discard rule and the naive scan.  See ``knn_oracle.c`` for the
passages each function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "knn_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

U8, F32 = 0, 1
L2, L1 = 0, 1  # distance: squared l2, or l1 (samples |x_ij - x_j|)


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-Wextra", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("h", ctypes.c_int64), ("delta", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("alpha_kind", ctypes.c_int32),
                ("c_alpha", ctypes.c_double), ("b0", ctypes.c_int32),
                ("growth", ctypes.c_float), ("theta_exact", ctypes.c_float),
                ("c_exact", ctypes.c_int32), ("sampling", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("coord_evals", ctypes.c_int64), ("rounds", ctypes.c_int32),
                ("count", ctypes.c_int32), ("exact_points", ctypes.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_draw.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64]
        L.orc_draw.restype = ctypes.c_uint32
        L.orc_index.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        L.orc_perm_index.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        L.orc_perm_index.restype = ctypes.c_int64
        L.orc_draw_shared.argtypes = [ctypes.c_uint64, ctypes.c_int64]
        L.orc_draw_shared.restype = ctypes.c_uint32
        L.orc_shared_index.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64]
        L.orc_shared_index.restype = ctypes.c_int64
        L.orc_shared_perm_index.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64]
        L.orc_shared_perm_index.restype = ctypes.c_int64
        L.orc_coord.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        L.orc_coord.restype = ctypes.c_int64
        L.orc_index.restype = ctypes.c_int64
        L.orc_alpha.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                ctypes.c_double, ctypes.c_double]
        L.orc_alpha.restype = ctypes.c_double
        L.orc_schedule.argtypes = [ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_int64, P, ctypes.c_int32]
        L.orc_schedule.restype = ctypes.c_int32
        L.orc_scaling.argtypes = [P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, P, P]
        L.orc_scaling.restype = ctypes.c_int32
        L.orc_adaptive.argtypes = [P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P,
                                   ctypes.c_int32, ctypes.POINTER(Params), ctypes.c_int32,
                                   P, ctypes.POINTER(Stats), P, P, P]
        L.orc_adaptive.restype = ctypes.c_int32
        L.orc_alg1.argtypes = [P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P,
                               ctypes.c_int32, ctypes.POINTER(Params), ctypes.c_int64,
                               P, ctypes.POINTER(Stats), P]
        L.orc_alg1.restype = ctypes.c_int32
        L.orc_alg1_heaps.argtypes = [P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P,
                                     ctypes.c_int32, ctypes.POINTER(Params), ctypes.c_int64,
                                     P, ctypes.POINTER(Stats), P]
        L.orc_alg1_heaps.restype = ctypes.c_int32
        L.orc_naive.argtypes = [P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P,
                                ctypes.c_int32, P, P]
        L.orc_naive.restype = ctypes.c_int32
        L.orc_exact_dist.argtypes = [P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P,
                                     ctypes.c_int64]
        L.orc_exact_dist.restype = ctypes.c_double
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dtype_code(X: np.ndarray) -> int:
    if X.dtype == np.uint8:
        return U8
    if X.dtype == np.float32:
        return F32
    raise TypeError(f"unsupported dtype {X.dtype}")


def make_params(h=-1, delta=0.01, seed=0, alpha_kind=0, c_alpha=0.0, b0=64,
                growth=2.0, theta_exact=1.0, c_exact=0, sampling=0) -> Params:
    return Params(h, delta, seed, alpha_kind, c_alpha, b0, growth, theta_exact, c_exact, sampling)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def perm_index(seed: int, i: int, t: int, m: int) -> int:
    return int(lib().orc_perm_index(seed, i, t, m))


def draw_shared(seed: int, t: int) -> int:
    return int(lib().orc_draw_shared(seed, t))


def shared_index(seed: int, t: int, m: int) -> int:
    return int(lib().orc_shared_index(seed, t, m))


def shared_perm_index(seed: int, t: int, m: int) -> int:
    return int(lib().orc_shared_perm_index(seed, t, m))


def coord(sampling: int, seed: int, i: int, t: int, m: int) -> int:
    return int(lib().orc_coord(sampling, seed, i, t, m))


def draw(seed: int, i: int, t: int) -> int:
    return int(lib().orc_draw(seed, i, t))


def index(seed: int, i: int, t: int, m: int) -> int:
    return int(lib().orc_index(seed, i, t, m))


def alpha(kind: int, u: int, n: int, delta: float, c_alpha: float = 0.0) -> float:
    return float(lib().orc_alpha(kind, u, n, delta, c_alpha))


def schedule(b0=64, growth=2.0, theta=1.0, m=256, maxlen=64):
    T = np.zeros(maxlen, dtype=np.int32)
    R = lib().orc_schedule(b0, growth, theta, m, _ptr(T), maxlen)
    if R < 0:
        raise ValueError("invalid schedule")
    return T[:R].copy()


def scaling(X: np.ndarray, q: np.ndarray, metric: int = 0):
    X = np.ascontiguousarray(X)
    q = np.ascontiguousarray(q)
    W = ctypes.c_double()
    F = ctypes.c_int32()
    rc = lib().orc_scaling(_ptr(X), X.shape[0], X.shape[1], _dtype_code(X), metric, _ptr(q),
                           ctypes.byref(W), ctypes.byref(F))
    return rc, W.value, F.value


def adaptive(X: np.ndarray, q: np.ndarray, k: int, params: Params | None = None,
             stop_after: int = 0, dump: bool = False, metric: int = 0):
    """Returns (idx[count], stats dict[, (S, fl, ri)])."""
    X = np.ascontiguousarray(X)
    q = np.ascontiguousarray(q, dtype=X.dtype)
    n, m = X.shape
    if params is None:
        params = make_params()
    h = params.h if params.h >= 0 else k
    out = np.full(k + h, -1, dtype=np.int64)
    st = Stats()
    S = np.zeros(n, dtype=np.int64) if dump else None
    fl = np.zeros(n, dtype=np.uint8) if dump else None
    ri = np.zeros(n, dtype=np.uint8) if dump else None
    rc = lib().orc_adaptive(_ptr(X), n, m, _dtype_code(X), metric, _ptr(q), k, ctypes.byref(params),
                            stop_after, _ptr(out), ctypes.byref(st),
                            _ptr(S) if dump else None, _ptr(fl) if dump else None,
                            _ptr(ri) if dump else None)
    if rc != 0:
        raise ValueError(f"oracle adaptive rejected arguments (rc={rc})")
    stats = dict(coord_evals=st.coord_evals, rounds=st.rounds, count=st.count,
                 exact_points=st.exact_points)
    idx = out[:st.count].copy()
    if dump:
        return idx, stats, (S, fl, ri)
    return idx, stats


def alg1(X: np.ndarray, q: np.ndarray, k: int, params: Params | None = None,
         max_iter: int = 1 << 40, metric: int = 0, heaps: bool = False):
    """Algorithm 1, sequential as published.  Returns (idx[k+h], stats dict,
    final sample counts T[n]).  heaps: the Section 4.1 bookkeeping (coupled
    heaps, O(log n) per iteration) instead of the ordered array; the same
    results."""
    X = np.ascontiguousarray(X)
    q = np.ascontiguousarray(q, dtype=X.dtype)
    n, m = X.shape
    if params is None:
        params = make_params()
    h = params.h if params.h >= 0 else k
    out = np.full(k + h, -1, dtype=np.int64)
    T = np.zeros(n, dtype=np.int64)
    st = Stats()
    fn = lib().orc_alg1_heaps if heaps else lib().orc_alg1
    rc = fn(_ptr(X), n, m, _dtype_code(X), metric, _ptr(q), k, ctypes.byref(params), max_iter,
            _ptr(out), ctypes.byref(st), _ptr(T))
    if rc == -2:
        raise RuntimeError("Algorithm 1 did not terminate within max_iter iterations")
    if rc != 0:
        raise ValueError(f"oracle alg1 rejected arguments (rc={rc})")
    stats = dict(coord_evals=st.coord_evals, iterations=st.rounds, count=st.count,
                 exact_points=st.exact_points)
    return out[:st.count].copy(), stats, T


def naive(X: np.ndarray, q: np.ndarray, k: int, metric: int = 0):
    X = np.ascontiguousarray(X)
    q = np.ascontiguousarray(q, dtype=X.dtype)
    n, m = X.shape
    out = np.full(k, -1, dtype=np.int64)
    dist = np.zeros(k, dtype=np.float64)
    rc = lib().orc_naive(_ptr(X), n, m, _dtype_code(X), metric, _ptr(q), k, _ptr(out), _ptr(dist))
    if rc != 0:
        raise ValueError(f"oracle naive rejected arguments (rc={rc})")
    return out, dist


def exact_dist(X: np.ndarray, q: np.ndarray, i: int, metric: int = 0) -> float:
    X = np.ascontiguousarray(X)
    q = np.ascontiguousarray(q, dtype=X.dtype)
    return float(lib().orc_exact_dist(_ptr(X), X.shape[0], X.shape[1], _dtype_code(X),
                                      metric, _ptr(q), i))
