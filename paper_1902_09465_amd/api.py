"""torch-facing wrapper over the C ABI (marshalling only)."""
from __future__ import annotations

import ctypes
from typing import Sequence

import numpy as np
import torch

from . import _lib
from ._lib import Params, Stats, check, default_params, lib

STATS_DTYPE = np.dtype([("coord_evals", "<i8"), ("rounds", "<i4"), ("count", "<i4"),
                        ("exact_points", "<i8")])


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.uint8:
        return _lib.KNN_U8
    if t.dtype == torch.float32:
        return _lib.KNN_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def schedule(params: Params, n: int, m: int):
    """(T[r], alpha[r]) of the sampled rounds; round len(T) is exact."""
    T = np.zeros(_lib.KNN_MAX_ROUNDS, dtype=np.int32)
    A = np.zeros(_lib.KNN_MAX_ROUNDS, dtype=np.float64)
    R = ctypes.c_int32()
    check(lib().knn_schedule(ctypes.byref(params), n, m, T.ctypes.data_as(ctypes.c_void_p),
                             A.ctypes.data_as(ctypes.c_void_p), ctypes.byref(R)))
    return T[:R.value].copy(), A[:R.value].copy()


class KnnDB:
    """A registered point set (Section 3: X = {x_1..x_n} in R^m), device resident."""

    def __init__(self, X: torch.Tensor, copy: bool = False, metric: str = "l2"):
        """metric: "l2" (squared Euclidean, the paper's) or "l1" (sum of
        absolute differences); every search on the DB uses it."""
        if not X.is_cuda or X.dim() != 2:
            raise ValueError("X must be a 2-D CUDA tensor")
        if metric not in ("l2", "l1"):
            raise ValueError('metric must be "l2" or "l1"')
        X = X.contiguous()
        self.X = X  # keeps a borrowed buffer alive
        self.n, self.m = X.shape
        self.dtype = X.dtype
        self.metric = metric
        flags = _lib.KNN_DB_COPY if copy else _lib.KNN_DB_BORROW
        if metric == "l1":
            flags |= _lib.KNN_DB_L1
        h = ctypes.c_void_p()
        check(lib().knn_db_create(ctypes.c_void_p(X.data_ptr()), self.n, self.m, _dtype_code(X), flags,
                                  ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            torch.cuda.synchronize()
            check(lib().knn_db_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _queries(self, Q: torch.Tensor) -> torch.Tensor:
        if Q.dim() == 1:
            Q = Q[None, :]
        if not Q.is_cuda or Q.dtype != self.dtype or Q.shape[1] != self.m:
            raise ValueError("queries must be CUDA [nq, m] of the DB dtype")
        return Q.contiguous()

    def adaptive(self, Q: torch.Tensor, k, params: Params | Sequence[Params] | None = None,
                 stream=None, with_stats: bool = True):
        """Adaptive k-NN (Algorithm 1, round form).  Returns (idx [nq, stride]
        int64 padded with -1, count [nq] int32, stats structured array or None)."""
        Q = self._queries(Q)
        nq = Q.shape[0]
        ks = np.full(nq, k, dtype=np.int32) if np.isscalar(k) else np.ascontiguousarray(k, dtype=np.int32)
        if params is None:
            params = default_params()
        plist = [params] if isinstance(params, Params) else list(params)
        parr = (Params * len(plist))(*plist)
        if len(plist) == 1:  # k + h per query (h < 0: h = k)
            h = plist[0].h
            kh_max = int(ks.max()) * 2 if h < 0 else int(ks.max()) + int(h)
        else:
            kh_max = max(int(ks[q]) + (plist[q].h if plist[q].h >= 0 else int(ks[q])) for q in range(nq))
        stride = int(max(1, min(kh_max, self.n)))
        dev = Q.device
        idx = torch.empty((nq, stride), dtype=torch.int64, device=dev)
        cnt = torch.empty((nq,), dtype=torch.int32, device=dev)
        st = torch.empty((nq, 24), dtype=torch.uint8, device=dev) if with_stats else None
        check(lib().knn_adaptive(self.handle, ctypes.c_void_p(Q.data_ptr()), nq,
                                 ks.ctypes.data_as(ctypes.c_void_p), parr, len(plist),
                                 ctypes.c_void_p(idx.data_ptr()), stride, ctypes.c_void_p(cnt.data_ptr()),
                                 ctypes.c_void_p(st.data_ptr()) if st is not None else None,
                                 _stream_handle(stream)))
        stats = None
        if st is not None:
            stats = st.cpu().numpy().view(STATS_DTYPE).reshape(nq)
        return idx, cnt, stats

    def autotune(self, Q: torch.Tensor, k: int, params: Params | None = None, reps: int = 2,
                 schedule_report: bool = False, stream=None) -> dict:
        """Times the performance knobs on these queries and keeps the fastest
        for this DB; returns {candidate: ms}."""
        Q = self._queries(Q)
        buf = ctypes.create_string_buffer(8192)
        check(lib().knn_autotune(self.handle, ctypes.c_void_p(Q.data_ptr()), Q.shape[0], k,
                                 ctypes.byref(params or default_params()), reps, int(schedule_report), buf,
                                 len(buf), _stream_handle(stream)))
        out = {}
        for line in buf.value.decode().splitlines():
            name, ms = line.rsplit(" ", 1)
            out[name] = float(ms)
        return out

    def adaptive_state(self, Q: torch.Tensor, k, params: Params | Sequence[Params], stop_after: int,
                       query: int = 0, stream=None):
        """Per-point state (S, fl, ri) of query `query` of the batch Q (run as
        knn_adaptive would run it) after `stop_after` decide steps."""
        Q = self._queries(Q)
        nq = Q.shape[0]
        ks = np.full(nq, k, dtype=np.int32) if np.isscalar(k) else np.ascontiguousarray(k, dtype=np.int32)
        plist = [params] if isinstance(params, Params) else list(params)
        parr = (Params * len(plist))(*plist)
        S = np.zeros(self.n, dtype=np.int64)
        fl = np.zeros(self.n, dtype=np.uint8)
        ri = np.zeros(self.n, dtype=np.uint8)
        check(lib().knn_adaptive_state(self.handle, ctypes.c_void_p(Q.data_ptr()), nq,
                                       ks.ctypes.data_as(ctypes.c_void_p), parr, len(plist), query, stop_after,
                                       S.ctypes.data_as(ctypes.c_void_p), fl.ctypes.data_as(ctypes.c_void_p),
                                       ri.ctypes.data_as(ctypes.c_void_p), _stream_handle(stream)))
        return S, fl, ri

    def naive(self, Q: torch.Tensor, k: int, stream=None, with_dist: bool = True):
        """Naive scan (Section 3): idx [nq, k] int64, dist [nq, k] float64."""
        Q = self._queries(Q)
        nq = Q.shape[0]
        idx = torch.empty((nq, k), dtype=torch.int64, device=Q.device)
        dist = torch.empty((nq, k), dtype=torch.float64, device=Q.device) if with_dist else None
        check(lib().knn_naive(self.handle, ctypes.c_void_p(Q.data_ptr()), nq, k,
                              ctypes.c_void_p(idx.data_ptr()),
                              ctypes.c_void_p(dist.data_ptr()) if dist is not None else None,
                              _stream_handle(stream)))
        return idx, dist


    def naive_noalloc(self, Q: torch.Tensor, k: int, idx: torch.Tensor, dist: torch.Tensor | None = None,
                      stream=None):
        """knn_naive_noalloc into caller-provided outputs (u8 DBs): idx [nq, k]
        int64 and dist [nq, k] float64 (or None).  The library allocates nothing."""
        Q = self._queries(Q)
        nq = Q.shape[0]
        if idx.shape != (nq, k) or idx.dtype != torch.int64 or not idx.is_contiguous():
            raise ValueError("idx must be a contiguous int64 [nq, k] tensor")
        if dist is not None and (dist.shape != (nq, k) or dist.dtype != torch.float64 or not dist.is_contiguous()):
            raise ValueError("dist must be a contiguous float64 [nq, k] tensor")
        check(lib().knn_naive_noalloc(self.handle, ctypes.c_void_p(Q.data_ptr()), nq, k,
                                      ctypes.c_void_p(idx.data_ptr()),
                                      ctypes.c_void_p(dist.data_ptr()) if dist is not None else None,
                                      _stream_handle(stream)))
        return idx, dist


class Session:
    """Serving session (continuous batching with memory admission)."""

    def __init__(self, hbm_budget_bytes: int = 8 << 30):
        h = ctypes.c_void_p()
        check(lib().knn_session_create(hbm_budget_bytes, ctypes.byref(h)))
        self.handle = h
        self.dbs = {}

    def add_db(self, db: KnnDB) -> int:
        i = ctypes.c_int32()
        check(lib().knn_session_add_db(self.handle, db.handle, ctypes.byref(i)))
        self.dbs[i.value] = db
        return i.value

    def submit(self, db_id: int, q: np.ndarray, k: int, params: Params | None = None) -> int:
        q = np.ascontiguousarray(q)
        t = ctypes.c_uint64()
        check(lib().knn_session_submit(self.handle, db_id, q.ctypes.data_as(ctypes.c_void_p), k,
                                       ctypes.byref(params or default_params()), ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int, kh: int):
        """None while pending, else (idx array, stats dict)."""
        out = np.full(max(1, kh), -1, dtype=np.int64)
        c = ctypes.c_int32()
        st = Stats()
        rc = check(lib().knn_session_poll(self.handle, ticket, out.ctypes.data_as(ctypes.c_void_p),
                                          ctypes.byref(c), ctypes.byref(st)))
        if rc == _lib.KNN_PENDING:
            return None
        return out[:c.value].copy(), dict(coord_evals=st.coord_evals, rounds=st.rounds, count=st.count,
                                          exact_points=st.exact_points)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            check(lib().knn_session_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
