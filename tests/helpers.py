"""Shared test helpers: brute-force distances and tie-aware containment."""
from __future__ import annotations

import numpy as np


def brute_dists(X: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Exact squared distances by numpy (int64 for u8, float64 for f32)."""
    q = np.asarray(q).reshape(-1)
    if X.dtype == np.uint8:
        d = X.astype(np.int64) - q.astype(np.int64)[None, :]
        return (d * d).sum(axis=1)
    d = X.astype(np.float64) - q.astype(np.float64)[None, :]
    return (d * d).sum(axis=1)


def brute_l1(X: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Exact l1 distances by numpy (int64 for u8, float64 for f32)."""
    q = np.asarray(q).reshape(-1)
    if X.dtype == np.uint8:
        return np.abs(X.astype(np.int64) - q.astype(np.int64)[None, :]).sum(axis=1)
    return np.abs(X.astype(np.float64) - q.astype(np.float64)[None, :]).sum(axis=1)


def knn_sets(dists: np.ndarray, k: int, rtol: float = 0.0):
    """(strictly-closer set, boundary-tie set, d_(k)) for tie-aware checks."""
    dk = np.sort(dists)[k - 1]
    tol = rtol * abs(float(dk))
    strict = set(np.nonzero(dists < dk - tol)[0].tolist())
    ties = set(np.nonzero(np.abs(dists - dk) <= tol)[0].tolist())
    return strict, ties, dk


def contains_knn(returned, dists: np.ndarray, k: int, rtol: float = 0.0) -> bool:
    """True when `returned` contains a k-nearest-neighbour set: every point
    strictly closer than the k-th distance, and enough points at the k-th
    distance to make up k."""
    R = set(int(i) for i in returned if i >= 0)
    strict, ties, _ = knn_sets(dists, k, rtol)
    if not strict <= R:
        return False
    return len(strict) + len(R & ties) >= k
