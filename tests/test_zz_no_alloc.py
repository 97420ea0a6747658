"""knn_naive_noalloc, the naive scan that allocates nothing (its working
memory is a fixed per-device array), against knn_naive through the C ABI:
equal indices and distances on consecutive calls, the second one smaller,
on squared-l2 and l1 DBs, and with point ranges widened to fit the array."""
from __future__ import annotations

import os

import numpy as np
import pytest
import torch

from knn_inputs import gmm_u8

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1902_09465_amd as P
    P.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return P


def _run_both(db, Q, nq, k):
    Qd = torch.from_numpy(np.ascontiguousarray(Q[:nq])).cuda()
    ref_i, ref_d = db.naive(Qd, k)
    idx = torch.full((nq, k), -7, dtype=torch.int64, device="cuda")
    dist = torch.full((nq, k), -1.0, dtype=torch.float64, device="cuda")
    db.naive_noalloc(Qd, k, idx, dist)
    torch.cuda.synchronize()
    return ref_i, ref_d, idx, dist


@pytest.mark.parametrize("metric", ["l2", "l1"])
def test_noalloc_equals_naive_twice(P, metric):
    X, Q = gmm_u8(8100, n=20011, m=700, n_centres=8, sigma=30.0, nq=300)
    db = P.KnnDB(torch.from_numpy(X).cuda(), metric=metric)
    for nq, k in ((300, 17), (37, 5)):  # the second call smaller: stale lists must not leak
        ref_i, ref_d, idx, dist = _run_both(db, Q, nq, k)
        assert torch.equal(idx, ref_i), (metric, nq, k)
        assert torch.equal(dist, ref_d), (metric, nq, k)
    db.close()


def test_noalloc_widens_ranges_to_fit(P, monkeypatch):
    """Many short point ranges (KNN_NAIVE_BLOCKS) would need 1000 x 157 x 128
    x 8 bytes of candidate lists, more than the fixed array: the ranges are
    widened and the result is unchanged; then a small call again."""
    monkeypatch.setenv("KNN_NAIVE_BLOCKS", "100000")
    X, Q = gmm_u8(8200, n=20011, m=256, n_centres=8, sigma=30.0, nq=1000)
    db = P.KnnDB(torch.from_numpy(X).cuda())
    for nq, k in ((1000, 128), (3, 2)):
        ref_i, ref_d, idx, dist = _run_both(db, Q, nq, k)
        assert torch.equal(idx, ref_i) and torch.equal(dist, ref_d), (nq, k)
    db.close()


def test_noalloc_rejects_f32(P):
    from paper_1902_09465_amd import KnnError
    X = torch.zeros((100, 8), dtype=torch.float32, device="cuda")
    db = P.KnnDB(X)
    idx = torch.empty((1, 3), dtype=torch.int64, device="cuda")
    with pytest.raises(KnnError):
        db.naive_noalloc(X[:1], 3, idx)
    db.close()
