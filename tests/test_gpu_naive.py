"""GPU parity of the naive scan (int8 MFMA for u8) against the oracle."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from knn_inputs import gmm_u8, rng

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1902_09465_amd as P
    P.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return P


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("n,m,nq,k", [(5003, 200, 70, 10), (300, 64, 1, 1), (4096, 3072, 65, 64),
                                      (1000, 33, 130, 128), (129, 1, 3, 100)])
def test_naive_u8_parity(P, orc, n, m, nq, k):
    g = rng(n + m)
    X = g.integers(0, 256, size=(n, m), dtype=np.uint8)
    Q = g.integers(0, 256, size=(nq, m), dtype=np.uint8)
    db = P.KnnDB(dev(X))
    idx, dist = db.naive(dev(Q), k)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    for q in range(nq):
        ri, rd = orc.naive(X, Q[q], k)
        assert idx[q].tolist() == ri.tolist(), q
        assert np.array_equal(dist[q], rd)


def test_naive_u8_ties(P, orc):
    g = rng(3)
    X = g.integers(0, 3, size=(3000, 17), dtype=np.uint8)  # many equal distances
    Q = g.integers(0, 3, size=(9, 17), dtype=np.uint8)
    db = P.KnnDB(dev(X))
    idx, dist = db.naive(dev(Q), 50)
    for q in range(9):
        ri, rd = orc.naive(X, Q[q], 50)
        assert idx.cpu().numpy()[q].tolist() == ri.tolist()


def test_naive_u8_batched_config_sampled(P, orc):
    """The batched-integer workload shape (n = 100,000, m = 3072, 1,024
    queries); eight sampled queries are checked against the oracle."""
    X, Q = gmm_u8(2000, n=100_000, m=3072, nq=1024)
    db = P.KnnDB(dev(X))
    idx, dist = db.naive(dev(Q), 10)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    for q in (0, 1, 255, 256, 511, 700, 1022, 1023):
        ri, rd = orc.naive(X, Q[q], 10)
        assert idx[q].tolist() == ri.tolist(), q
        assert np.array_equal(dist[q], rd)


@pytest.mark.parametrize("n,m,nq,k,blocks", [(5000, 256, 200, 10, 2), (5000, 128, 130, 64, 2), (9000, 64, 300, 1, 3),
                                              (3000, 320, 129, 33, 1), (2600, 192, 1, 5, 1), (70, 64, 3, 10, 256),
                                              (1000, 100, 5, 64, 1), (1000, 65536, 5, 7, 256),
                                              (3000, 64, 1100, 10, 256)])
def test_naive_u8_wide_tile_ranges(P, orc, monkeypatch, n, m, nq, k, blocks):
    """The scan's 128-query x 256-point tile (k <= 64) with few point ranges,
    so that a block walks many tiles: a range's first tile fills the lists
    through LDS, later tiles are screened in the fragment layout against
    each list's k-th key, and a buffer that overflows sends its query the
    staged way again.  Half the queries sit next to a point, so the top of
    each list is crowded.  Every query equals the oracle, and the 64 x 128
    tile (KNN_NAIVE_WIDE=0) gives the same indices and distances."""
    g = rng(11 * n + m + k)
    X = g.integers(0, 256, size=(n, m), dtype=np.uint8)
    Q = g.integers(0, 256, size=(nq, m), dtype=np.uint8)
    near = X[g.integers(0, n, nq // 2)].astype(np.int64) + g.integers(-3, 4, (nq // 2, m))
    Q[: nq // 2] = np.clip(near, 0, 255).astype(np.uint8)
    db = P.KnnDB(dev(X))
    monkeypatch.setenv("KNN_NAIVE_BLOCKS", str(blocks))
    idx, dist = db.naive(dev(Q), k)
    monkeypatch.setenv("KNN_NAIVE_WIDE", "0")
    idx0, dist0 = db.naive(dev(Q), k)
    assert torch.equal(idx, idx0) and torch.equal(dist, dist0)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    for q in range(nq):
        ri, rd = orc.naive(X, Q[q], k)
        assert idx[q].tolist() == ri.tolist(), q
        assert np.array_equal(dist[q], rd), q


@pytest.mark.parametrize("n,m,nq,k", [(5003, 100, 70, 10), (3000, 128, 65, 64), (777, 3, 5, 1),
                                      (2049, 300, 17, 33)])
def test_naive_f32_parity(P, orc, n, m, nq, k):
    """Split-BF16 MFMA candidates rescored in FP64: the set and the
    distances equal the FP64 oracle exactly."""
    g = rng(7 * n + m)
    X = g.standard_normal((n, m)).astype(np.float32)
    Q = (X[g.integers(0, n, size=nq)] + 0.05 * g.standard_normal((nq, m))).astype(np.float32)
    db = P.KnnDB(dev(X))
    idx, dist = db.naive(dev(Q), k)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    for q in range(nq):
        ri, rd = orc.naive(X, Q[q], k)
        assert idx[q].tolist() == ri.tolist(), q
        assert np.array_equal(dist[q], rd)


def test_naive_f32_clustered_and_ties(P, orc):
    from knn_inputs import gmm_f32
    X, Q = gmm_f32(3100, n=50_000, m=128, n_centres=50, sigma=0.1, nq=40)
    X[100:120] = X[99]  # exact duplicates: equal distances, index order decides
    Q[0] = X[99]
    db = P.KnnDB(dev(X))
    idx, dist = db.naive(dev(Q), 25)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    for q in range(40):
        ri, rd = orc.naive(X, Q[q], 25)
        assert idx[q].tolist() == ri.tolist(), q
        assert np.array_equal(dist[q], rd)


def test_naive_f32_float_config_sampled(P, orc):
    """The float workload (n = 1,000,000 x 128, 10,000 queries from a
    1,000-cluster mixture); eight sampled queries against the oracle, and
    no query needs the exact rescan (the probe is sized so that every
    candidate list fits, also with few point ranges per query tile)."""
    import ctypes
    from knn_inputs import gmm_f32
    X, Q = gmm_f32(3000, n=1_000_000, m=128, n_centres=1000, sigma=0.1, nq=10_000)
    db = P.KnnDB(dev(X))
    lib = P.lib()
    P._lib.check(lib.knn_prof_enable(1))
    try:
        idx, dist = db.naive(dev(Q), 10)
        torch.cuda.synchronize()
        cnts = np.zeros(8, dtype=np.uint64)
        P._lib.check(lib.knn_prof_counters(cnts.ctypes.data_as(ctypes.c_void_p)))
    finally:
        P._lib.check(lib.knn_prof_enable(0))
    assert int(cnts[4]) == 0, f"{int(cnts[4])} queries rescanned"
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    for q in (0, 1, 63, 64, 4999, 9998, 9999, 1234):
        ri, rd = orc.naive(X, Q[q], 10)
        assert idx[q].tolist() == ri.tolist(), q
        assert np.array_equal(dist[q], rd)


@pytest.mark.parametrize("dtype,metric,k", [("u8", "l2", 129), ("u8", "l2", 700), ("u8", "l1", 300),
                                            ("f32", "l2", 65), ("f32", "l1", 200)])
def test_naive_large_k_exact_scan(P, orc, dtype, metric, k):
    """k above the fused lists' capacity (u8 128, f32 64): every query is
    scanned exactly; indices and distances equal the oracle's, ties by index
    included (few distinct values for u8)."""
    g = rng(k + (7 if dtype == "f32" else 0) + (1 if metric == "l1" else 0))
    n, m, nq = 3001, 61, 7
    if dtype == "u8":
        X = g.integers(0, 6, size=(n, m), dtype=np.uint8)
        Q = g.integers(0, 6, size=(nq, m), dtype=np.uint8)
    else:
        X = g.standard_normal((n, m)).astype(np.float32)
        Q = (X[g.integers(0, n, size=nq)] + 0.1 * g.standard_normal((nq, m))).astype(np.float32)
    db = P.KnnDB(dev(X), metric=metric)
    idx, dist = db.naive(dev(Q), k)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    for q in range(nq):
        ri, rd = orc.naive(X, Q[q], k, metric=1 if metric == "l1" else 0)
        assert idx[q].tolist() == ri.tolist(), q
        assert np.array_equal(dist[q], rd), q


def test_naive_f32_one_query_many_ranges(P, orc):
    """One query over 200,000 points: the scan splits the points into about
    a thousand ranges, the probe takes a tile of each; the set and the
    distances equal the oracle's and no query is rescanned."""
    import ctypes
    g = rng(4242)
    X = g.standard_normal((200_000, 64)).astype(np.float32)
    Q = (X[[12345]] + 0.05 * g.standard_normal((1, 64))).astype(np.float32)
    db = P.KnnDB(dev(X))
    lib = P.lib()
    P._lib.check(lib.knn_prof_enable(1))
    try:
        idx, dist = db.naive(dev(Q), 10)
        torch.cuda.synchronize()
        cnts = np.zeros(8, dtype=np.uint64)
        P._lib.check(lib.knn_prof_counters(cnts.ctypes.data_as(ctypes.c_void_p)))
    finally:
        P._lib.check(lib.knn_prof_enable(0))
    assert int(cnts[4]) == 0
    ri, rd = orc.naive(X, Q[0], 10)
    assert idx.cpu().numpy()[0].tolist() == ri.tolist()
    assert np.array_equal(dist.cpu().numpy()[0], rd)
