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
