"""GPU parity of the l1 distance (samples |x_ij - x_j|) against the oracle,
through the C ABI: the naive scans (v_sad_u8 for u8, fp32 bound + FP64
rescoring for f32), the adaptive round form on every sampling path
(per-query, 16-slot groups, query lanes; with and without replacement),
per-round state, batches and the serving session."""
from __future__ import annotations

import os
import time

import numpy as np
import pytest
import torch

from knn_inputs import antipodal, gmm_f32, gmm_u8, pm_half, rng, tiny
from tests.helpers import brute_l1, contains_knn

pytestmark = pytest.mark.gpu

L1 = 1


@pytest.fixture(scope="module")
def P():
    import paper_1902_09465_amd as P
    P.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return P


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def l1db(P, X):
    db = P.KnnDB(dev(X), metric="l1")
    return db


def check_batch(P, orc, db, X, Q, k, **kw):
    idx, cnt, st = db.adaptive(dev(Q), k, P.default_params(**kw))
    idx, cnt = idx.cpu().numpy(), cnt.cpu().numpy()
    refs = []
    for q in range(Q.shape[0]):
        ref, rst = orc.adaptive(X, Q[q], k, orc.make_params(**kw), metric=L1)
        c = int(cnt[q])
        assert c == len(ref), (q, c, len(ref))
        assert idx[q, :c].tolist() == ref.tolist(), q
        assert np.all(idx[q, c:] == -1)
        s = st[q]
        assert (int(s["coord_evals"]), int(s["rounds"]), int(s["count"]), int(s["exact_points"])) == \
            (rst["coord_evals"], rst["rounds"], rst["count"], rst["exact_points"]), q
        refs.append(ref)
    return refs


@pytest.mark.parametrize("n,m,nq,k", [(5003, 200, 70, 10), (300, 64, 1, 1), (4096, 3072, 65, 64),
                                      (1000, 33, 130, 128), (129, 1, 3, 100)])
def test_l1_naive_u8_parity(P, orc, n, m, nq, k):
    g = rng(n + m + 1)
    X = g.integers(0, 256, size=(n, m), dtype=np.uint8)
    Q = g.integers(0, 256, size=(nq, m), dtype=np.uint8)
    db = l1db(P, X)
    idx, dist = db.naive(dev(Q), k)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    for q in range(nq):
        ri, rd = orc.naive(X, Q[q], k, metric=L1)
        assert idx[q].tolist() == ri.tolist(), q
        assert np.array_equal(dist[q], rd), q


def test_l1_naive_u8_ties(P, orc):
    """Many equal distances: the order by (distance, index) decides."""
    g = rng(5)
    X = g.integers(0, 3, size=(3000, 40), dtype=np.uint8)
    Q = g.integers(0, 3, size=(9, 40), dtype=np.uint8)
    db = l1db(P, X)
    idx, dist = db.naive(dev(Q), 50)
    for q in range(9):
        ri, rd = orc.naive(X, Q[q], 50, metric=L1)
        assert idx.cpu().numpy()[q].tolist() == ri.tolist()
        assert np.array_equal(dist.cpu().numpy()[q], rd)


@pytest.mark.parametrize("n,m,nq,k", [(5003, 100, 70, 10), (3000, 128, 65, 64), (777, 3, 5, 1),
                                      (2000, 515, 3, 17)])
def test_l1_naive_f32_parity(P, orc, n, m, nq, k):
    g = rng(n + m + 2)
    X = g.standard_normal((n, m)).astype(np.float32)
    Q = g.standard_normal((nq, m)).astype(np.float32)
    db = l1db(P, X)
    idx, dist = db.naive(dev(Q), k)
    idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
    for q in range(nq):
        ri, rd = orc.naive(X, Q[q], k, metric=L1)
        assert idx[q].tolist() == ri.tolist(), q
        assert np.array_equal(dist[q], rd), q  # the same FP64 sum in coordinate order


def test_l1_naive_f32_clustered_and_ties(P, orc):
    """Near-duplicates (candidate lists overflow into the exact rescan) and
    exact duplicates (ties broken by index)."""
    g = rng(8)
    base = g.standard_normal((20, 64)).astype(np.float32)
    X = np.repeat(base, 150, axis=0) + (g.standard_normal((3000, 64)) * 1e-4).astype(np.float32)
    X[::7] = base[0]
    Q = base[:4] + np.float32(1e-5)
    db = l1db(P, X)
    idx, dist = db.naive(dev(Q), 40)
    for q in range(4):
        ri, rd = orc.naive(X, Q[q], 40, metric=L1)
        assert idx.cpu().numpy()[q].tolist() == ri.tolist()
        assert np.array_equal(dist.cpu().numpy()[q], rd)


def test_l1_db_metric_and_flags(P):
    from paper_1902_09465_amd import KnnError, _lib
    import ctypes
    X = rng(1).integers(0, 256, size=(100, 16), dtype=np.uint8)
    a, b = P.KnnDB(dev(X)), P.KnnDB(dev(X), metric="l1", copy=True)
    v = ctypes.c_int32(-1)
    assert P.lib().knn_db_metric(a.handle, ctypes.byref(v)) == 0 and v.value == _lib.KNN_METRIC_L2
    assert P.lib().knn_db_metric(b.handle, ctypes.byref(v)) == 0 and v.value == _lib.KNN_METRIC_L1
    h = ctypes.c_void_p()
    Xd = dev(X)
    assert P.lib().knn_db_create(ctypes.c_void_p(Xd.data_ptr()), 100, 16, 0, 4, ctypes.byref(h)) == -1
    with pytest.raises(ValueError):
        P.KnnDB(Xd, metric="cosine")


@pytest.mark.parametrize("seed", range(4))
def test_l1_tiny_parity(P, orc, seed):
    X, Q, planted = tiny(seed=1100 + seed)
    db = l1db(P, X)
    for c_exact in (0, 10):
        for sampling in (0, 1):
            ref = check_batch(P, orc, db, X, Q, 5, h=5, delta=0.01, seed=seed, c_exact=c_exact,
                              sampling=sampling)[0]
            assert set(planted.tolist()) <= set(ref.tolist())


@pytest.mark.parametrize("path", ["u8", "u8_ungrouped", "u8_qlane", "u8_qlane_pure", "u8_qlane_pure_sparse",
                                  "u8_norepl", "u8_qlane_norepl", "f32", "f32_norepl", "u8_shared",
                                  "u8_qlane_pure_shared", "u8_qlane_pure_shared_norepl", "f32_shared_norepl"])
def test_l1_per_round_state_parity(P, orc, path, monkeypatch):
    """After every decide step the per-point (S, flags, round) equal the oracle's."""
    if path.startswith("u8_qlane"):
        monkeypatch.setenv("KNN_QL_MIN", "1")
    if path.startswith("u8_ungrouped"):
        monkeypatch.setenv("KNN_GROUP", "0")
    if "_sparse" in path:  # per-slot lists from round 1 on
        monkeypatch.setenv("KNN_SPARSE_DIV", "1")
    g = rng(78)
    if path.startswith("u8"):
        X, Q = gmm_u8(78, n=5003, m=202, n_centres=6, sigma=25.0, nq=1)
    else:
        X, Q = gmm_f32(78, n=5003, m=101, n_centres=6, sigma=0.3, nq=1)
    db = l1db(P, X)
    kw = dict(h=4, delta=0.05, seed=int(g.integers(1 << 40)), b0=8, growth=1.5,
              c_exact=0 if "pure" in path else 3,
              sampling=(1 if "norepl" in path else 0) + (2 if "shared" in path else 0))
    T = orc.schedule(8, 1.5, 1.0, X.shape[1])
    for r in range(1, len(T) + 2):
        S, fl, ri = db.adaptive_state(dev(Q), 6, P.default_params(**kw), r)
        _, _, (So, flo, rio) = orc.adaptive(X, Q[0], 6, orc.make_params(**kw), stop_after=r, dump=True,
                                            metric=L1)
        assert np.array_equal(fl, flo), f"round {r}: flags differ"
        assert np.array_equal(S, So), f"round {r}: sums differ"
        assert np.array_equal(ri, rio), f"round {r}: round index differs"


KNOBS = [{}, {"KNN_GROUP": "0"}, {"KNN_QL_MIN": "1"}, {"KNN_QL_MIN": "1", "KNN_SPARSE_DIV": "1"}, {"KNN_QL": "0"},
         {"KNN_LPP": "4"},
         {"KNN_CH_SAMPLE": "100"}, {"KNN_STAGE_MIN": "4", "KNN_STAGE_ROWS": "16"}]


@pytest.mark.parametrize("knob", KNOBS, ids=lambda k: ",".join(f"{a}={b}" for a, b in k.items()) or "default")
@pytest.mark.parametrize("sampling", [0, 1, 2, 3])
def test_l1_batched_paths_parity(P, orc, knob, sampling, monkeypatch):
    """A batch sharing seed and schedule (16-slot groups, or query lanes with
    KNN_QL_MIN=1), each query equal to the oracle run alone."""
    for a, b in knob.items():
        monkeypatch.setenv(a, b)
    X, Q = gmm_u8(14, n=3001, m=200, n_centres=5, sigma=20.0, nq=20)
    db = l1db(P, X)
    check_batch(P, orc, db, X, Q, 6, h=6, delta=0.05, seed=3, c_exact=4, sampling=sampling)
    check_batch(P, orc, db, X, Q, 6, h=6, delta=0.05, seed=4, c_exact=0, sampling=sampling)


def test_l1_query_lane_batch_large(P, orc):
    """70 queries (query lanes by default), the exact round on the per-slot
    path (l1 has no GEMM form); sampled queries checked against the oracle."""
    X, Q = gmm_u8(15, n=20011, m=256, n_centres=8, sigma=25.0, nq=70)
    db = l1db(P, X)
    kw = dict(h=5, delta=0.01, seed=11)
    idx, cnt, st = db.adaptive(dev(Q), 5, P.default_params(**kw))
    idx, cnt = idx.cpu().numpy(), cnt.cpu().numpy()
    for q in (0, 1, 33, 68, 69):
        ref, rst = orc.adaptive(X, Q[q], 5, orc.make_params(**kw), metric=L1)
        assert idx[q, :cnt[q]].tolist() == ref.tolist(), q
        assert int(st[q]["coord_evals"]) == rst["coord_evals"]
    for q in range(70):
        assert contains_knn(idx[q, :cnt[q]], brute_l1(X, Q[q]), 5)


def test_l1_two_valued_equals_l2(P, orc):
    """On {0,255} data l1 and l2 make identical decisions (the estimates are
    the same numbers), on the GPU as in the oracle."""
    X, Q, _ = pm_half(23, 4000, 256)
    Qb = np.repeat(Q, 20, axis=0)
    kw = dict(h=4, delta=0.05, seed=5, c_exact=3)
    a = P.KnnDB(dev(X)).adaptive(dev(Qb), 6, P.default_params(**kw))
    b = l1db(P, X).adaptive(dev(Qb), 6, P.default_params(**kw))
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_l1_f32_parity(P, orc):
    X, Q = gmm_f32(22, n=3000, m=100, n_centres=10, sigma=0.2, nq=4)
    db = l1db(P, X)
    for sampling in (0, 1):
        for q, ref in enumerate(check_batch(P, orc, db, X, Q, 5, h=5, delta=0.05, seed=7, c_exact=5,
                                            sampling=sampling)):
            assert contains_knn(ref, brute_l1(X, Q[q]), 5, rtol=1e-6)


def test_l1_worked_example(P, orc):
    X, Q, where = antipodal()
    db = l1db(P, X)
    idx, cnt, st = db.adaptive(dev(Q), 5, P.default_params(h=5, delta=0.01, seed=123))
    assert sorted(idx.cpu().numpy()[0, :int(cnt[0])].tolist()) == where.tolist()
    assert int(st[0]["coord_evals"]) == 256_000 and int(st[0]["rounds"]) == 3


def test_l1_session(P, orc):
    """Serving session on an l1 DB: each result equals the oracle's."""
    X, Q = gmm_u8(32, n=6000, m=200, n_centres=5, sigma=30.0, nq=12)
    db = l1db(P, X)
    sess = P.Session(1 << 30)
    try:
        did = sess.add_db(db)
        g = rng(32)
        reqs = []
        for q in range(12):
            p = P.default_params(h=4, seed=int(g.integers(1 << 40)), c_exact=int(q % 2) * 4)
            reqs.append((q, p, sess.submit(did, Q[q], 5, p)))
        for q, p, t in reqs:
            t0 = time.time()
            while True:
                r = sess.poll(t, 9)
                if r is not None:
                    break
                assert time.time() - t0 < 60, "request did not finish"
                time.sleep(0.0005)
            idx, st = r
            ref, rst = orc.adaptive(X, Q[q], 5, orc.make_params(h=4, seed=p.seed, c_exact=p.c_exact), metric=L1)
            assert idx.tolist() == ref.tolist(), q
            assert int(st["coord_evals"]) == rst["coord_evals"]
    finally:
        sess.close()
