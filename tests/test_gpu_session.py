"""Serving session on the GPU: continuous batching over resident DBs; each
result is the same alone and in a mix, and equals the oracle."""
from __future__ import annotations

import os
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

from knn_inputs import gmm_f32, gmm_u8, rng

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1902_09465_amd as P
    P.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return P


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def wait(sess, ticket, kh, timeout=60.0):
    t0 = time.time()
    while True:
        r = sess.poll(ticket, kh)
        if r is not None:
            return r
        if time.time() - t0 > timeout:
            raise TimeoutError("request did not finish")
        time.sleep(0.0005)


def test_session_alone_vs_mix_and_oracle(P, orc):
    XA, QA = gmm_u8(31, n=6000, m=200, n_centres=5, sigma=30.0, nq=30)
    XB, QB = gmm_f32(32, n=5000, m=64, n_centres=20, sigma=0.1, nq=30)
    dbA, dbB = P.KnnDB(dev(XA)), P.KnnDB(dev(XB))
    sess = P.Session(1 << 30)
    a, b = sess.add_db(dbA), sess.add_db(dbB)
    g = rng(33)
    reqs = []
    for i in range(60):
        use_a = i % 2 == 0
        q = QA[i // 2] if use_a else QB[i // 2]
        k = int(g.integers(1, 30))
        p = P.default_params(h=int(g.integers(0, 10)), delta=float(g.choice([0.01, 0.05])),
                             seed=int(g.integers(1 << 40)), c_exact=int(g.choice([0, 8])))
        reqs.append((a if use_a else b, q, k, p))
    # alone: one request at a time
    alone = []
    for dbid, q, k, p in reqs[:12]:
        kh = k + (p.h if p.h >= 0 else k)
        alone.append(wait(sess, sess.submit(dbid, q, k, p), kh))
    # mixed: everything in flight at once
    tickets = [sess.submit(dbid, q, k, p) for dbid, q, k, p in reqs]
    mixed = []
    for (dbid, q, k, p), t in zip(reqs, tickets):
        kh = k + (p.h if p.h >= 0 else k)
        mixed.append(wait(sess, t, kh))
    for i in range(12):
        assert alone[i][0].tolist() == mixed[i][0].tolist()
        assert alone[i][1] == mixed[i][1]
    for (dbid, q, k, p), (idx, st) in zip(reqs, mixed):
        X = XA if dbid == a else XB
        ref, rst = orc.adaptive(X, q, k, orc.make_params(h=p.h, delta=p.delta, seed=p.seed, c_exact=p.c_exact))
        assert idx.tolist() == ref.tolist()
        assert st["coord_evals"] == rst["coord_evals"]
    sess.close()


def test_session_tiny_budget_queues_requests(P, orc):
    X, Q = gmm_u8(41, n=3000, m=128, n_centres=4, sigma=30.0, nq=25)
    db = P.KnnDB(dev(X))
    sess = P.Session(2 << 20)  # room for a few queries of this DB: most requests wait on the host
    d = sess.add_db(db)
    p = P.default_params(h=5, seed=7)
    tickets = [sess.submit(d, Q[i], 5, p) for i in range(25)]
    for i, t in enumerate(tickets):
        idx, _ = wait(sess, t, 10)
        ref, _ = orc.adaptive(X, Q[i], 5, orc.make_params(h=5, seed=7))
        assert idx.tolist() == ref.tolist()
    sess.close()


def test_session_errors(P):
    from paper_1902_09465_amd import KnnError
    X, Q = gmm_u8(51, n=500, m=32, n_centres=2, sigma=30.0, nq=2)
    db = P.KnnDB(dev(X))
    sess = P.Session(64 << 20)
    d = sess.add_db(db)
    with pytest.raises(KnnError) as e:
        sess.poll(123456, 4)
    assert e.value.code == -5
    with pytest.raises(KnnError):
        sess.submit(d + 7, Q[0], 3)
    with pytest.raises(KnnError):
        sess.submit(d, Q[0], 0)
    with pytest.raises(KnnError) as e:  # the DB is held by the session
        from paper_1902_09465_amd import lib
        from paper_1902_09465_amd._lib import check
        check(lib().knn_db_destroy(db.handle))
    assert e.value.code == -4
    sess.close()


def test_session_upload_failure(P, monkeypatch):
    """A device copy that fails while a batch is uploaded, forced from the
    host (KNN_SESSION_FAIL_UPLOAD=1: the upload of the session's second
    request returns a device error, the first one already in the ring, in
    the same batch or still running from an earlier one).  Every request
    ends -- the second and later ones with the error (or, submitted after
    the failure, refused) -- with no ring entry left on a freed request;
    later submits are refused and the session closes."""
    from paper_1902_09465_amd import KnnError
    monkeypatch.setenv("KNN_SESSION_FAIL_UPLOAD", "1")
    X, Q = gmm_u8(52, n=3000, m=256, n_centres=3, sigma=30.0, nq=6)
    db = P.KnnDB(dev(X))
    sess = P.Session(64 << 20)
    d = sess.add_db(db)
    tickets, refused = [], 0
    for i in range(6):
        try:
            tickets.append(sess.submit(d, Q[i], 3))
        except KnnError:
            refused += 1
    t0 = time.time()
    outcome = []
    for t in tickets:
        while True:
            try:
                r = sess.poll(t, 3)
            except KnnError as e:
                assert e.code == -3, e.code  # KNN_EDEVICE
                outcome.append("error")
                break
            if r is not None:
                outcome.append("ok")
                break
            assert time.time() - t0 < 60, "a request never finished"
            time.sleep(0.001)
    # only the first request can have been uploaded: every other one fails
    assert outcome[1:].count("error") == len(outcome) - 1, outcome
    assert refused + outcome.count("error") >= 5
    with pytest.raises(KnnError):
        sess.submit(d, Q[0], 3)
    sess.close()
    db.close()


def test_session_serving_dbs_full_size(P, orc):
    """The three serving databases at their full sizes (50,000 x 784 u8;
    500,000 x 256 f32; 2,000,000 x 96 f32) resident in one session with a
    shared budget: 300 requests of random DB, k in 1..50, delta in {0.01,
    0.05} and seeds, all in flight together; sampled requests equal the same
    request run alone and the oracle."""
    from knn_inputs import serving_dbs
    data = serving_dbs(5000, scale=1.0)
    dbs = [P.KnnDB(dev(X)) for X, _ in data]
    sess = P.Session(48 << 30)
    ids = [sess.add_db(db) for db in dbs]
    g = rng(5200)
    reqs = []
    for _ in range(300):
        d = int(g.integers(0, 3))
        q = data[d][1][int(g.integers(0, data[d][1].shape[0]))]
        k = int(g.integers(1, 51))
        p = P.default_params(h=k, delta=0.01 if g.integers(0, 2) == 0 else 0.05, seed=int(g.integers(1 << 40)))
        reqs.append((d, q, k, p))
    tickets = [sess.submit(ids[d], q, k, p) for d, q, k, p in reqs]
    mixed = [wait(sess, t, 2 * k, timeout=120.0) for (d, q, k, p), t in zip(reqs, tickets)]
    sample = []
    for d in range(3):  # two requests of each DB
        sample += [i for i, r in enumerate(reqs) if r[0] == d][:2]
    for i in sample:
        d, q, k, p = reqs[i]
        alone = wait(sess, sess.submit(ids[d], q, k, p), 2 * k, timeout=120.0)
        assert alone[0].tolist() == mixed[i][0].tolist(), i
        assert alone[1] == mixed[i][1], i

    def ref(i):
        d, q, k, p = reqs[i]
        return orc.adaptive(data[d][0], q, k, orc.make_params(h=p.h, delta=p.delta, seed=p.seed))

    with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as ex:
        refs = list(ex.map(ref, sample))
    for i, (ridx, rst) in zip(sample, refs):
        assert mixed[i][0].tolist() == ridx.tolist(), i
        assert mixed[i][1]["coord_evals"] == rst["coord_evals"], i
    sess.close()
