"""GPU parity: the HIP adaptive path (through the C ABI) against the CPU
oracle -- returned sets, statistics and per-round state, bit-exact."""
from __future__ import annotations

import ctypes
import os

import numpy as np
import pytest
import torch

from concurrent.futures import ThreadPoolExecutor

from knn_inputs import antipodal, coherent, gmm_f32, gmm_u8, planted_corners, pm_half, rng, tiny, uniform_u8
from tests.helpers import brute_dists, contains_knn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1902_09465_amd as P
    P.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return P


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def oparams(orc, **kw):
    return orc.make_params(**kw)


def oracle_many(orc, X, Q, ks, kw, queries):
    """The oracle on several queries at once (one thread per query; the
    oracle is plain C called through ctypes, which releases the GIL)."""
    workers = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(lambda q: orc.adaptive(X, Q[q], int(ks[q]), oparams(orc, **kw)), queries))


def check_query(P, orc, db, X, q, k, **kw):
    idx, cnt, st = db.adaptive(dev(q[None]), k, P.default_params(**kw))
    ref, rst = orc.adaptive(X, q, k, oparams(orc, **kw))
    c = int(cnt.cpu()[0])
    got = idx.cpu().numpy()[0]
    assert c == len(ref), (c, len(ref))
    assert got[:c].tolist() == ref.tolist()
    assert np.all(got[c:] == -1)
    s = st[0]
    assert (int(s["coord_evals"]), int(s["rounds"]), int(s["count"]), int(s["exact_points"])) == \
        (rst["coord_evals"], rst["rounds"], rst["count"], rst["exact_points"])
    return ref, rst


@pytest.mark.parametrize("seed", range(8))
def test_tiny_config_parity(P, orc, seed):
    X, Q, planted = tiny(seed=1000 + seed)
    db = P.KnnDB(dev(X))
    for c_exact in (0, 10):
        ref, _ = check_query(P, orc, db, X, Q[0], 5, h=5, delta=0.01, seed=seed, c_exact=c_exact)
        assert set(planted.tolist()) <= set(ref.tolist())


def sampling_of(name: str) -> int:
    """Sampling mode of a parametrisation name: _norepl without replacement,
    _shared one coordinate sequence for all points (modes 0..3)."""
    return (1 if "norepl" in name else 0) + (2 if "shared" in name else 0)


@pytest.mark.parametrize("dtype", ["u8", "u8_staged", "u8_qlane", "u8_qlane_pure", "u8_qlane_pure_sparse", "f32",
                                   "u8_norepl", "u8_qlane_norepl", "u8_ungrouped_norepl", "f32_norepl",
                                   "u8_shared", "u8_shared_norepl", "u8_ungrouped_shared", "u8_qlane_shared_norepl",
                                   "u8_qlane_pure_shared", "u8_qlane_pure_shared_norepl",
                                   "u8_qlane_pure_sparse_shared_norepl", "f32_shared", "f32_shared_norepl"])
def test_per_round_state_parity(P, orc, dtype, monkeypatch):
    """After every decide step the per-point (S, flags, round) equal the oracle's."""
    g = rng(77)
    if dtype == "u8_staged":  # every sampled round reads the point rows from LDS tiles
        monkeypatch.setenv("KNN_STAGE_MIN", "4")
        monkeypatch.setenv("KNN_STAGE_ROWS", "16")
    if dtype.startswith("u8_qlane"):  # query-lane sampling even for a single slot
        monkeypatch.setenv("KNN_QL_MIN", "1")
    if "_sparse" in dtype:  # per-slot lists from round 1 on, one chunk-looping block per slot
        monkeypatch.setenv("KNN_SPARSE_DIV", "1")
        monkeypatch.setenv("KNN_SPARSE_LIST", "1")
    if dtype.startswith("u8_ungrouped"):  # the per-query sampling kernel
        monkeypatch.setenv("KNN_GROUP", "0")
    if dtype.startswith("u8"):
        X, Q = gmm_u8(77, n=5003, m=202, n_centres=6, sigma=25.0, nq=1)
    else:
        X, Q = gmm_f32(77, n=5003, m=101, n_centres=6, sigma=0.3, nq=1)
    db = P.KnnDB(dev(X))
    # candidate-exact on, except in the pure variant (fused fold + selection)
    kw = dict(h=4, delta=0.05, seed=int(g.integers(1 << 40)), b0=8, growth=1.5,
              c_exact=0 if "pure" in dtype else 3, sampling=sampling_of(dtype))
    T = orc.schedule(8, 1.5, 1.0, X.shape[1])
    for r in range(1, len(T) + 2):
        S, fl, ri = db.adaptive_state(dev(Q), 6, P.default_params(**kw), r)
        _, _, (So, flo, rio) = orc.adaptive(X, Q[0], 6, oparams(orc, **kw), stop_after=r, dump=True)
        assert np.array_equal(fl, flo), f"round {r}: flags differ"
        assert np.array_equal(S, So), f"round {r}: sums differ"
        assert np.array_equal(ri, rio), f"round {r}: round index differs"


@pytest.mark.parametrize("m", [2048, 512])
def test_point_major_mixed_widths(P, orc, monkeypatch, m):
    """Point-major batch (query lanes, no candidate-exact, dense flags) where a
    pair is accepted rounds before the rest are decided: the selection tiles
    that hold it mix widths (at m = 2048 in sampled rounds, at m = 512 also
    in the exact round, beside exact pairs).  Every round's state equals the
    oracle's, and so does the result."""
    monkeypatch.setenv("KNN_QL_MIN", "1")
    monkeypatch.setenv("KNN_SPARSE_DIV", "0")
    g = rng(31)
    n = 3000
    d = np.concatenate([[0.002, 0.1], g.uniform(0.15, 0.2, 300), g.uniform(0.3, 0.5, n - 302)])
    d = d[g.permutation(n)]
    X, Q, _ = pm_half(31, n, m, d)
    db = P.KnnDB(dev(X))
    kw = dict(h=2, delta=0.05, seed=5, alpha_kind=2, c_alpha=0.01, c_exact=0)
    T = orc.schedule(64, 2.0, 1.0, m)
    mixed_rounds, mixed_exact = 0, False
    for r in range(1, len(T) + 2):
        S, fl, ri = db.adaptive_state(dev(Q), 2, P.default_params(**kw), r)
        _, _, (So, flo, rio) = orc.adaptive(X, Q[0], 2, oparams(orc, **kw), stop_after=r, dump=True)
        assert np.array_equal(fl, flo), f"round {r}: flags differ"
        assert np.array_equal(S, So), f"round {r}: sums differ"
        assert np.array_equal(ri, rio), f"round {r}: round index differs"
        late = (flo & 2) != 0
        late &= (flo & 1) == 0
        exact = (flo & 1) != 0
        mixed_rounds += int(late.any() and ((flo == 0).any() or exact.any()))
        mixed_exact |= bool(late.any() and exact.any())
    assert mixed_rounds >= 1, "the instance never mixed widths"
    if m == 512:
        assert mixed_exact, "the exact round never saw a pair accepted earlier"
    check_query(P, orc, db, X, Q[0], 2, **kw)


def _decisive_batch():
    """80 queries over one database of corners (n = 6000, m = 1024), each with
    its own near points at its own distance, k cycling over 1, 5, 10, 20."""
    nq = 80
    ks = np.array([(1, 5, 10, 20)[j % 4] for j in range(nq)], dtype=np.int32)
    gaps = rng(5).uniform(0.02, 0.4, size=nq)
    X, Q = planted_corners(91, 6000, 1024, nq, ks, gaps)
    return X, Q, ks


DECISIVE_KW = dict(h=-1, delta=0.01, seed=2024, alpha_kind=2, c_alpha=0.1, c_exact=0)


@pytest.mark.parametrize("sparse_div,sampling", [("16", 0), ("0", 0), ("16", 2), ("0", 2), ("16", 3), ("0", 3)])
def test_point_major_batch_decides_in_sampled_rounds(P, orc, monkeypatch, sparse_div, sampling):
    """The launch shape the benchmark times -- one seed shared by many queries,
    k + 1 <= 64, no candidate-exact: query-lane sampling, point-major sums,
    four-slot selection tiles and 64-slot decide tiles (80 queries: two decide
    tiles) -- on data where sampled rounds discard and accept points and the
    queries decide differently.  Every query's set and statistics equal the
    oracle's; the per-round state of slots 0, 1, 64 and 79 equals the
    oracle's after every decide step.  With the default switch (slots whose
    undecided set falls to n/16 continue on per-slot lists) and with slots
    kept dense to the end.  With one coordinate sequence for all points
    (sampling 2 and 3) the rounds run as int8 products over the gathered
    coordinates (without replacement the exact round adds the rest)."""
    monkeypatch.setenv("KNN_SPARSE_DIV", sparse_div)
    X, Q, ks = _decisive_batch()
    n = X.shape[0]
    db = P.KnnDB(dev(X))
    kw = dict(DECISIVE_KW, sampling=sampling)
    p = P.default_params(**kw)
    idx, cnt, st = db.adaptive(dev(Q), ks, p)
    idx, cnt = idx.cpu().numpy(), cnt.cpu().numpy()
    refs = oracle_many(orc, X, Q, ks, kw, range(len(ks)))
    for q, (ref, rst) in enumerate(refs):
        assert idx[q, :cnt[q]].tolist() == ref.tolist(), q
        assert (int(st[q]["coord_evals"]), int(st[q]["rounds"]), int(st[q]["count"]),
                int(st[q]["exact_points"])) == (rst["coord_evals"], rst["rounds"], rst["count"],
                                                rst["exact_points"]), q
    # decisions are taken before the exact round for most queries, after a
    # different number of rounds
    assert sum(r[1]["exact_points"] < n for r in refs) >= 60
    assert len({r[1]["rounds"] for r in refs}) >= 3
    Qd = dev(Q)
    for slot in (0, 1, 64, 79):
        for r in range(1, refs[slot][1]["rounds"] + 1):
            S, fl, ri = db.adaptive_state(Qd, ks, p, r, query=slot)
            _, _, (So, flo, rio) = orc.adaptive(X, Q[slot], int(ks[slot]), oparams(orc, **kw),
                                                stop_after=r, dump=True)
            assert np.array_equal(fl, flo), f"slot {slot} round {r}: flags differ"
            assert np.array_equal(S, So), f"slot {slot} round {r}: sums differ"
            assert np.array_equal(ri, rio), f"slot {slot} round {r}: round index differs"


@pytest.mark.parametrize("sampling", [0, 3])
def test_point_major_batch_wide_k(P, orc, monkeypatch, sampling):
    """Point-major batches with k + 1 up to 128: selection lists of two
    registers per lane.  80 queries with k cycling over 1, 63, 64, 100, 127
    (ranks k - 1 and k on either side of the 64-lane boundary) on data where
    sampled rounds decide; every query's set and statistics equal the
    oracle's, and so does the per-round state of slots 2 (k = 64), 3
    (k = 100) and 4 (k = 127)."""
    monkeypatch.setenv("KNN_SPARSE_DIV", "0")  # every round on the point-major kernels
    nq = 80
    ks = np.array([(1, 63, 64, 100, 127)[j % 5] for j in range(nq)], dtype=np.int32)
    gaps = rng(6).uniform(0.02, 0.3, size=nq)
    X, Q = planted_corners(92, 12000, 1024, nq, ks, gaps)
    db = P.KnnDB(dev(X))
    kw = dict(DECISIVE_KW, sampling=sampling)
    p = P.default_params(**kw)
    idx, cnt, st = db.adaptive(dev(Q), ks, p)
    idx, cnt = idx.cpu().numpy(), cnt.cpu().numpy()
    refs = oracle_many(orc, X, Q, ks, kw, range(nq))
    for q, (ref, rst) in enumerate(refs):
        assert idx[q, :cnt[q]].tolist() == ref.tolist(), q
        assert (int(st[q]["coord_evals"]), int(st[q]["rounds"]), int(st[q]["exact_points"])) == \
            (rst["coord_evals"], rst["rounds"], rst["exact_points"]), q
    assert sum(r[1]["exact_points"] < X.shape[0] for r in refs) >= 40
    Qd = dev(Q)
    for slot in (2, 3, 4):
        for r in range(1, refs[slot][1]["rounds"] + 1):
            S, fl, ri = db.adaptive_state(Qd, ks, p, r, query=slot)
            _, _, (So, flo, rio) = orc.adaptive(X, Q[slot], int(ks[slot]), oparams(orc, **kw), stop_after=r,
                                                dump=True)
            assert np.array_equal(fl, flo), f"slot {slot} round {r}: flags differ"
            assert np.array_equal(S, So), f"slot {slot} round {r}: sums differ"
            assert np.array_equal(ri, rio), f"slot {slot} round {r}: round index differs"


@pytest.mark.parametrize("variant", ["pure", "cexact", "b0_4", "lemma", "calpha", "theta"])
def test_variants_parity(P, orc, variant):
    X, Q = gmm_u8(5, n=3000, m=300, n_centres=4, sigma=20.0, nq=3)
    db = P.KnnDB(dev(X))
    kw = dict(pure=dict(), cexact=dict(c_exact=8), b0_4=dict(b0=4, growth=3.0),
              lemma=dict(alpha_kind=1), calpha=dict(alpha_kind=2, c_alpha=0.01),
              theta=dict(theta_exact=0.4, c_exact=2))[variant]
    for qi in range(3):
        check_query(P, orc, db, X, Q[qi], 7, h=3, delta=0.02, seed=qi, **kw)


def test_batched_mixed_k_and_params(P, orc):
    """One call, queries of different k, h, delta and seed: each equals the
    oracle run alone (the slot engine shares nothing between queries)."""
    X, Q = gmm_u8(9, n=4097, m=128, n_centres=8, sigma=30.0, nq=40)
    db = P.KnnDB(dev(X))
    g = rng(9)
    ks = g.integers(1, 20, size=40).astype(np.int32)
    plist = [P.default_params(h=int(g.integers(0, 8)), delta=float(g.choice([0.01, 0.05, 0.2])),
                              seed=int(g.integers(1 << 62)), c_exact=int(g.choice([0, 0, 5])))
             for _ in range(40)]
    idx, cnt, st = db.adaptive(dev(Q), ks, plist)
    idx, cnt = idx.cpu().numpy(), cnt.cpu().numpy()
    for q in range(40):
        p = plist[q]
        ref, rst = orc.adaptive(X, Q[q], int(ks[q]), oparams(
            orc, h=p.h, delta=p.delta, seed=p.seed, c_exact=p.c_exact))
        assert idx[q, :cnt[q]].tolist() == ref.tolist(), q
        assert int(st[q]["coord_evals"]) == rst["coord_evals"]


def test_more_queries_than_slots(P, orc):
    """Slots are recycled on the device when the queries do not fit at once."""
    X, Q = gmm_u8(11, n=2500, m=96, n_centres=5, sigma=30.0, nq=23)
    db = P.KnnDB(dev(X))
    os.environ["KNN_MAX_SLOTS"] = "4"
    try:
        idx, cnt, _ = db.adaptive(dev(Q), 5, P.default_params(h=5, seed=3))
    finally:
        del os.environ["KNN_MAX_SLOTS"]
    idx, cnt = idx.cpu().numpy(), cnt.cpu().numpy()
    for q in range(23):
        ref, _ = orc.adaptive(X, Q[q], 5, oparams(orc, h=5, seed=3))
        assert idx[q, :cnt[q]].tolist() == ref.tolist()


KNOBS = ([{"KNN_LPP": v} for v in ("1", "2", "4", "8", "16", "32", "64")] +
         [{"KNN_QL_MIN": "1"}, {"KNN_QL_MIN": "1", "KNN_GROUP": "0"}] +
         # query-lane batches whose slots switch to per-slot lists after round 0, or never
         [{"KNN_QL_MIN": "1", "KNN_SPARSE_DIV": "1"}, {"KNN_QL_MIN": "1", "KNN_SPARSE_DIV": "0"}] +
         # ... whose per-slot kernels then run one block per slot, looping over the list's chunks
         [{"KNN_QL_MIN": "1", "KNN_SPARSE_DIV": "1", "KNN_SPARSE_LIST": "1"}] +
         # prefetch depth of the exact round's tiles
         [{"KNN_QL_MIN": "1", "KNN_EXACT_PF": v} for v in ("4", "6")] +
         [{"KNN_CH_SAMPLE": v} for v in ("64", "256", "4096")] + [{"KNN_GROUP": "0"}] +
         # every sampled round from point rows staged in LDS, at each tile height
         [{"KNN_STAGE_MIN": "4", "KNN_STAGE_ROWS": v} for v in ("8", "16", "32", "64")] +
         [{"KNN_STAGE_MIN": "4", "KNN_STAGE_ROWS": "8", "KNN_CH_SAMPLE": "100"}])


@pytest.mark.parametrize("knob", KNOBS, ids=lambda k: ",".join(f"{a}={b}" for a, b in k.items()))
@pytest.mark.parametrize("m", [256, 200])
def test_performance_knobs_do_not_change_results(P, orc, knob, m):
    X, Q = gmm_u8(13, n=3001, m=m, n_centres=5, sigma=20.0, nq=4)
    db = P.KnnDB(dev(X))
    base = db.adaptive(dev(Q), 6, P.default_params(seed=1, c_exact=4))
    os.environ.update(knob)
    try:
        alt = db.adaptive(dev(Q), 6, P.default_params(seed=1, c_exact=4))
    finally:
        for k in knob:
            del os.environ[k]
    assert torch.equal(base[0], alt[0]) and torch.equal(base[1], alt[1])
    assert np.array_equal(base[2], alt[2])


def test_f32_parity(P, orc):
    X, Q = gmm_f32(21, n=3000, m=100, n_centres=10, sigma=0.2, nq=4)
    db = P.KnnDB(dev(X))
    for qi in range(4):
        ref, _ = check_query(P, orc, db, X, Q[qi], 5, h=5, delta=0.05, seed=qi, c_exact=(qi % 2) * 10)
        assert contains_knn(ref, brute_dists(X, Q[qi]), 5, rtol=1e-6)


def test_worked_example(P, orc):
    X, Q, where = antipodal()
    db = P.KnnDB(dev(X))
    idx, cnt, st = db.adaptive(dev(Q), 5, P.default_params(h=5, delta=0.01, seed=123))
    assert sorted(idx.cpu().numpy()[0, :int(cnt[0])].tolist()) == where.tolist()
    assert int(st[0]["coord_evals"]) == 256_000 and int(st[0]["rounds"]) == 3
    idx, cnt, st = db.adaptive(dev(Q), 5, P.default_params(h=5, delta=0.01, seed=9, c_exact=10))
    assert int(st[0]["coord_evals"]) == 74_240


def test_edge_cases(P, orc):
    # n <= k + h: everything, no evaluations
    X, Q = uniform_u8(1, 7, 16)
    db = P.KnnDB(dev(X))
    idx, cnt, st = db.adaptive(dev(Q), 4, P.default_params(h=3))
    assert int(cnt[0]) == 7 and idx.cpu().numpy()[0].tolist() == list(range(7))
    # all points identical: every distance ties (oversized stop path)
    X = np.full((300, 40), 7, dtype=np.uint8)
    q = np.full((40,), 9, dtype=np.uint8)
    db = P.KnnDB(dev(X))
    check_query(P, orc, db, X, q, 4, h=2, seed=1)
    # coherent data, k = 1, h = 0
    X, Q = coherent(5, 1500, 100)
    db = P.KnnDB(dev(X))
    check_query(P, orc, db, X, Q[0], 1, h=0, seed=2)
    # f32 with zero range: first k + h indices
    Xf = np.zeros((50, 8), dtype=np.float32)
    dbf = P.KnnDB(dev(Xf))
    idx, cnt, _ = dbf.adaptive(dev(Xf[:1]), 3, P.default_params(h=2))
    assert idx.cpu().numpy()[0, :5].tolist() == list(range(5))


def test_invalid_arguments_raise(P):
    from paper_1902_09465_amd import KnnError
    X, Q = uniform_u8(1, 100, 16)
    db = P.KnnDB(dev(X))
    with pytest.raises(KnnError):
        db.adaptive(dev(Q), 0)
    with pytest.raises(KnnError):
        db.adaptive(dev(Q), 3, P.default_params(b0=6))
    with pytest.raises(KnnError):
        db.adaptive(dev(Q), 3, P.default_params(h=5000))


def test_containment_many_seeds(P, orc):
    """Theorem 1 on the GPU path: over many seeds every returned set contains
    the k nearest neighbours (tie-aware) and has at most k+h points."""
    X, Q, _ = tiny(seed=1500, n=1200, m=256)
    d = brute_dists(X, Q[0])
    db = P.KnnDB(dev(X))
    plist = [P.default_params(h=5, delta=0.01, seed=s, c_exact=(s % 2) * 10) for s in range(200)]
    Qs = np.repeat(Q, 200, axis=0)
    idx, cnt, _ = db.adaptive(dev(Qs), 5, plist)
    idx, cnt = idx.cpu().numpy(), cnt.cpu().numpy()
    for s in range(200):
        assert cnt[s] <= 10 and contains_knn(idx[s, :cnt[s]], d, 5)


def test_grouped_shared_seed_batch(P, orc):
    """64 queries with one seed: the sampling kernel serves them sixteen at a
    time (shared draws and gathers; exact round on the matrix cores).  Every
    query equals the oracle, and equals the ungrouped path."""
    X, Q = gmm_u8(61, n=20011, m=1000, n_centres=12, sigma=30.0, nq=64)
    db = P.KnnDB(dev(X))
    p = P.default_params(h=10, delta=0.01, seed=99, c_exact=0)
    idx, cnt, st = db.adaptive(dev(Q), 10, p)
    os.environ["KNN_GROUP"] = "0"
    try:
        idx2, cnt2, st2 = db.adaptive(dev(Q), 10, p)
    finally:
        del os.environ["KNN_GROUP"]
    assert torch.equal(idx, idx2) and np.array_equal(st, st2)
    os.environ["KNN_STAGE_MIN"] = "4"  # rows staged in LDS in every sampled round (m = 1000: byte copies)
    try:
        idx3, cnt3, st3 = db.adaptive(dev(Q), 10, p)
    finally:
        del os.environ["KNN_STAGE_MIN"]
    assert torch.equal(idx, idx3) and np.array_equal(st, st3)
    os.environ["KNN_QL"] = "0"  # the default here is query-lane sampling (64 slots); compare with it off
    try:
        idx4, cnt4, st4 = db.adaptive(dev(Q), 10, p)
    finally:
        del os.environ["KNN_QL"]
    assert torch.equal(idx, idx4) and np.array_equal(st, st4)
    idx, cnt = idx.cpu().numpy(), cnt.cpu().numpy()
    for q in range(0, 64, 9):
        ref, rst = orc.adaptive(X, Q[q], 10, oparams(orc, h=10, delta=0.01, seed=99))
        assert idx[q, :cnt[q]].tolist() == ref.tolist(), q
        assert int(st[q]["coord_evals"]) == rst["coord_evals"]


def test_graph_replays_equal_eager(P, orc):
    """Repeated batches of one shape replay a captured launch sequence on a
    cached engine.  Several replays with different queries, with eager work
    in between, each equal the eager (uncaptured) result."""
    X, Q = gmm_u8(71, n=6007, m=300, n_centres=6, sigma=25.0, nq=192)
    db = P.KnnDB(dev(X))
    p = P.default_params(h=6, delta=0.05, seed=5)
    batches = [dev(Q[:96]), dev(Q[96:]), dev(Q[:96][::-1].copy())]
    os.environ["KNN_GRAPH"] = "0"
    try:
        eager = [db.adaptive(b, 6, p) for b in batches]
    finally:
        del os.environ["KNN_GRAPH"]
    for rep in range(3):
        for b, ref in zip(batches, eager):
            got = db.adaptive(b, 6, p)
            torch.cuda.synchronize()
            assert torch.equal(got[0], ref[0]) and torch.equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])
            _ = db.naive(b, 3)  # eager work between replays
    # the same shape with another seed (and with a shared coordinate sequence)
    # replays nothing captured for the first seed
    for p2 in (P.default_params(h=6, delta=0.05, seed=6), P.default_params(h=6, delta=0.05, seed=6, sampling=3)):
        got = db.adaptive(batches[0], 6, p2)
        os.environ["KNN_GRAPH"] = "0"
        try:
            ref = db.adaptive(batches[0], 6, p2)
        finally:
            del os.environ["KNN_GRAPH"]
        assert torch.equal(got[0], ref[0]) and np.array_equal(got[2], ref[2])
        o = orc.adaptive(X, Q[7], 6, oparams(orc, h=6, delta=0.05, seed=6, sampling=p2.sampling))[0]
        assert got[0][7, :got[1][7]].cpu().tolist() == o.tolist()
    # a batch of another shape rebuilds the plan, then the first shape again
    other = db.adaptive(dev(Q[:50]), 6, p)
    ref50 = orc.adaptive(X, Q[3], 6, oparams(orc, h=6, delta=0.05, seed=5))[0]
    assert other[0][3, :other[1][3]].cpu().tolist() == ref50.tolist()
    got = db.adaptive(batches[0], 6, p)
    assert torch.equal(got[0], eager[0][0])


def test_batches_queued_without_sync(P, orc, monkeypatch):
    """A batch whose queries all fit is stream-ordered: batches of different
    queries and sizes queued back to back, with no synchronisation between
    them, equal the same batches run one at a time (the host staging buffer
    is reused and regrown, the engine arenas come from the pool)."""
    monkeypatch.setenv("KNN_GRAPH", "0")  # the eager engine
    X, Q = gmm_u8(73, n=6007, m=300, n_centres=6, sigma=25.0, nq=200)
    db = P.KnnDB(dev(X))
    p = P.default_params(h=6, delta=0.05, seed=9)
    batches = [dev(Q[:96]), dev(Q[96:200]), dev(Q[:40]), dev(Q[50:146])]
    ref = []
    for b in batches:
        i, c, _ = db.adaptive(b, 6, p, with_stats=False)
        torch.cuda.synchronize()
        ref.append((i.clone(), c.clone()))
    got = [db.adaptive(b, 6, p, with_stats=False) for b in batches]
    torch.cuda.synchronize()
    for (gi, gc, _), (ri, rc) in zip(got, ref):
        assert torch.equal(gi, ri) and torch.equal(gc, rc)
    o = orc.adaptive(X, Q[100], 6, oparams(orc, h=6, delta=0.05, seed=9))[0]
    assert got[1][0][4, :got[1][1][4]].cpu().tolist() == o.tolist()


def test_autotune_keeps_results(P, orc):
    """The autotuner times every knob candidate, checks that all of them give
    the same output, keeps the fastest, and later calls still equal the oracle."""
    X, Q = gmm_u8(73, n=5003, m=256, n_centres=5, sigma=25.0, nq=80)
    db = P.KnnDB(dev(X))
    p = P.default_params(h=5, seed=9)
    rep = db.autotune(dev(Q), 5, p, reps=1, schedule_report=True)
    assert {"default", "grouped", "per-query", "default no-graph"} <= set(rep)
    assert any(k.startswith("schedule b0=16") for k in rep)
    assert all(v > 0 for v in rep.values())
    idx, cnt, st = db.adaptive(dev(Q), 5, p)
    idx, cnt = idx.cpu().numpy(), cnt.cpu().numpy()
    for q in (0, 41, 79):
        ref, rst = orc.adaptive(X, Q[q], 5, oparams(orc, h=5, seed=9))
        assert idx[q, :cnt[q]].tolist() == ref.tolist()
        assert int(st[q]["coord_evals"]) == rst["coord_evals"]


@pytest.mark.parametrize("c_alpha", [0.01, 0.3])
def test_subspace_calpha_parity(P, orc, c_alpha):
    """Section 5's synthetic data (x = cQy, float) with the C_alpha width: the
    returned set and the evaluation count equal the oracle's."""
    from knn_inputs import subspace
    X, Q = subspace(4242, n=300, m=2048, p=10, nq=3)
    db = P.KnnDB(dev(X))
    kw = dict(h=10, delta=0.001, seed=17, alpha_kind=2, c_alpha=c_alpha)
    idx, cnt, st = db.adaptive(dev(Q), 10, P.default_params(**kw))
    idx, cnt = idx.cpu().numpy(), cnt.cpu().numpy()
    for q in range(3):
        ref, rst = orc.adaptive(X, Q[q], 10, oparams(orc, **kw))
        assert idx[q, :cnt[q]].tolist() == ref.tolist(), q
        assert int(st[q]["coord_evals"]) == rst["coord_evals"]


@pytest.mark.parametrize("pdim", [10, 1000])
def test_subspace_paper_shape_parity(P, orc, pdim):
    """Section 5 at the paper's shape: n = 1000 points of m = 12288
    coordinates (x = cQy with subspace dimension p), k = h = 10,
    delta = 0.001, the C_alpha width at 0.01; three trials each with its own
    data and seed (one query per call, as in the experiment).  Sets and
    statistics equal the oracle's."""
    from knn_inputs import subspace
    for trial in range(3):
        X, Q = subspace(10_000 + 97 * pdim + trial, n=1000, m=12288, p=pdim, nq=1)
        db = P.KnnDB(dev(X))
        kw = dict(h=10, delta=0.001, seed=trial + 1, alpha_kind=2, c_alpha=0.01)
        check_query(P, orc, db, X, Q[0], 10, **kw)
        db.close()


def test_uneven_config_sampled(P, orc):
    """The uneven workload at full size (n = 250,000 x m = 1024, 4,096 queries,
    half easy / half hard, k cycling over 1, 10, 100, one seed): every query's
    set contains its true k-NN (against the exact scan, tie-aware), and sampled
    easy and hard queries of each k equal the oracle exactly."""
    from knn_inputs import uneven
    X, Q, ks = uneven(4000)
    db = P.KnnDB(dev(X))
    Qd = dev(Q)
    p = P.default_params(h=-1, delta=0.01, seed=4001)
    idx, cnt, st = db.adaptive(Qd, ks, p)
    idx_c, cnt_c = idx.cpu().numpy(), cnt.cpu().numpy()
    # containment for all queries, per k, against the int8-MFMA exact scan
    for kk in (1, 10, 100):
        sel = np.nonzero(ks == kk)[0]
        nidx, ndist = db.naive(Qd[torch.from_numpy(sel).cuda()], kk)
        nidx, ndist = nidx.cpu().numpy(), ndist.cpu().numpy()
        for row, qi in enumerate(sel):
            got = idx_c[qi, :cnt_c[qi]]
            dk = ndist[row, kk - 1]
            strict = set(nidx[row][ndist[row] < dk].tolist())
            assert strict <= set(got.tolist()), (qi, kk)
            dg = ((X[got].astype(np.int64) - Q[qi].astype(np.int64)) ** 2).sum(1)
            assert (dg <= dk).sum() >= kk, (qi, kk)
    n_easy = Q.shape[0] // 2
    for qi in (0, 1, 2, n_easy, n_easy + 1, n_easy + 2):
        ref, rst = orc.adaptive(X, Q[qi], int(ks[qi]), oparams(orc, h=-1, delta=0.01, seed=4001))
        assert idx_c[qi, :cnt_c[qi]].tolist() == ref.tolist(), qi
        assert int(st[qi]["coord_evals"]) == rst["coord_evals"], qi


@pytest.mark.parametrize("sampling", [1, 2, 3])
def test_sampling_modes_batched(P, orc, sampling):
    """Sampling without replacement (1), or one coordinate sequence for all
    points (2: with replacement, 3: without; the rounds as products over the
    gathered coordinates), 64 queries with one seed, against the oracle, the
    grouped and the per-query paths; knob invariance."""
    X, Q = gmm_u8(81, n=9001, m=500, n_centres=8, sigma=30.0, nq=64)
    db = P.KnnDB(dev(X))
    kw = dict(h=10, delta=0.01, seed=77, sampling=sampling)
    base = db.adaptive(dev(Q), 10, P.default_params(**kw))
    for env in ({"KNN_QL": "0"}, {"KNN_QL": "0", "KNN_GROUP": "0"}, {"KNN_QL_MIN": "1", "KNN_CH_SAMPLE": "64"}):
        os.environ.update(env)
        try:
            alt = db.adaptive(dev(Q), 10, P.default_params(**kw))
        finally:
            for e in env:
                del os.environ[e]
        assert torch.equal(base[0], alt[0]) and torch.equal(base[1], alt[1]) and np.array_equal(base[2], alt[2])
    idx, cnt = base[0].cpu().numpy(), base[1].cpu().numpy()
    for q in (0, 31, 63):
        ref, rst = orc.adaptive(X, Q[q], 10, oparams(orc, **kw))
        assert idx[q, :cnt[q]].tolist() == ref.tolist(), q
        assert int(base[2][q]["coord_evals"]) == rst["coord_evals"]


@pytest.mark.parametrize("sampling", [2, 3])
@pytest.mark.parametrize("metric", ["l2", "l1"])
def test_f32_shared_sequence_batched(P, orc, monkeypatch, sampling, metric):
    """A float batch of 48 queries with one seed and one coordinate sequence
    for all points: every round is a tile pass over the point and query
    copies gathered at the sequence (without replacement the exact round adds
    the columns not yet sampled).  Equal to the same batch with the copies
    switched off (per-pair draws of the same sequence), and to the oracle on
    sampled queries (indices and statistics)."""
    X, Q = gmm_f32(83, n=6007, m=300, n_centres=8, sigma=0.3, nq=48)
    db = P.KnnDB(dev(X), metric=metric)
    kw = dict(h=8, delta=0.02, seed=91, sampling=sampling, b0=16, growth=2.0)
    lib = P.lib()

    def gathers():  # launches of the sequence gather (profiling kind 8) since the last enable
        ms, nl, u = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        P._lib.check(lib.knn_prof_read(8, ctypes.byref(ms), ctypes.byref(nl), ctypes.byref(u)))
        return nl.value

    P._lib.check(lib.knn_prof_enable(1))
    try:
        base = db.adaptive(dev(Q), 8, P.default_params(**kw))
        assert gathers() == 1, "the batch did not run on the gathered copies"
        monkeypatch.setenv("KNN_SEQ", "0")
        P._lib.check(lib.knn_prof_enable(1))
        alt = db.adaptive(dev(Q), 8, P.default_params(**kw))
        assert gathers() == 0
    finally:
        P._lib.check(lib.knn_prof_enable(0))
    assert torch.equal(base[0], alt[0]) and torch.equal(base[1], alt[1]) and np.array_equal(base[2], alt[2])
    idx, cnt = base[0].cpu().numpy(), base[1].cpu().numpy()
    refs = oracle_many(orc, X, Q, [8] * 48, dict(kw), range(0, 48, 7)) if metric == "l2" else \
        [orc.adaptive(X, Q[q], 8, oparams(orc, **kw), metric=1) for q in range(0, 48, 7)]
    for q, (ref, rst) in zip(range(0, 48, 7), refs):
        assert idx[q, :cnt[q]].tolist() == ref.tolist(), q
        assert int(base[2][q]["coord_evals"]) == rst["coord_evals"], q
        assert int(base[2][q]["rounds"]) == rst["rounds"], q


@pytest.mark.parametrize("n,m,k,h,sampling,metric", [(257, 3, 20, 20, 3, "l2"), (130, 1, 5, 3, 2, "l2"),
                                                  (300, 70, 1, 0, 3, "l1"), (1000, 129, 33, 10, 2, "l1")])
def test_f32_shared_sequence_odd_shapes(P, orc, n, m, k, h, sampling, metric):
    """The fp32 shared-sequence tiles on ragged shapes (point and column
    counts off the tile sizes, m = 1, k = 1 with h = 0, k + h near n):
    every query of a 21-query batch equals the oracle and the per-pair path."""
    g = rng(n + 7 * m + k)
    X = g.standard_normal((n, m)).astype(np.float32)
    Q = (X[g.integers(0, n, size=21)] + 0.3 * g.standard_normal((21, m))).astype(np.float32)
    db = P.KnnDB(dev(X), metric=metric)
    kw = dict(h=h, delta=0.05, seed=29, sampling=sampling, b0=4, growth=2.0)
    base = db.adaptive(dev(Q), k, P.default_params(**kw))
    os.environ["KNN_SEQ"] = "0"
    try:
        alt = db.adaptive(dev(Q), k, P.default_params(**kw))
    finally:
        del os.environ["KNN_SEQ"]
    assert torch.equal(base[0], alt[0]) and torch.equal(base[1], alt[1]) and np.array_equal(base[2], alt[2])
    idx, cnt = base[0].cpu().numpy(), base[1].cpu().numpy()
    for q in range(21):
        ref, rst = orc.adaptive(X, Q[q], k, oparams(orc, **kw), metric=1 if metric == "l1" else 0)
        assert idx[q, :cnt[q]].tolist() == ref.tolist(), q
        assert int(base[2][q]["coord_evals"]) == rst["coord_evals"], q


@pytest.mark.parametrize("dtype,sampling", [("u8", 3), ("u8", 0), ("f32", 3), ("f32", 1)])
def test_batch_larger_than_slots_in_chunks(P, orc, monkeypatch, dtype, sampling):
    """A one-seed batch with more queries than slots runs as consecutive
    lock-step batches (equal sizes, the last one smaller and uncaptured):
    results and statistics equal those of the batch run at once, on both a
    first and a repeated (replayed) call, and the oracle's on a few queries."""
    if dtype == "u8":
        X, Q = gmm_u8(85, n=4001, m=256, n_centres=6, sigma=30.0, nq=100)
    else:
        X, Q = gmm_f32(85, n=4001, m=96, n_centres=6, sigma=0.3, nq=100)
    db = P.KnnDB(dev(X))
    kw = dict(h=6, delta=0.05, seed=17, sampling=sampling)
    base = db.adaptive(dev(Q), 6, P.default_params(**kw))
    for cap in ("33", "40"):  # four chunks of 25; chunks of 34, 34 and 32
        monkeypatch.setenv("KNN_MAX_SLOTS", cap)
        for _ in range(2):
            got = db.adaptive(dev(Q), 6, P.default_params(**kw))
            assert torch.equal(base[0], got[0]) and torch.equal(base[1], got[1]), cap
            assert np.array_equal(base[2], got[2]), cap
    idx, cnt = base[0].cpu().numpy(), base[1].cpu().numpy()
    for q in (0, 34, 99):
        ref, rst = orc.adaptive(X, Q[q], 6, oparams(orc, **kw))
        assert idx[q, :cnt[q]].tolist() == ref.tolist(), q
        assert int(base[2][q]["coord_evals"]) == rst["coord_evals"], q


@pytest.mark.parametrize("data", ["hard", "easy"])
def test_shared_sequence_gather_in_parts(P, orc, data):
    """Sampling 3 at m = 8192 (T = 64 ... 4096, then the exact round): the
    points' rows at the sequence's coordinates are gathered in three parts,
    the first rounds' columns (T <= 2048) up front, T = 4096's before its
    round if a slot still runs, the exact round's before it if a slot is
    still dense.  On uniform rows every point of every query reaches the
    exact round, so every part is gathered and read; on easy corners every
    query settles by T = 1024 and the later parts are skipped on the device.
    Every query's set and statistics equal the oracle's."""
    from knn_inputs import easy_corners
    n, m, nq, k = 1500, 8192, 70, 5
    if data == "hard":
        g = rng(4242)
        X = g.integers(0, 256, (n, m), dtype=np.uint8)
        Q = g.integers(0, 256, (nq, m), dtype=np.uint8)
    else:
        X, Q = easy_corners(4243, n, m, nq, k)
    db = P.KnnDB(dev(X))
    kw = dict(h=k, delta=0.01, seed=21, sampling=3)
    idx, cnt, st = db.adaptive(dev(Q), k, P.default_params(**kw))
    idx, cnt = idx.cpu().numpy(), cnt.cpu().numpy()
    refs = oracle_many(orc, X, Q, [k] * nq, kw, range(nq))
    for q, (ref, rst) in enumerate(refs):
        assert idx[q, :cnt[q]].tolist() == ref.tolist(), q
        assert (int(st[q]["coord_evals"]), int(st[q]["rounds"]), int(st[q]["count"]), int(st[q]["exact_points"])) == \
            (rst["coord_evals"], rst["rounds"], rst["count"], rst["exact_points"]), q
    exact = [rst["exact_points"] for _, rst in refs]
    if data == "hard":
        assert all(e == n for e in exact)  # the exact round's columns were gathered and used
    else:
        assert all(e == 0 for e in exact) and max(rst["rounds"] for _, rst in refs) <= 6
    db.close()


@pytest.mark.parametrize("m,sampling,data", [(1001, 3, "gmm"), (1001, 2, "gmm"), (8191, 3, "hard")])
def test_shared_sequence_unaligned_rows(P, orc, m, sampling, data):
    """A borrowed point matrix that starts 3 bytes past a 16-byte boundary
    (the DB takes an aligned copy of it; the bytes around it are 0xEE, so a
    copy that took any of them would change the sums), with odd m: the point
    rows start at every offset modulo 16 and the last row's trailing word
    reaches past the matrix.  The staged gather copies each row as the
    aligned words that cover it, the bytes past the matrix one by one.  At
    m = 8191 on uniform rows every query reaches the exact round, so all
    three parts of the gather run.  Every query's set and statistics equal
    the oracle's."""
    n, nq, k = (3001, 40, 5) if m == 1001 else (1500, 40, 5)
    if data == "hard":
        g = rng(4244)
        X = g.integers(0, 256, (n, m), dtype=np.uint8)
        Q = g.integers(0, 256, (nq, m), dtype=np.uint8)
    else:
        X, Q = gmm_u8(4245, n=n, m=m, n_centres=6, sigma=25.0, nq=nq)
    off = 3
    buf = torch.full((X.size + off + 29,), 0xEE, dtype=torch.uint8, device="cuda")
    buf[off:off + X.size] = dev(X.reshape(-1))
    Xd = buf[off:off + X.size].view(n, m)
    assert Xd.data_ptr() % 16 == off
    db = P.KnnDB(Xd)
    kw = dict(h=k, delta=0.01, seed=23, sampling=sampling)
    idx, cnt, st = db.adaptive(dev(Q), k, P.default_params(**kw))
    idx, cnt = idx.cpu().numpy(), cnt.cpu().numpy()
    refs = oracle_many(orc, X, Q, [k] * nq, kw, range(nq))
    for q, (ref, rst) in enumerate(refs):
        assert idx[q, :cnt[q]].tolist() == ref.tolist(), q
        assert (int(st[q]["coord_evals"]), int(st[q]["rounds"]), int(st[q]["count"]), int(st[q]["exact_points"])) == \
            (rst["coord_evals"], rst["rounds"], rst["count"], rst["exact_points"]), q
    if data == "hard":
        assert all(rst["exact_points"] == n for _, rst in refs)
    db.close()


def test_batched_int_config_sampled(P, orc):
    """The batched-integer workload at full size (n = 100,000 x m = 3072 uint8
    32-centre mixture, 1,024 queries, k = h = 10, delta = 0.01) in the launch
    configuration the benchmark times (one query-lane batch with point-major
    sums, graph replay on the second call): every set contains the true 10-NN
    of the exact scan, the replay equals the eager call, and sampled queries
    equal the oracle exactly (indices and statistics)."""
    X, Q = gmm_u8(2000, n=100_000, m=3072, n_centres=32, sigma=30.0, nq=1024)
    db = P.KnnDB(dev(X))
    Qd = dev(Q)
    p = P.default_params(h=10, delta=0.01, seed=12345)
    idx, cnt, st = db.adaptive(Qd, 10, p)
    idx2, cnt2, _ = db.adaptive(Qd, 10, p, with_stats=False)
    assert torch.equal(idx, idx2) and torch.equal(cnt, cnt2)
    nidx, ndist = db.naive(Qd, 10)
    idx_c, cnt_c, nidx, ndist = idx.cpu().numpy(), cnt.cpu().numpy(), nidx.cpu().numpy(), ndist.cpu().numpy()
    for qi in range(1024):
        got = idx_c[qi, :cnt_c[qi]]
        dk = ndist[qi, 9]
        assert set(nidx[qi][ndist[qi] < dk].tolist()) <= set(got.tolist()), qi
    sample = list(range(0, 1024, 16))  # 64 queries spread over the batch's slots
    refs = oracle_many(orc, X, Q, np.full(1024, 10), dict(h=10, delta=0.01, seed=12345), sample)
    for qi, (ref, rst) in zip(sample, refs):
        assert idx_c[qi, :cnt_c[qi]].tolist() == ref.tolist(), qi
        assert (int(st[qi]["coord_evals"]), int(st[qi]["rounds"]), int(st[qi]["exact_points"])) == \
            (rst["coord_evals"], rst["rounds"], rst["exact_points"]), qi


def test_float_config_sampled(P, orc):
    """The float workload at full DB size (n = 1,000,000 x m = 128 fp32,
    1,000-cluster mixture, k = h = 10, delta = 0.05), 256 of its queries in
    one call: sampled queries equal the oracle (fixed-point sums, FP64
    decisions) and contain the FP64 10-NN."""
    X, Q = gmm_f32(3000, n=1_000_000, m=128, n_centres=1000, sigma=0.1, nq=256)
    db = P.KnnDB(dev(X))
    p = P.default_params(h=10, delta=0.05, seed=77)
    idx, cnt, st = db.adaptive(dev(Q), 10, p)
    idx_c, cnt_c = idx.cpu().numpy(), cnt.cpu().numpy()
    for qi in (0, 255):
        ref, rst = orc.adaptive(X, Q[qi], 10, oparams(orc, h=10, delta=0.05, seed=77))
        assert idx_c[qi, :cnt_c[qi]].tolist() == ref.tolist(), qi
        assert int(st[qi]["coord_evals"]) == rst["coord_evals"], qi
        assert contains_knn(ref, brute_dists(X, Q[qi]), 10, rtol=1e-9)
