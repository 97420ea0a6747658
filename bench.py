#!/usr/bin/env python3
"""Benchmark: adaptive k-NN (LeJeune, Baraniuk, Heckel, AISTATS 2019) against
the naive MFMA scan on one MI355X.

Workload (batched integer): n = 100,000 points, m = 3072 dims, uint8 from a
32-component Gaussian mixture (centres uniform in [0,255], sigma 30, rounded
and clipped), 1,024 queries from the same mixture sharing one seed, k = 10,
h = 10, delta = 0.01, all inputs resident in HBM before the timed region.
The headline batch samples one coordinate sequence shared by all points,
without replacement (sampling 3, Section 4 and its footnote); the other
three sampling modes are timed on the same batch and reported beside it.

One step = one adaptive k-NN pass over the whole batch of 1,024 queries
(every stage: sampling, bounds, selection, decisions, compaction, output).
A query counts only when its returned set contains the true k nearest
neighbours (tie-aware, against the exact int8-MFMA scan computed before the
timed region).  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "k-NN queries/s adaptive vs naive MFMA (true k-NN contained), p50/p99 latency"
N, M, NQ, K, H, DELTA = 100_000, 3072, 1024, 10, 10, 0.01
HBM_PEAK_GBS = 8000.0
INT8_PEAK_TOPS = 5000.0
# Sampled rounds are bound by the vector ALU.  Its peak in 8-op slots:
# 256 CU x 4 SIMD x 16 lanes x 2.4 GHz = 39.3 T lane-instructions/s, each at
# most a v_dot4 of four multiply-adds (8 ops): 314.6 TOP/s.  Algorithmic work
# of a sampled round: 3 integer ops (difference, square, add) per (query,
# sample) pair, and one random index per distinct coordinate draw (shared by
# every query with the same seed), counted as the lane-instructions it takes:
# Philox4x32-10's share 20 (10 rounds x (2 mul_lo + 2 mul_hi + 4 xor) / 4
# draws), the multiply-shift 1 and the gather 1 = 22.
VALU_LANE_INSTR_PEAK = 39.3e12
DOT4_PEAK_TOPS = 314.6
OPS_PER_PAIR = 3
OPS_PER_DRAW = 22
# l1 distance: 3 ops per (query, sample) pair in the sampled rounds as well
# (difference, absolute value, add); the exact round and the naive scan run
# one v_sad_u8 (four absolute differences and four additions, 8 op slots)
# per query and four coordinates: 2 ops per (query, coordinate) pair.
OPS_PER_PAIR_L1 = 3
OPS_PER_ELEM_L1 = 2
METRIC_L1 = "l1 distance: k-NN queries/s adaptive vs naive v_sad_u8 scan (true k-NN contained)"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# HBM traffic of the dominant kernel: measured by two rocprofv3 --pmc passes
# over `bench.py --profile-pass` (FETCH_SIZE, then WRITE_SIZE), each scaled
# by what the counter reads for a plain copy of known size in the same run,
# and stored with the hash of the kernel's source; reported only while the
# source is unchanged.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sample_ql_u8_batched_int_traffic.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1902_09465_amd", "csrc", "k_adaptive.hip")
ROUND_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_round_seq_u8_batched_int_traffic.txt")
ROUND_KERNEL_SRC = os.path.join(ROOT, "paper_1902_09465_amd", "csrc", "k_naive.hip")
COPY_BYTES = 1 << 30


def source_hash(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def stored_traffic(path, src):
    """Bytes per launch of a kernel from its committed counter summary, or
    None when the summary is missing or was taken on other source."""
    try:
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith(" "):
                a, b = line.split(":", 1)
                kv[a.strip()] = b.strip()
        if kv.get("source_sha256_16") != source_hash(src):
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def profile_pass(args):
    """The workload of the counter and kernel-trace passes: a plain device copy
    of COPY_BYTES (calibrates FETCH_SIZE / WRITE_SIZE), then `--steps`
    adaptive batches of the batched-integer workload in sampling mode
    `--sampling`, launched eagerly (no graph); with --naive, `--steps` naive
    scans of the same batch instead."""
    os.environ["KNN_GRAPH"] = "0"
    import torch
    from knn_inputs import gmm_u8
    P = load_lib()
    src = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda").fill_(7)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    X, Q = gmm_u8(2000, n=N, m=M, n_centres=32, sigma=30.0, nq=NQ)
    db = P.KnnDB(torch.from_numpy(X).cuda())
    Qd = torch.from_numpy(Q).cuda()
    if args.naive:
        for s in range(args.steps):
            db.naive(Qd, K, with_dist=False)
            torch.cuda.synchronize()
            log(f"profile pass naive scan {s + 1}/{args.steps} done")
        return 0
    for s in range(args.steps):
        idx, cnt, _ = db.adaptive(Qd, K, P.default_params(h=H, delta=DELTA, seed=12345, sampling=args.sampling),
                                  with_stats=False)
        torch.cuda.synchronize()
        log(f"profile pass batch {s + 1}/{args.steps} done: {int((cnt > 0).sum())} queries answered")
    return 0


def load_lib():
    import paper_1902_09465_amd as P
    try:
        P.lib()
    except ImportError:
        from paper_1902_09465_amd import build
        build.build()
        P.lib()
    return P


def contained(idx, cnt, X_t, Q_t, nidx, ndist, k, metric="l2"):
    """Per query: does the returned set contain a k-NN set (tie-aware)?"""
    import torch
    nq = idx.shape[0]
    dk = ndist[:, k - 1]  # exact k-th distance
    ok = torch.zeros(nq, dtype=torch.bool, device=idx.device)
    valid = idx >= 0
    safe = torch.where(valid, idx, torch.zeros_like(idx))
    pts = X_t[safe.reshape(-1)].reshape(nq, idx.shape[1], -1).to(torch.int32)
    diff = pts - Q_t[:, None, :].to(torch.int32)
    d = (diff.abs() if metric == "l1" else diff ** 2).sum(-1).to(torch.float64)
    d = torch.where(valid, d, torch.full_like(d, float("inf")))
    n_le = (d <= dk[:, None]).sum(1)
    strict = ndist < dk[:, None]  # neighbours strictly closer than d_(k)
    member = (nidx[:, :, None] == idx[:, None, :]).any(-1)
    ok = (~strict | member).all(1) & (n_le >= k)
    return ok


def _oracle_worker(args):
    X, q, k, h, delta, seed, metric, sampling = args
    import oracle
    t0 = time.perf_counter()
    idx, st = oracle.adaptive(X, q, k, oracle.make_params(h=h, delta=delta, seed=seed, sampling=sampling),
                              metric=metric)
    return time.perf_counter() - t0, st["coord_evals"]


def cpu_baseline(X, Q, seconds_hint, metric=0, sampling=0):
    """The oracle, untuned, on this host's cores: one query per process."""
    import oracle
    oracle.build()
    cores = max(1, min(os.cpu_count() or 1, 16))
    nqs = cores
    jobs = [(X, Q[i], K, H, DELTA, 12345, metric, sampling) for i in range(nqs)]
    t0 = time.perf_counter()
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    per_q = [r[0] for r in res]
    return {"value": nqs / wall, "unit": "queries/s", "cores": cores, "kind": "oracle",
            "sample": f"{nqs} queries of the same workload, one per process ({cores} processes), "
                      f"single-threaded C oracle each; wall {wall:.1f} s, median per-query "
                      f"{np.median(per_q):.1f} s"}


def serving(args):
    """Serving workload: three resident DBs in one session, requests with
    k ~ U{1..50}, delta in {0.01, 0.05} and their own seeds.  First the
    closed-loop saturation rate (every request submitted at once), then
    Poisson arrivals at 0.3, 0.6 and 0.9 of it; latency = completion - arrival
    on the host clock, completion seen by a poller thread."""
    import threading
    import torch
    from knn_inputs import serving_dbs, rng

    P = load_lib()
    log("generating the three serving databases")
    data = serving_dbs(5000, scale=args.serving_scale)
    dbs, qpools = [], []
    for X, Q in data:
        dbs.append(P.KnnDB(torch.from_numpy(X).cuda()))
        qpools.append(Q)
    torch.cuda.synchronize()
    free = torch.cuda.mem_get_info()[0]
    sess = P.Session(int(min(free * 0.6, args.serving_budget_gb * (1 << 30))))
    ids = [sess.add_db(db) for db in dbs]
    g = rng(5100)

    def make_requests(count):
        reqs = []
        for _ in range(count):
            d = int(g.integers(0, 3))
            q = qpools[d][int(g.integers(0, qpools[d].shape[0]))]
            k = int(g.integers(1, 51))
            delta = 0.01 if g.integers(0, 2) == 0 else 0.05
            reqs.append((d, q, k, P.default_params(h=k, delta=delta, seed=int(g.integers(1 << 40)))))
        return reqs

    def run(reqs, arrivals):
        """Submits reqs at the given arrival offsets (seconds; None = all at
        once) and returns (latencies, completion results, wall seconds)."""
        n = len(reqs)
        t_sub = [0.0] * n
        tickets = [None] * n
        lat = [None] * n
        res = [None] * n
        done_sub = threading.Event()
        t0 = time.perf_counter()

        def submitter():
            for i, (d, q, k, p) in enumerate(reqs):
                if arrivals is not None:
                    wait = t0 + arrivals[i] - time.perf_counter()
                    if wait > 0:
                        time.sleep(wait)
                t_sub[i] = time.perf_counter() if arrivals is None else t0 + arrivals[i]
                tickets[i] = sess.submit(ids[d], q, k, p)
            done_sub.set()

        th = threading.Thread(target=submitter)
        th.start()
        pending = set()
        nxt = 0
        finished = 0
        while finished < n:
            while nxt < n and tickets[nxt] is not None:
                pending.add(nxt)
                nxt += 1
            for i in list(pending):
                r = sess.poll(tickets[i], reqs[i][2] * 2)
                if r is not None:
                    lat[i] = time.perf_counter() - t_sub[i]
                    res[i] = r
                    pending.discard(i)
                    finished += 1
            time.sleep(0.0002)
        th.join()
        return lat, res, time.perf_counter() - t0

    log("warm-up")
    run(make_requests(args.serving_warmup), None)
    log("closed-loop saturation")
    sat_reqs = make_requests(args.serving_requests)
    _, _, wall = run(sat_reqs, None)
    sat_rate = len(sat_reqs) / wall
    out_rates = []
    for frac in (0.3, 0.6, 0.9):
        rate = frac * sat_rate
        reqs = make_requests(args.serving_requests)
        arrivals = np.cumsum(g.exponential(1.0 / rate, size=len(reqs)))
        log(f"Poisson arrivals at {rate:.1f} req/s ({frac} x saturation)")
        lat, res, wall = run(reqs, arrivals)
        lat_ms = np.array(lat) * 1e3
        # containment of a sample of the answers, against the exact scan
        ok = tot = 0
        for i in range(0, len(reqs), max(1, len(reqs) // 64)):
            d, q, k, _ = reqs[i]
            qd = torch.from_numpy(np.ascontiguousarray(q[None])).cuda()
            nidx, ndist = dbs[d].naive(qd, k)
            got = set(res[i][0].tolist())
            X = data[d][0]
            dk = float(ndist[0, k - 1])
            need = [int(j) for j, dj in zip(nidx[0].tolist(), ndist[0].tolist()) if dj < dk]
            dist_got = [float(((X[j].astype(np.float64) - q.astype(np.float64)) ** 2).sum()) for j in got]
            n_le = sum(1 for v in dist_got if v <= dk * (1 + 1e-12))
            ok += int(all(j in got for j in need) and n_le >= k)
            tot += 1
        out_rates.append({"offered_per_s": rate, "fraction_of_saturation": frac, "requests": len(reqs),
                          "achieved_per_s": len(reqs) / wall, "p50_ms": float(np.percentile(lat_ms, 50)),
                          "p99_ms": float(np.percentile(lat_ms, 99)), "mean_ms": float(lat_ms.mean()),
                          "contained_sampled": f"{ok}/{tot}"})
    sess.close()
    out = {"metric": "serving queries/s and p50/p99 latency (continuous batching, three resident DBs)",
           "value": sat_rate, "unit": "queries/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "u8+f32", "data": "synthetic",
           "config": {"workload": "serving: DB A 50,000x784 u8 (10-centre mixture, sigma 30), DB B 500,000x256 "
                                  "f32 and DB C 2,000,000x96 f32 (1,000-cluster mixtures, sigma 0.1), sizes x "
                                  f"{args.serving_scale}; k ~ U(1..50), h = k, delta in (0.01, 0.05), "
                                  "DB uniform, per-request seeds"},
           "saturation_per_s": sat_rate, "rates": out_rates}
    print(json.dumps(out), flush=True)
    return 0


def paper_sweep(args):
    """Section 5's experiment on its synthetic data: x = c Q y (subspace
    dimension p in {10, 100, 1000}), n = 1000, m = 12288, k = h = 10,
    delta = 0.001, the C_alpha width (alpha_kind 2), several trials (data and
    seed per trial).  Reports, per (p, C_alpha), the median and interquartile
    range of recall (true 10-NN found among the 20 returned) and of the
    fraction of coordinate evaluations of the naive scan, plus the median
    single-query latency of adaptive and of the naive scan."""
    import torch
    from knn_inputs import subspace

    P = load_lib()
    n, m, k = 1000, 12288, 10
    cs = [0.001, 0.003, 0.01, 0.03, 0.1, 0.3, 1.0]
    rows = []
    for pdim in (10, 100, 1000):
        per_c = {c: {"recall": [], "frac": [], "ms": []} for c in cs}
        naive_ms = []
        for trial in range(args.trials):
            X, Q = subspace(10_000 + 97 * pdim + trial, n=n, m=m, p=pdim, nq=1)
            db = P.KnnDB(torch.from_numpy(X).cuda())
            qd = torch.from_numpy(Q).cuda()
            nidx, _ = db.naive(qd, k)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nidx, _ = db.naive(qd, k)
            torch.cuda.synchronize()
            naive_ms.append((time.perf_counter() - t0) * 1e3)
            true = set(nidx[0].tolist())
            for c in cs:
                prm = P.default_params(h=k, delta=0.001, seed=trial + 1, alpha_kind=2, c_alpha=c)
                db.adaptive(qd, k, prm)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                idx, cnt, st = db.adaptive(qd, k, prm)
                torch.cuda.synchronize()
                per_c[c]["ms"].append((time.perf_counter() - t0) * 1e3)
                got = set(idx[0, :int(cnt[0])].tolist())
                per_c[c]["recall"].append(len(true & got) / k)
                per_c[c]["frac"].append(float(st[0]["coord_evals"]) / (n * m))
            db.close()
        for c in cs:
            r, f, t = (np.array(per_c[c][x]) for x in ("recall", "frac", "ms"))
            rows.append({"p": pdim, "c_alpha": c,
                         "recall_median": float(np.median(r)),
                         "recall_iqr": [float(np.percentile(r, 25)), float(np.percentile(r, 75))],
                         "eval_fraction_median": float(np.median(f)),
                         "eval_fraction_iqr": [float(np.percentile(f, 25)), float(np.percentile(f, 75))],
                         "adaptive_ms_median": float(np.median(t)),
                         "naive_ms_median": float(np.median(naive_ms))})
            log(f"p={pdim} C={c}: recall {rows[-1]['recall_median']:.2f} "
                f"fraction {rows[-1]['eval_fraction_median']:.3f} "
                f"adaptive {rows[-1]['adaptive_ms_median']:.2f} ms naive {rows[-1]['naive_ms_median']:.2f} ms")
    out = {"metric": "Section 5 sweep: recall and fraction of naive coordinate evaluations vs C_alpha",
           "unit": "fraction", "n_gpus": 1, "data": "synthetic", "dtype": "f32",
           "config": {"workload": f"subspace x = cQy, n = {n}, m = {m}, k = h = {k}, delta = 0.001, "
                                  f"{args.trials} trials per p, one query each"},
           "rows": rows}
    print(json.dumps(out), flush=True)
    return 0


def uneven_bench(args):
    """The uneven workload (n = 250,000 x m = 1024 u8; 4,096 queries, half
    easy -- k planted points at a small gap, the rest far -- and half hard,
    near-equal distances; k cycling over 1, 10, 100; delta = 0.01; one seed):
    adaptive on the whole batch, on the easy half and on the hard half, each
    against the naive int8-MFMA scan of the same queries (one call per k)."""
    import torch
    from knn_inputs import uneven

    P = load_lib()
    log("generating the uneven workload")
    X, Q, ks = uneven(4000)
    db = P.KnnDB(torch.from_numpy(X).cuda())
    Qd = torch.from_numpy(Q).cuda()
    n_easy = Q.shape[0] // 2
    parts = {"all": np.arange(Q.shape[0]), "easy": np.arange(n_easy), "hard": np.arange(n_easy, Q.shape[0])}
    res = {}
    variants = ("pure", "pure_shared", "candidate_exact")
    for variant, (name, sel) in [(v, pn) for v in variants for pn in parts.items()]:
        qs = Qd[torch.from_numpy(sel).cuda()].contiguous()
        kk = ks[sel]
        # pure round form (coordinates drawn per point, or one sequence shared
        # by all points without replacement), or with the 2k smallest
        # estimates made exact each round
        if variant == "pure":
            p = P.default_params(h=-1, delta=0.01, seed=4001)
        elif variant == "pure_shared":
            p = P.default_params(h=-1, delta=0.01, seed=4001, sampling=3)
        else:
            p = [P.default_params(h=-1, delta=0.01, seed=4001, c_exact=int(2 * kv)) for kv in kk]
        name = f"{variant}_{name}"
        db.adaptive(qs, kk, p, with_stats=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            idx, cnt, _ = db.adaptive(qs, kk, p, with_stats=False)
        torch.cuda.synchronize()
        ad_s = (time.perf_counter() - t0) / args.steps
        _, _, st = db.adaptive(qs, kk, p)
        evals = st["coord_evals"].astype(np.float64)
        # naive: one call per k
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for kv in (1, 10, 100):
                sub = torch.from_numpy(np.nonzero(kk == kv)[0]).cuda()
                if sub.numel():
                    db.naive(qs[sub].contiguous(), kv, with_dist=False)
        torch.cuda.synchronize()
        nv_s = (time.perf_counter() - t0) / args.steps
        res[name] = {"queries": int(len(sel)), "adaptive_queries_per_s": len(sel) / ad_s,
                     "naive_queries_per_s": len(sel) / nv_s, "adaptive_vs_naive": nv_s / ad_s,
                     "evals_fraction_of_naive": float(evals.mean() / (X.shape[0] * X.shape[1]))}
        log(f"{name}: adaptive {len(sel) / ad_s:.0f} q/s, naive {len(sel) / nv_s:.0f} q/s, "
            f"evaluations {res[name]['evals_fraction_of_naive']:.3f} of naive")
    out = {"metric": "uneven workload: queries/s adaptive vs naive MFMA (whole batch, easy half, hard half)",
           "value": res["pure_shared_all"]["adaptive_queries_per_s"], "unit": "queries/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "u8", "data": "synthetic",
           "config": {"workload": "uneven: n=250000 x m=1024 uint8 binary corners, 4096 queries (2048 easy with k "
                                  "planted points, 2048 hard), k in (1, 10, 100), h = k, delta = 0.01, one seed; "
                                  "value: the pure round form with one coordinate sequence shared by all points"},
           "parts": res}
    print(json.dumps(out), flush=True)
    return 0


def easy_bench(args):
    """Easy-gap batches, where adaptive is meant to win: the easy half of the
    uneven workload on its own (n = 100,000 corners of {0,255}^m, 1,024
    queries each owning k = 10 planted points at a small gap, the rest far;
    h = k, delta = 0.01, the footnote width, one seed) at m = 1024, 4096,
    16384, 32768 and 65535 (the largest m of the shared-sequence kernels).  Adaptive
    in sampling modes 0 and 3 (first round B0 = 64), and in mode 3 with the
    larger first rounds of --easy-b0, against the naive int8-MFMA scan of the
    same queries; containment against that scan."""
    import torch
    from knn_inputs import easy_corners

    P = load_lib()
    n, nq, k = 100_000, 1024, 10
    rows = []
    for m in args.easy_m:
        log(f"easy-gap workload m = {m}: generating")
        X, Q = easy_corners(6000 + m, n, m, nq, k)
        X_t = torch.from_numpy(X).cuda()
        Q_t = torch.from_numpy(Q).cuda()
        db = P.KnnDB(X_t)
        nidx, ndist = db.naive(Q_t, k)
        for _ in range(args.warmup):
            db.naive(Q_t, k, with_dist=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            db.naive(Q_t, k, with_dist=False)
        torch.cuda.synchronize()
        nv_s = (time.perf_counter() - t0) / args.steps
        row = {"m": m, "naive_ms": nv_s * 1e3, "naive_queries_per_s": nq / nv_s}
        # sampling 0 and 3 with the default first round (B0 = 64); sampling 3
        # again with each larger first round of --easy-b0
        runs = [(0, 64), (3, 64)] + [(3, b) for b in args.easy_b0 if b != 64]
        for mode, b0 in runs:
            p = P.default_params(h=k, delta=0.01, seed=6001, sampling=mode, b0=b0)
            for _ in range(args.warmup):
                db.adaptive(Q_t, k, p, with_stats=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                idx, cnt, _ = db.adaptive(Q_t, k, p, with_stats=False)
            torch.cuda.synchronize()
            ad_s = (time.perf_counter() - t0) / args.steps
            ok = int(contained(idx, cnt, X_t, Q_t, nidx, ndist, k).sum().item())
            _, _, st = db.adaptive(Q_t, k, p)
            frac = float(st["coord_evals"].astype(np.float64).mean() / (n * m))
            key = f"sampling{mode}" + ("" if b0 == 64 else f"_b0_{b0}")
            row[key] = {"ms": ad_s * 1e3, "queries_per_s": ok / ad_s, "contained": f"{ok}/{nq}", "b0": b0,
                        "evals_fraction_of_naive": frac, "adaptive_vs_naive": nv_s / ad_s}
            log(f"m = {m} sampling {mode} B0 = {b0}: adaptive {ad_s * 1e3:.2f} ms ({ok}/{nq} contained, "
                f"{frac:.3f} of the naive evaluations), naive {nv_s * 1e3:.2f} ms")
        rows.append(row)
        db.close()
        del X_t, Q_t, X, Q
        torch.cuda.empty_cache()
    out = {"metric": "easy-gap batches: queries/s adaptive vs naive MFMA (true k-NN contained)",
           "unit": "queries/s", "n_gpus": 1, "higher_is_better": True, "dtype": "u8", "data": "synthetic",
           "config": {"workload": f"easy corners: n = {n} corners of (0,255)^m, {nq} queries with k = {k} planted "
                                  "points each (inward noise 0..8), h = k, delta = 0.01, footnote width, one seed, "
                                  "first round B0 = 64 (and the --easy-b0 values in sampling 3), growth 2"},
           "rows": rows}
    print(json.dumps(out), flush=True)
    return 0


def float_bench(args):
    """The float workload (n = 1,000,000 x m = 128 fp32 points from a
    1,000-centre Gaussian mixture, centres N(0,1), sigma = 0.1; k = h = 10,
    delta = 0.05; one seed) on the first --float-queries of its 10,000
    queries: adaptive in the --sampling mode (fixed-point sums; with a shared
    coordinate sequence every round is a tile pass over the point and query
    copies gathered at it, otherwise per-slot draws) against the naive
    split-BF16 MFMA scan with FP64 rescoring, whose sets and distances are the
    exact reference for the containment check."""
    import torch
    from knn_inputs import gmm_f32

    P = load_lib()
    nq = int(args.float_queries)
    log(f"generating the float workload ({nq} of its 10000 queries)")
    X, Q = gmm_f32(3000, n=1_000_000, m=128, n_centres=1000, sigma=0.1, nq=10_000)
    Q = np.ascontiguousarray(Q[:nq])
    Xd = torch.from_numpy(X).cuda()
    Qd = torch.from_numpy(Q).cuda()
    db = P.KnnDB(Xd)
    K = 10
    p = P.default_params(h=10, delta=0.05, seed=3001, sampling=args.sampling)
    import ctypes
    lib = P.lib()
    P._lib.check(lib.knn_prof_enable(1))
    nidx, ndist = db.naive(Qd, K)
    torch.cuda.synchronize()
    cnts = np.zeros(8, dtype=np.uint64)
    P._lib.check(lib.knn_prof_counters(cnts.ctypes.data_as(ctypes.c_void_p)))
    P._lib.check(lib.knn_prof_enable(0))
    rescans = int(cnts[4])
    db.adaptive(Qd, K, p, with_stats=False)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        idx, cnt, _ = db.adaptive(Qd, K, p, with_stats=False)
    torch.cuda.synchronize()
    ad_s = (time.perf_counter() - t0) / args.steps
    _, _, st = db.adaptive(Qd, K, p)
    evals = st["coord_evals"].astype(np.float64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        db.naive(Qd, K, with_dist=False)
    torch.cuda.synchronize()
    nv_s = (time.perf_counter() - t0) / args.steps
    # containment: every returned set holds the exact k nearest (FP64 distances of the naive scan,
    # summed in coordinate order; the sums here run in another order, hence the relative 1e-9)
    rtol = 1e-9
    valid = idx >= 0
    safe = torch.where(valid, idx, torch.zeros_like(idx))
    pts = Xd[safe.reshape(-1)].reshape(nq, idx.shape[1], -1).double()
    d = ((pts - Qd[:, None, :].double()) ** 2).sum(-1)
    d = torch.where(valid, d, torch.full_like(d, float("inf")))
    dk = ndist[:, K - 1]
    strict = ndist < dk[:, None] * (1 - rtol)
    member = (nidx[:, :, None] == idx[:, None, :]).any(-1)
    ok = ((~strict | member).all(1) & ((d <= dk[:, None] * (1 + rtol)).sum(1) >= K)).sum().item()
    out = {"metric": "float workload: queries/s adaptive vs naive BF16 MFMA + FP64 rescoring",
           "value": nq / ad_s, "unit": "queries/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"float: n=1000000 x m=128 fp32, 1000-centre Gaussian mixture sigma=0.1, "
                                  f"{nq} of 10000 queries, k=10 h=10 delta=0.05",
                      "sampling": SAMPLING_NAMES[args.sampling]},
           "contained": f"{ok}/{nq}",
           "adaptive_ms_per_batch": ad_s * 1e3, "naive_ms_per_batch": nv_s * 1e3,
           "naive_queries_per_s": nq / nv_s, "adaptive_vs_naive": nv_s / ad_s,
           "naive_exact_rescans": rescans,
           "evals_fraction_of_naive": float(evals.mean() / (X.shape[0] * X.shape[1]))}
    print(json.dumps(out), flush=True)
    return 0


SAMPLING_NAMES = {0: "coordinates drawn per point with replacement",
                  1: "coordinates drawn per point without replacement",
                  2: "one coordinate sequence shared by all points, with replacement",
                  3: "one coordinate sequence shared by all points, without replacement"}


def run_adaptive(P, lib, db, X_t, Q_t, params, nidx, ndist, args, warmup, steps, label, graph=True):
    """Warm-up, then `steps` timed adaptive batches with per-kernel events;
    containment, statistics, the rooflines of the step's kernels and (graph)
    the same batch replayed as a captured graph."""
    import ctypes
    import torch
    l1 = args.metric == "l1"
    for w in range(warmup):
        log(f"{label} warmup {w + 1}/{warmup}")
        db.adaptive(Q_t, K, params, with_stats=False)
    torch.cuda.synchronize()
    P._lib.check(lib.knn_prof_enable(1))
    # the calls are stream-ordered: the host queues step s + 1 while step s
    # runs; each step's span is read from events between the steps (the
    # library and torch both use the null stream here)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    marks[0].record()
    for s in range(steps):
        idx, cnt, _ = db.adaptive(Q_t, K, params, with_stats=False)
        marks[s + 1].record()
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t_all
    step_ms = [marks[s].elapsed_time(marks[s + 1]) for s in range(steps)]
    for s in range(steps):
        log(f"{label} step {s + 1}/{steps}: {step_ms[s]:.1f} ms")
    # containment and statistics (outside the timed region)
    ok = contained(idx, cnt, X_t, Q_t, nidx, ndist, K, args.metric)
    n_ok = int(ok.sum().item())
    prof = {}
    for kind, name in ((0, "sample"), (7, "sample_exact_round"), (8, "sample_aux"), (9, "sample_sparse"),
                       (1, "cand"), (2, "select"), (3, "decide"), (4, "finish")):
        ms, n_l, u = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        P._lib.check(lib.knn_prof_read(kind, ctypes.byref(ms), ctypes.byref(n_l), ctypes.byref(u)))
        prof[name] = dict(ms=ms.value, launches=n_l.value)
    cnts = np.zeros(8, dtype=np.uint64)
    P._lib.check(lib.knn_prof_counters(cnts.ctypes.data_as(ctypes.c_void_p)))
    P._lib.check(lib.knn_prof_enable(0))
    _, _, stats = db.adaptive(Q_t, K, params, with_stats=True)
    torch.cuda.synchronize()
    evals = stats["coord_evals"].astype(np.float64)
    ms_per_step = total_s * 1e3 / steps
    out = {"value": n_ok / (ms_per_step / 1e3), "ms_per_step": ms_per_step, "step_ms": step_ms, "n_ok": n_ok,
           "contained": f"{n_ok}/{NQ}", "evals": evals, "idx": idx, "cnt": cnt, "prof": prof,
           "fraction_of_naive_evals": float(evals.mean() / (N * M)),
           "kernels_ms_per_step": {k_: v["ms"] / steps for k_, v in prof.items()}}
    if graph:
        # the same batch replayed through the cached engine's captured graph
        # (timing events off: the graph path is taken only then)
        db.adaptive(Q_t, K, params, with_stats=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            idx_g, cnt_g, _ = db.adaptive(Q_t, K, params, with_stats=False)
        torch.cuda.synchronize()
        out["graph_ms"] = (time.perf_counter() - t0) * 1e3 / steps
        out["same_graph"] = bool(torch.equal(idx_g, idx) and torch.equal(cnt_g, cnt))

    # rooflines (averages over the timed steps)
    shared = params.sampling >= 2
    alg_bytes, pairs, exact_elems, draws_pp = (float(c) for c in cnts[:4])
    draws = draws_pp + float(cnts[5])
    out["work"] = (alg_bytes, pairs, exact_elems, draws)
    samp, exr = prof["sample"], prof["sample_exact_round"]
    s_avg = samp["ms"] / max(1, samp["launches"]) / 1e3
    e_avg = exr["ms"] / max(1, exr["launches"]) / 1e3
    if shared:
        # sampled rounds as products over the gathered coordinates (int8 MFMA
        # for squared l2, v_sad_u8 for l1).  Per launch the running sums D
        # [n][1024] u32 are written (round 0) or read and written with the
        # "not sampled" bytes A (later rounds): 4 or 9 bytes per (query,
        # point), against a product of 2 B_r ops per pair -- at these round
        # sizes the state traffic, not the matrix cores, bounds the kernel.
        r_per_step = samp["launches"] / max(1, steps)
        b_pair = (4.0 + 9.0 * (r_per_step - 1)) / max(1.0, r_per_step)
        cols = pairs / max(1.0, float(N * NQ))  # columns the timed launches sampled (all steps)
        s_bytes = b_pair * N * NQ + (N + NQ) * cols / max(1, samp["launches"])
        s_ops = (2.0 if not l1 else OPS_PER_ELEM_L1) * pairs / max(1, samp["launches"])
        rl_sample = {"bound": "hbm", "achieved": s_bytes / s_avg / 1e9 if s_avg > 0 else 0.0,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": None,
                     "kernel": ("k_round_seq_u8<l1> (sampled rounds, v_sad_u8 tiles over the gathered coordinates)"
                                if l1 else
                                "k_round_seq_u8<l2> (sampled rounds, int8 MFMA over the gathered coordinates)"),
                     "avg_launch_ms": s_avg * 1e3, "launches": samp["launches"], "alg_bytes_per_launch": s_bytes,
                     "ops_per_launch": s_ops,
                     "ops_rate_tops": s_ops / s_avg / 1e12 if s_avg > 0 else 0.0}
        rl_sample["frac"] = rl_sample["achieved"] / HBM_PEAK_GBS
        if not l1 and params.sampling == 3:
            rl_sample["traffic"] = stored_traffic(ROUND_TRAFFIC_FILE, ROUND_KERNEL_SRC)
        if rl_sample["traffic"] and s_avg > 0:
            rl_sample["traffic_gbs"] = rl_sample["traffic"] / s_avg / 1e9
    else:
        s_ops = (draws * OPS_PER_DRAW + pairs * (OPS_PER_PAIR_L1 if l1 else OPS_PER_PAIR)) / max(1, samp["launches"])
        rl_sample = {"bound": "alu", "achieved": s_ops / s_avg / 1e12 if s_avg > 0 else 0.0,
                     "peak": DOT4_PEAK_TOPS, "unit": "TOP/s", "traffic": None,
                     "kernel": ("k_round_seq_u8<l1> (sampled rounds, v_sad_u8 tiles over the gathered coordinates)"
                                if shared else "k_sample_ql_u8 (sampled rounds, query-lane)"),
                     "avg_launch_ms": s_avg * 1e3,
                     "launches": samp["launches"], "ops_per_launch": s_ops}
        rl_sample["frac"] = rl_sample["achieved"] / DOT4_PEAK_TOPS
        if not shared:
            # with the draws shared by all queries of the batch: the running
            # sums D [n][1024] u32 written in every round and read in every
            # round but the first, the point-major flags A [n][1024] read in
            # every round but the first, and one byte per distinct draw
            r_per_step = samp["launches"] / max(1, steps)
            later = (r_per_step - 1) / max(1.0, r_per_step)
            rl_sample["alg_bytes_per_launch"] = (N * NQ * 4 + N * NQ * (4 + 1) * later +
                                                 draws / max(1, samp["launches"]))
            if not l1 and params.sampling == 0:
                rl_sample["traffic"] = stored_traffic(TRAFFIC_FILE, KERNEL_SRC)
            if rl_sample["traffic"] and s_avg > 0:
                rl_sample["achieved_hbm_gbs"] = rl_sample["traffic"] / s_avg / 1e9
                rl_sample["hbm_frac"] = rl_sample["achieved_hbm_gbs"] / HBM_PEAK_GBS
    # exact round: one tiled pass over (queries x points), a GEMM on the
    # matrix cores for squared l2, v_sad_u8 sums on the vector ALU for l1
    e_ops = (OPS_PER_ELEM_L1 if l1 else 2.0) * exact_elems / max(1, exr["launches"])
    e_peak = DOT4_PEAK_TOPS if l1 else INT8_PEAK_TOPS
    rl_exact = {"bound": "alu" if l1 else "mfma", "achieved": e_ops / e_avg / 1e12 if e_avg > 0 else 0.0,
                "peak": e_peak, "unit": "TOP/s", "traffic": None,
                "kernel": (("k_round_seq_u8" if params.sampling == 3 else "k_exact_ql_u8") +
                           ("<l1> (exact round, v_sad_u8 tiles)" if l1 else "<l2> (exact round, int8 MFMA GEMM)")),
                "avg_launch_ms": e_avg * 1e3, "launches": exr["launches"], "ops_per_launch": e_ops}
    rl_exact["frac"] = rl_exact["achieved"] / e_peak
    # selection and decisions stream the point-major sums D [n][1024] u32
    # and the flags [1024][n] (5 bytes per (query, point)); decisions also
    # write the next round's "not sampled" bytes A (1 byte)
    def hbm_rl(name, kernel, per_pair):
        pr = prof[name]
        avg = pr["ms"] / max(1, pr["launches"]) / 1e3
        b = per_pair * N * NQ
        ach = b / avg / 1e9 if avg > 0 else 0.0
        return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": None, "kernel": kernel, "avg_launch_ms": avg * 1e3, "launches": pr["launches"],
                "alg_bytes_per_launch": b}
    rl_select = hbm_rl("select", "k_select_pm + merges (k-th bound selection)", 5)
    rl_decide = hbm_rl("decide", "k_decide_pm + k_decide (decisions)", 6)
    dom = max(prof, key=lambda k_: prof[k_]["ms"])
    out["dominant_kernel"] = dom
    out["roofline"] = {"sample_exact_round": rl_exact, "select": rl_select, "decide": rl_decide}.get(dom, rl_sample)
    out["roofline_sampled_rounds"] = rl_sample
    out["roofline_exact_round"] = rl_exact
    out["roofline_select"] = rl_select
    out["roofline_decide"] = rl_decide
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--serving", action="store_true", help="serving workload instead of the batch line")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-warmup", type=int, default=200)
    ap.add_argument("--serving-scale", type=float, default=1.0)
    ap.add_argument("--serving-budget-gb", type=float, default=96.0)
    ap.add_argument("--paper-sweep", action="store_true", help="Section 5 C_alpha sweep instead of the batch line")
    ap.add_argument("--trials", type=int, default=20)
    ap.add_argument("--uneven", action="store_true", help="uneven workload instead of the batch line")
    ap.add_argument("--float", action="store_true", help="float workload instead of the batch line")
    ap.add_argument("--easy", action="store_true", help="easy-gap batches at several m instead of the batch line")
    ap.add_argument("--easy-m", type=int, nargs="+", default=[1024, 4096, 16384, 32768, 65535])
    ap.add_argument("--easy-b0", type=int, nargs="+", default=[1024],
                    help="first-round sample counts tried in sampling 3 besides the default 64")
    ap.add_argument("--float-queries", type=int, default=1024)
    ap.add_argument("--sampling", type=int, choices=(0, 1, 2, 3), default=3,
                    help="sampling mode of the headline batch (knn_params.sampling; the other modes are "
                         "reported beside it)")
    ap.add_argument("--metric", choices=("l2", "l1"), default="l2",
                    help="distance of the batch line (l1: the same workload on an l1 DB)")
    ap.add_argument("--naive", action="store_true", help="with --profile-pass: naive scans instead of adaptive batches")
    ap.add_argument("--profile-pass", action="store_true",
                    help="one copy of known size and one adaptive batch, for rocprofv3 --pmc")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures a single MI355X; multi-GPU runs are not supported "
              "(run with --gpus 1)", file=sys.stderr)
        return 2
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py is single-GPU; do not launch it with several ranks", file=sys.stderr)
        return 2
    if args.serving:
        return serving(args)
    if args.paper_sweep:
        return paper_sweep(args)
    if args.uneven:
        return uneven_bench(args)
    if args.float:
        return float_bench(args)
    if args.easy:
        return easy_bench(args)
    if args.profile_pass:
        return profile_pass(args)
    import torch
    from knn_inputs import gmm_u8

    P = load_lib()
    lib = P.lib()
    import ctypes

    log("generating inputs")
    X, Q = gmm_u8(2000, n=N, m=M, n_centres=32, sigma=30.0, nq=NQ)
    X_t = torch.from_numpy(X).cuda()
    Q_t = torch.from_numpy(Q).cuda()
    l1 = args.metric == "l1"
    db = P.KnnDB(X_t, metric=args.metric)
    params = P.default_params(h=H, delta=DELTA, seed=12345, sampling=args.sampling)
    torch.cuda.synchronize()

    log("exact reference (naive scan: int8 MFMA, or v_sad_u8 for l1)")
    nidx, ndist = db.naive(Q_t, K)
    torch.cuda.synchronize()

    # ---------------- adaptive: warmup, then exactly `steps` timed steps
    head = run_adaptive(P, lib, db, X_t, Q_t, params, nidx, ndist, args, args.warmup, args.steps, "adaptive")
    value, ms_per_step, step_ms, prof = head["value"], head["ms_per_step"], head["step_ms"], head["prof"]
    n_ok, evals, idx, cnt = head["n_ok"], head["evals"], head["idx"], head["cnt"]
    dom, roofline, rl_exact = head["dominant_kernel"], head["roofline"], head["roofline_exact_round"]
    graph_ms, same_graph = head["graph_ms"], head["same_graph"]
    alg_bytes, pairs, exact_elems, draws = head["work"]

    # ---------------- the other sampling modes on the same batch (one seed):
    # 0 and 1 draw per point (query-lane sampler), 2 and 3 share one coordinate
    # sequence between all points (rounds as int8 products over the gathered
    # coordinates)
    other_modes = {}
    for mode in (0, 1, 2, 3):
        if mode == args.sampling:
            continue
        pm = P.default_params(h=H, delta=DELTA, seed=12345, sampling=mode)
        r = run_adaptive(P, lib, db, X_t, Q_t, pm, nidx, ndist, args, 1, args.steps, f"sampling {mode}",
                         graph=False)
        other_modes[str(mode)] = {k_: r[k_] for k_ in ("value", "ms_per_step", "contained", "fraction_of_naive_evals",
                                                      "kernels_ms_per_step", "dominant_kernel", "roofline")}

    # ---------------- the same workload with a seed per query (what independent
    # callers and the serving session send): the draws are not shared, so the
    # batch runs on the per-query sampling kernels
    seeds_q = [P.default_params(h=H, delta=DELTA, seed=12345 + q, sampling=args.sampling) for q in range(NQ)]
    log("per-query seeds: warmup")
    db.adaptive(Q_t, K, seeds_q, with_stats=False)
    torch.cuda.synchronize()
    pq_steps = max(1, min(args.steps, 2))
    t0 = time.perf_counter()
    for s in range(pq_steps):
        idx_p, cnt_p, _ = db.adaptive(Q_t, K, seeds_q, with_stats=False)
    torch.cuda.synchronize()
    pq_ms = (time.perf_counter() - t0) * 1e3 / pq_steps
    pq_ok = int(contained(idx_p, cnt_p, X_t, Q_t, nidx, ndist, K, args.metric).sum().item())
    log(f"per-query seeds: {pq_ms:.1f} ms per batch, {pq_ok}/{NQ} contained")
    per_query_seeds = {"ms_per_step": pq_ms, "queries_per_s": pq_ok / (pq_ms / 1e3), "steps": pq_steps,
                       "contained": f"{pq_ok}/{NQ}",
                       "note": "same queries, seed 12345 + q for query q: no draws shared between queries"}

    # ---------------- naive MFMA scan, same batch
    for w in range(args.warmup):
        db.naive(Q_t, K, with_dist=False)
    torch.cuda.synchronize()
    P._lib.check(lib.knn_prof_enable(1))
    t0 = time.perf_counter()
    for s in range(args.steps):
        db.naive(Q_t, K, with_dist=False)
    torch.cuda.synchronize()
    naive_s = (time.perf_counter() - t0) / args.steps
    ms, n_l, u = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    P._lib.check(lib.knn_prof_read(5, ctypes.byref(ms), ctypes.byref(n_l), ctypes.byref(u)))
    P._lib.check(lib.knn_prof_enable(0))
    gemm_avg_s = ms.value / max(1, n_l.value) / 1e3
    naive_tops = (u.value / max(1, n_l.value)) / gemm_avg_s / 1e12 if gemm_avg_s > 0 else 0.0
    naive_peak = DOT4_PEAK_TOPS if l1 else INT8_PEAK_TOPS
    if l1:
        naive_info = {"queries_per_s": NQ / naive_s, "ms_per_batch": naive_s * 1e3,
                      "kernel": "k_naive_u8_k64<l1> (v_sad_u8 tiles)", "valu_sad_tops": naive_tops,
                      "valu_frac": naive_tops / naive_peak}
    else:
        naive_info = {"queries_per_s": NQ / naive_s, "ms_per_batch": naive_s * 1e3,
                      "mfma_int8_tops": naive_tops, "mfma_frac": naive_tops / naive_peak}

    # ---------------- a plain 1 GiB device-to-device copy: the rate this
    # memory system sustains for streaming reads and writes, beside the peak
    src = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda").fill_(7)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2.0 * COPY_BYTES * 5 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    for rl_ in (roofline, head["roofline_sampled_rounds"], rl_exact, head["roofline_select"], head["roofline_decide"]):
        if rl_.get("bound") == "hbm":
            rl_["copy_gbs"] = copy_gbs  # bytes read + written per second by a 1 GiB device copy, same run
            rl_["frac_of_copy"] = rl_["achieved"] / copy_gbs

    out = {
        "metric": METRIC_L1 if l1 else METRIC,
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": ("batched_int_l1" if l1 else "batched_int") +
                               ": n=100000 points x m=3072 uint8, 32-centre Gaussian mixture "
                               "sigma=30, 1024 queries sharing one seed, k=10 h=10 delta=0.01, footnote width, "
                               "B0=64, g=2, " + SAMPLING_NAMES[args.sampling] +
                               (", l1 distance" if l1 else ""),
                   "queries": NQ, "n": N, "m": M, "parallelism": "single GPU"},
        "contained": f"{n_ok}/{NQ}",
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                       "note": "whole-batch span per step on the stream (all 1024 queries finish together; "
                               "steps are queued back to back, host preparation overlaps the previous step)"},
        "coord_evals_per_query": float(evals.mean()),
        "fraction_of_naive_evals": float(evals.mean() / (N * M)),
        "naive": naive_info,
        "adaptive_vs_naive": (value / (NQ / naive_s)) if naive_s > 0 else None,
        "kernels_ms_per_step": {k_: v["ms"] / args.steps for k_, v in prof.items()},
        "per_query_seeds": per_query_seeds,
        "other_sampling_modes": other_modes,
        "graph_replay": {"ms_per_step": graph_ms, "same_result": same_graph,
                         "note": "timed region above runs eagerly with per-kernel HIP events; this is the "
                                 "cached engine replaying its captured launch graph, events off"},
        "dominant_kernel": dom,
        "roofline": roofline,
        "roofline_sampled_rounds": head["roofline_sampled_rounds"],
        "roofline_exact_round": rl_exact,
        "roofline_select": head["roofline_select"],
        "roofline_decide": head["roofline_decide"],
        "work": {"draws": draws, "query_samples": pairs, "exact_elements": exact_elems,
                 "alg_bytes": alg_bytes},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on host cores)")
        out["cpu_baseline"] = cpu_baseline(X, Q, args.cpu_seconds, 1 if l1 else 0, args.sampling)
    print(json.dumps(out), flush=True)
    db.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
