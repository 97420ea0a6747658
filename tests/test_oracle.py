"""Pins for the CPU oracle: each test ties it to something other than its
own code -- published known-answer vectors, an independent RNG library, a
worked example derived from the paper's bound, brute force, Lemma 3's
coverage guarantee (with a negative control), Appendix A's explicit sample
bound, Theorem 1's miss rate and Theorem 2's lower bound."""
from __future__ import annotations

import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats as sps

from knn_inputs import antipodal, coherent, pm_half, tiny, uniform_u8, rng
from tests.helpers import brute_dists, contains_knn

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Philox


def test_philox_known_answers(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = orc.philox(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_draw_matches_rocrand_engine(orc):
    """The draw for sample t of point i is rocRAND's Philox4x32-10
    engine(seed, subsequence=i, offset=t).next(); compiled from rocRAND's
    header-only engine as an independent implementation."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("rocRAND headers / hipcc not available")
    g = rng(11)
    triples = [(0, 0, 0), (1, 2, 3), (2**64 - 1, 7, 1000001)]
    for _ in range(200):
        triples.append((int(g.integers(0, 2**63)), int(g.integers(0, 2**21)),
                        int(g.integers(0, 2**20))))
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "probe")
        subprocess.check_call([hipcc, "-O1", "-I/opt/rocm/include",
                               os.path.join(GOLDEN, "rocrand_philox_probe.cpp"), "-o", exe],
                              stderr=subprocess.DEVNULL)
        inp = "".join(f"{s} {i} {t}\n" for s, i, t in triples)
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [int(x) for x in out.split()]
    mine = [orc.draw(s, i, t) for s, i, t in triples]
    assert mine == ref


@pytest.mark.parametrize("m", [256, 3072])
def test_index_uniform_chi_square(orc, m):
    counts = np.zeros(m, dtype=np.int64)
    N = 200 * m if m <= 256 else 100 * m
    for t in range(N):
        counts[orc.index(99, t % 97, t, m)] += 1
    chi2, p = sps.chisquare(counts)
    assert p > 1e-4, (chi2, p)


# ---------------------------------------------------------------- alpha


def test_alpha_monotone_and_lil_growth(orc):
    us = np.arange(1, 4097)
    a = np.array([orc.alpha(0, int(u), 2000, 0.01) for u in us])
    assert np.all(np.isfinite(a)) and np.all(a > 0)
    assert np.all(np.diff(a) < 0), "alpha must shrink with more samples"
    # sqrt(u) alpha(u) grows like sqrt(log log u): nondecreasing, sublinear.
    g = a * np.sqrt(us)
    assert np.all(np.diff(g) >= -1e-12)
    assert g[-1] / g[0] < 1.5


def test_alpha_footnote_falls_back_to_lemma(orc):
    # delta/n = 0.9 > 1/e would make 3 log log(1/delta') negative; the
    # Lemma 3 form (valid for all delta) must be used instead.
    a0 = orc.alpha(0, 100, 1, 0.9)
    a1 = orc.alpha(1, 100, 1, 0.9)
    assert a0 == a1 and a0 > 0
    # far below 0.05 the two forms differ
    assert orc.alpha(0, 100, 1000, 0.01) != orc.alpha(1, 100, 1000, 0.01)
    assert math.isnan(orc.alpha(0, 0, 10, 0.1))
    assert math.isnan(orc.alpha(0, 5, 10, 1.5))


def _alpha_golden():
    rows = []
    for line in open(os.path.join(GOLDEN, "alpha.txt")):
        if line.strip() and not line.startswith("#"):
            kind, n, delta, c_alpha, u, a = line.split()
            rows.append((int(kind), int(n), float(delta), float(c_alpha), int(u), float(a)))
    return rows


def test_alpha_golden_values(orc):
    """Hand-derived widths (Section 4 footnote, Lemma 3 second form, its use
    as the footnote's fallback when delta/n >= 0.05, and the Section 5 C_alpha
    form), with the arithmetic written out in tests/golden/alpha.txt.  A change
    to any term of any form moves at least one of these values by far more
    than 1e-9."""
    rows = _alpha_golden()
    assert {r[0] for r in rows} == {0, 1, 2} and len(rows) >= 11
    for kind, n, delta, c_alpha, u, want in rows:
        got = orc.alpha(kind, u, n, delta, c_alpha)
        assert abs(got - want) <= 1e-9 * max(1.0, want), (kind, n, delta, c_alpha, u, got, want)


@pytest.mark.parametrize("kind,delta,shrink,expect_ok", [
    (0, 0.04, 1.0, True), (1, 0.2, 1.0, True), (0, 0.04, 0.2, False)])
def test_alpha_anytime_coverage(orc, kind, delta, shrink, expect_ok):
    """Lemma 3: for one arm (n = 1, delta' = delta) of i.i.d. [0,1] samples,
    |d^(t) - d| <= alpha(t) for all t at once with probability >= 1 - delta.
    A band shrunk by 5x must fail that (negative control: the test has power)."""
    g = rng(5 + kind)
    trials, tmax, p = 4000, 1500, 0.3
    t = np.arange(1, tmax + 1)
    a = np.array([orc.alpha(kind, int(u), 1, delta) for u in t]) * shrink
    bad = 0
    for s in range(0, trials, 500):
        x = (g.random((500, tmax)) < p).astype(np.float64)
        est = np.cumsum(x, axis=1) / t
        bad += int(np.any(np.abs(est - p) > a, axis=1).sum())
    rate = bad / trials
    if expect_ok:
        assert rate <= delta, rate
    else:
        assert rate > 5 * delta, rate


@pytest.mark.parametrize("gap", [0.9, 0.5, 0.2, 0.05])
def test_fact6_sample_bound(orc, gap):
    """Appendix A (proof of Fact 6) with the Lemma 3 constants: the smallest u
    with alpha(u) <= gap/8 is at most
      c2 / gap^2 * log(125 (n/delta) log(1.12 * 128 / gap^2)),
    c2 = c1 + 1, c1 = 128 / (1 - 2 / log(1.12 * 32))."""
    n, delta = 1000, 0.01
    c1 = 128.0 / (1.0 - 2.0 / math.log(1.12 * 32.0))
    bound = (c1 + 1.0) / gap**2 * math.log(125.0 * n / delta * math.log(1.12 * 128.0 / gap**2))
    # smallest u by doubling then bisection on the monotone alpha
    hi = 1
    while orc.alpha(1, hi, n, delta) > gap / 8:
        hi *= 2
    lo = hi // 2
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if orc.alpha(1, mid, n, delta) <= gap / 8:
            hi = mid
        else:
            lo = mid
    assert hi <= bound
    assert hi >= 0.05 * bound  # same order: the bound is not vacuous


# ---------------------------------------------------------------- schedule


def test_schedule(orc):
    assert list(orc.schedule(64, 2.0, 1.0, 3072)) == [64, 128, 256, 512, 1024, 2048]
    assert list(orc.schedule(64, 2.0, 1.0, 256)) == [64, 128]
    assert list(orc.schedule(256, 2.0, 1.0, 256)) == []
    assert list(orc.schedule(8, 1.5, 1.0, 40)) == [8, 12, 20, 32]
    assert list(orc.schedule(0, 0.0, 0.0, 3072)) == [64, 128, 256, 512, 1024, 2048]
    assert list(orc.schedule(64, 2.0, 0.5, 3072)) == [64, 128, 256, 512, 1024]
    with pytest.raises(ValueError):
        orc.schedule(62, 2.0, 1.0, 3072)
    with pytest.raises(ValueError):
        orc.schedule(4, 1.0, 1.0, 1 << 20)  # too many rounds


# ---------------------------------------------------------------- estimator


def test_exact_at_m_u8(orc):
    """Algorithm 1: once a point is made exact, d^ = d.  With B0 >= m every
    point is exact at once; S must equal the brute-force sum."""
    X, Q = uniform_u8(3, 300, 64)
    p = orc.make_params(b0=64)
    _, st, (S, fl, _) = orc.adaptive(X, Q[0], 5, p, stop_after=1, dump=True)
    assert np.array_equal(S, brute_dists(X, Q[0]))
    assert np.all(fl & 1)
    assert st["coord_evals"] == 300 * 64 and st["exact_points"] == 300


def test_exact_at_m_f32(orc):
    g = rng(4)
    X = g.standard_normal((200, 48)).astype(np.float32)
    q = g.standard_normal((48,)).astype(np.float32)
    rc, W, F = orc.scaling(X, q)
    assert rc == 0 and 30 < F < 62
    _, _, (S, fl, _) = orc.adaptive(X, q, 3, orc.make_params(b0=48), stop_after=1, dump=True)
    d = brute_dists(X, q)
    lo, hi = min(X.min(), q.min()), max(X.max(), q.max())
    Rp = (float(hi) - float(lo)) ** 2 * (1 + 2**-20)
    est = S / (48 * W)
    ref = d / (48 * Rp)
    # fixed-point truncation and fp32 rounding of (x - q)^2 only
    assert np.max(np.abs(est - ref) / ref) < 1e-6
    assert np.all(est <= 1.0)


def test_unbiased_estimator(orc):
    """Lemma 3's premise: E d^(T) = d (uniform draws, Section 4)."""
    X, Q = uniform_u8(8, 200, 128)
    d = brute_dists(X, Q[0]) / (128 * 65025.0)
    est = []
    for seed in range(300):
        _, _, (S, _, _) = orc.adaptive(X, Q[0], 5, orc.make_params(seed=seed), stop_after=1, dump=True)
        est.append(S / (64 * 65025.0))
    est = np.array(est)
    se = est.std(axis=0, ddof=1) / np.sqrt(est.shape[0])
    z = (est.mean(axis=0) - d) / se
    assert np.max(np.abs(z)) < 5.0
    assert abs(z.mean() * np.sqrt(len(z))) < 4.0


# ---------------------------------------------------------------- algorithm


def test_worked_example_pure(orc):
    """RNG-free example from the paper's bound: 5 copies of the query (every
    sample 0) among 995 antipodes (every sample 1), n = 1000, m = 1024,
    delta = 0.01, k = h = 5.  alpha(64) = 0.816 and alpha(128) = 0.580
    exceed 1/2, so nothing is decided; alpha(256) = 0.411 < 1/2, so at T = 256
    every antipode has LCB 0.589 > U = 0.411 and is discarded, and the copies
    (UCB 0.411 <= L2 = 0.589) are accepted: 1000 * 256 evaluations."""
    X, Q, where = antipodal()
    assert orc.alpha(0, 64, 1000, 0.01) > 0.5 and orc.alpha(0, 128, 1000, 0.01) > 0.5
    assert orc.alpha(0, 256, 1000, 0.01) < 0.5
    idx, st = orc.adaptive(X, Q[0], 5, orc.make_params(h=5, delta=0.01, seed=123))
    assert sorted(idx.tolist()) == where.tolist()
    assert st == dict(coord_evals=256_000, rounds=3, count=5, exact_points=0)


def test_worked_example_candidate_exact(orc):
    """Same instance with the 10 smallest estimates made exact after round 0:
    U = 0 (five exact copies), every antipode has LCB >= 1 - 0.816 > 0 and is
    discarded at T = 64: 64,000 + 10 * 1024 evaluations."""
    X, Q, where = antipodal()
    idx, st = orc.adaptive(X, Q[0], 5, orc.make_params(h=5, delta=0.01, seed=9, c_exact=10))
    assert sorted(idx.tolist()) == where.tolist()
    assert st == dict(coord_evals=74_240, rounds=1, count=5, exact_points=10)


@pytest.mark.parametrize("seed", range(12))
def test_contains_knn_bruteforce(orc, seed):
    g = rng(100 + seed)
    n, m = int(g.integers(50, 400)), int(g.choice([16, 64, 200, 256]))
    k = int(g.integers(1, 8))
    h = int(g.integers(0, 6))
    X, Q, _ = tiny(seed=200 + seed, n=n, m=m, planted=max(1, k), noise=int(g.integers(1, 40)))
    for c_exact in (0, k + h):
        p = orc.make_params(h=h, delta=0.05, seed=seed, b0=4 * int(g.integers(1, 9)),
                            growth=float(g.choice([1.5, 2.0, 3.0])), c_exact=c_exact)
        idx, st = orc.adaptive(X, Q[0], k, p)
        assert len(idx) <= k + h and len(set(idx.tolist())) == len(idx)
        assert contains_knn(idx, brute_dists(X, Q[0]), k)
        assert st["coord_evals"] <= n * (2 * m + 4)


def test_ties_everywhere(orc):
    """All points identical: every distance ties; any k+h points are valid."""
    X = np.full((100, 32), 7, dtype=np.uint8)
    q = np.full((32,), 9, dtype=np.uint8)
    idx, st = orc.adaptive(X, q, 4, orc.make_params(h=2))
    assert len(idx) == 6 and contains_knn(idx, brute_dists(X, q), 4)


def test_small_n_returns_all(orc):
    X, Q = uniform_u8(1, 7, 16)
    idx, st = orc.adaptive(X, Q[0], 4, orc.make_params(h=3))
    assert idx.tolist() == list(range(7)) and st["coord_evals"] == 0


def test_invalid_args(orc):
    X, Q = uniform_u8(1, 20, 16)
    with pytest.raises(ValueError):
        orc.adaptive(X, Q[0], 0)
    with pytest.raises(ValueError):
        orc.adaptive(X, Q[0], 3, orc.make_params(delta=0.0))
    with pytest.raises(ValueError):
        orc.adaptive(X, Q[0], 3, orc.make_params(b0=6))
    with pytest.raises(ValueError):
        orc.adaptive(X, Q[0], 3, orc.make_params(alpha_kind=2, c_alpha=0.0))


def _miss_instance(seed, n=600, m=1024):
    g = rng(seed)
    d = np.concatenate([g.uniform(0.10, 0.14, 5), g.uniform(0.145, 0.25, 30),
                        g.uniform(0.35, 0.65, n - 35)])
    X, Q, flips = pm_half(seed, n, m, d)
    return X, Q, flips


def _miss_count(orc, seeds, params_fn, m=1024):
    misses, evals = 0, []
    for s in seeds:
        X, Q, flips = _miss_instance(s, m=m)
        idx, st = orc.adaptive(X, Q[0], 5, params_fn(s))
        misses += 0 if contains_knn(idx, flips.astype(np.int64), 5) else 1
        evals.append(st["coord_evals"])
    return misses, np.array(evals)


def test_miss_rate_within_delta(orc):
    """Theorem 1: the returned set misses a nearest neighbour with
    probability <= delta.  Instances are decided before the exact round
    (candidate-exact on), so the bound is what keeps them right."""
    delta, N = 0.01, 1000
    misses, evals = _miss_count(
        orc, range(N), lambda s: orc.make_params(h=5, delta=delta, seed=10_000 + s, c_exact=10))
    limit = sps.binom.ppf(0.999, N, delta)
    assert misses <= limit, misses
    assert np.median(evals) < 600 * 1024  # decisions really happen before exact


def test_miss_rate_negative_control(orc):
    """A width far below the paper's (experimental form, tiny C_alpha) must
    produce misses on the same instances: the test above has power."""
    misses, _ = _miss_count(
        orc, range(200), lambda s: orc.make_params(h=5, delta=0.01, seed=s, alpha_kind=2,
                                                   c_alpha=1e-4))
    assert misses >= 20, misses


def test_miss_rate_pure_form(orc):
    delta, N = 0.05, 150
    misses, evals = _miss_count(
        orc, range(N), lambda s: orc.make_params(h=5, delta=delta, seed=s), m=4096)
    assert misses <= sps.binom.ppf(0.999, N, delta)
    assert np.median(evals) < 600 * 4096


def test_theorem2_lower_bound(orc):
    """Theorem 2 on +-1/2 data (h < k, delta <= 0.14): expected coordinate
    evaluations of any correct sampling algorithm are at least
    c' (sum_{i<=k-h} D_{i,k+1+h}^-2 + sum_{i>=k+1+h} D_{k-h,i}^-2)."""
    k, h, delta, n, m = 5, 2, 0.05, 300, 1024
    tot, runs = 0, 40
    for s in range(runs):
        g = rng(700 + s)
        dists = np.sort(np.concatenate([g.uniform(0.05, 0.15, 8), g.uniform(0.3, 0.6, n - 8)]))
        X, Q, flips = pm_half(700 + s, n, m, dists)
        d = np.sort(flips / m)
        idx, st = orc.adaptive(X, Q[0], k, orc.make_params(h=h, delta=delta, seed=s, c_exact=k + h))
        assert contains_knn(idx, flips.astype(np.int64), k)
        cprime = math.log(1 / (2 * delta)) * min(d[k - h - 1] * (1 - d[k - h - 1]),
                                                  d[k + h] * (1 - d[k + h]))
        nlow = cprime * (sum((d[i] - d[k + h]) ** -2.0 for i in range(k - h)) +
                         sum((d[k - h - 1] - d[i]) ** -2.0 for i in range(k + h, n)))
        assert st["coord_evals"] >= nlow
        tot += st["coord_evals"]


def test_coherent_no_savings(orc):
    """Section 4.2: all mass on one coordinate -- sampling cannot resolve the
    distances before nearly all coordinates are read."""
    X, Q = coherent(5, 400, 512)
    idx, st = orc.adaptive(X, Q[0], 5, orc.make_params(h=5, seed=1))
    assert contains_knn(idx, brute_dists(X, Q[0]), 5)
    assert st["coord_evals"] >= 400 * 512


# ---------------------------------------------------------------- naive


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_naive_matches_numpy(orc, dtype):
    g = rng(21)
    if dtype == "u8":
        X = g.integers(0, 4, size=(500, 24), dtype=np.uint8)  # many ties
        q = g.integers(0, 4, size=(24,), dtype=np.uint8)
    else:
        X = g.standard_normal((500, 24)).astype(np.float32)
        q = g.standard_normal((24,)).astype(np.float32)
    d = brute_dists(X, q)
    ref = np.lexsort((np.arange(500), d))[:17]
    idx, dist = orc.naive(X, q, 17)
    assert idx.tolist() == ref.tolist()
    if dtype == "u8":
        assert np.array_equal(dist, d[ref].astype(np.float64))
    else:  # numpy sums pairwise, the oracle in coordinate order
        assert np.allclose(dist, d[ref], rtol=1e-12, atol=0)


def test_f32_adaptive_contains(orc):
    g = rng(31)
    for s in range(6):
        X = g.standard_normal((300, 40)).astype(np.float32)
        q = X[g.integers(0, 300)] + 0.05 * g.standard_normal(40).astype(np.float32)
        idx, _ = orc.adaptive(X, q, 3, orc.make_params(h=3, seed=s, b0=8, c_exact=s % 2 * 6))
        assert contains_knn(idx, brute_dists(X, q), 3, rtol=1e-6)


# ----------------------------------------------------------------------------
# Algorithm 1 as published (sequential LUCB, Section 4)


def _tbar(orc, delta_i, n, delta, m):
    """Smallest u with alpha(u) <= Delta_i / 8 (Theorem 1's proof), capped at m."""
    if delta_i <= 0:
        return m
    lo, hi = 1, m
    if orc.alpha(0, m, n, delta) > delta_i / 8:
        return m
    while lo < hi:
        mid = (lo + hi) // 2
        if orc.alpha(0, mid, n, delta) <= delta_i / 8:
            hi = mid
        else:
            lo = mid + 1
    return lo


@pytest.mark.parametrize("seed", range(4))
def test_alg1_contains_knn(orc, seed):
    from knn_inputs import gap_family
    X, q = gap_family(200 + seed, n=400, m=256, k=5, near=5, mid=20)
    idx, st, T = orc.alg1(X, q, 5, orc.make_params(h=5, delta=0.05, seed=seed))
    assert len(idx) == 10 and len(set(idx.tolist())) == 10
    assert contains_knn(idx, brute_dists(X, q), 5)
    # bookkeeping: evaluations = samples drawn (T_i each) + m per exact point
    assert st["coord_evals"] == int(T.sum()) + 256 * st["exact_points"]
    assert (T >= 1).all() and (T <= 256).all()


def test_alg1_planted_and_antipodal(orc):
    X, q, where = tiny(1000)
    idx, st, _ = orc.alg1(X, q[0], 5, orc.make_params(h=5, delta=0.01, seed=1))
    assert set(where.tolist()) <= set(idx.tolist())
    Xa, qa, wa = antipodal(7, n=1000, m=1024, copies=5)
    idx, st, T = orc.alg1(Xa, qa[0], 5, orc.make_params(h=5, delta=0.01, seed=1))
    assert set(wa.tolist()) <= set(idx.tolist())
    # every sample of a far point is the exact distance 1: it leaves the
    # running after few samples, while the round form samples every point to
    # the first round whose width separates 0 from 1 (256,000 evaluations)
    far = np.setdiff1d(np.arange(1000), wa)
    assert T[far].max() < 64
    _, rst = orc.adaptive(Xa, qa[0], 5, orc.make_params(h=5, delta=0.01, seed=1))
    assert st["coord_evals"] < rst["coord_evals"] / 2


@pytest.mark.parametrize("seed", range(3))
def test_alg1_sample_bound(orc, seed):
    """Theorem 1's count: on the confidence event every iteration that does not
    terminate selects a 'bad' point (Lemma 4), and point i can be bad only
    while T_i <= Tbar_i, the first u with alpha(u) <= Delta_i / 8; an exact point
    (alpha = 0) is never bad.  So iterations <= sum_i min(Tbar_i, m) and the
    samples drawn in them <= twice that."""
    from knn_inputs import gap_family
    k, h, m, n, delta = 5, 5, 256, 300, 0.05
    X, q = gap_family(300 + seed, n=n, m=m, k=k, near=5, mid=15)
    idx, st, T = orc.alg1(X, q, k, orc.make_params(h=h, delta=delta, seed=seed))
    d = brute_dists(X, q) / (m * 65025.0)
    order = np.argsort(d, kind="stable")
    ds = d[order]
    rank = np.empty(n, dtype=np.int64)
    rank[order] = np.arange(n)
    bound = 0
    for i in range(n):
        r = rank[i]
        if r < k:
            gap = ds[k + h] - d[i]
        elif r >= k + h:
            gap = d[i] - ds[k - 1]
        else:
            gap = ds[k + h] - ds[k - 1]
        bound += _tbar(orc, gap, n, delta, m)
    updates = st["coord_evals"] - n - m * st["exact_points"]
    assert st["iterations"] <= bound
    assert updates <= 2 * bound


def _alg1_cases():
    from knn_inputs import gap_family, gmm_f32
    cases = []
    for seed in range(3):
        X, q = gap_family(500 + seed, n=500, m=256, k=5, near=5, mid=20)
        cases.append((f"gap{seed}", X, q, 5, dict(h=5, delta=0.05, seed=seed), 0))
    X, Q, _ = tiny(1001, n=600)
    cases.append(("tiny_h0", X, Q[0], 5, dict(h=0, delta=0.01, seed=3), 0))
    cases.append(("tiny_k1", X, Q[0], 1, dict(h=2, delta=0.01, seed=4, alpha_kind=1), 0))
    Xa, qa, _ = antipodal(9, n=800, m=512, copies=5)
    cases.append(("antipodal", Xa, qa[0], 5, dict(h=5, delta=0.01, seed=5), 0))
    Xt, qt = uniform_u8(11, n=400, m=24)  # few distinct values: many equal estimates and widths
    Xt = (Xt % 3).astype(np.uint8)
    qt = (qt % 3).astype(np.uint8)
    cases.append(("ties", Xt, qt[0], 4, dict(h=3, delta=0.1, seed=6), 0))
    cases.append(("ties_l1_shared", Xt, qt[0], 4, dict(h=3, delta=0.1, seed=7, sampling=3), 1))
    Xf, Qf = gmm_f32(12, n=500, m=64, n_centres=5, sigma=0.3, nq=1)
    cases.append(("f32_calpha", Xf, Qf[0], 6, dict(h=6, delta=0.05, seed=8, alpha_kind=2, c_alpha=0.05), 0))
    cases.append(("f32_norepl", Xf, Qf[0], 6, dict(h=4, delta=0.05, seed=9, sampling=1), 0))
    return cases


@pytest.mark.parametrize("case", _alg1_cases(), ids=lambda c: c[0])
def test_alg1_heaps_equal_ordered_array(orc, case):
    """Section 4.1: the heap bookkeeping (seven coupled heaps, O(log n) per
    iteration) makes the same choices as the ordered array -- the same
    returned set in order, iterations, evaluations, exact points and final
    sample counts -- on gaps, planted, antipodal, tie-heavy, l1, shared and
    without-replacement draws, h = 0, k = 1 and every width kind."""
    _, X, q, k, kw, metric = case
    a = orc.alg1(X, q, k, orc.make_params(**kw), metric=metric)
    b = orc.alg1(X, q, k, orc.make_params(**kw), metric=metric, heaps=True)
    assert a[0].tolist() == b[0].tolist()
    assert a[1] == b[1]
    assert np.array_equal(a[2], b[2])
    assert a[1]["iterations"] > 0


def test_alg1_heaps_large_n(orc):
    """The heap form at a size where the ordered array's O(n) fix-ups would
    dominate (n = 50,000): it returns a set containing the true k-NN."""
    from knn_inputs import gap_family
    X, q = gap_family(77, n=50_000, m=128, k=5, near=5, mid=20)
    idx, st, T = orc.alg1(X, q, 5, orc.make_params(h=5, delta=0.05, seed=1), heaps=True)
    assert contains_knn(idx, brute_dists(X, q), 5)
    assert st["coord_evals"] == int(T.sum()) + 128 * st["exact_points"]


def test_alg1_small_n_and_invalid(orc):
    X, _ = uniform_u8(5, n=8, m=16)
    idx, st, _ = orc.alg1(X, X[0], 3, orc.make_params(h=5))
    assert idx.tolist() == list(range(8))
    with pytest.raises(ValueError):
        orc.alg1(X, X[0], 3, orc.make_params(h=1, delta=0.0))


# ----------------------------------------------------------------------------
# Sampling without replacement (Section 4 footnote)


@pytest.mark.parametrize("m", [1, 2, 3, 5, 64, 100, 1000, 3072, 4097])
def test_perm_is_bijection(orc, m):
    for seed, i in ((0, 0), (12345, 7), (2**40 + 3, 99999)):
        vals = [orc.perm_index(seed, i, t, m) for t in range(m)]
        assert sorted(vals) == list(range(m)), (m, seed, i)


def test_perm_uniform_and_point_specific(orc):
    m = 97
    counts = np.zeros(m)
    firsts = set()
    for i in range(3000):
        v = orc.perm_index(5, i, 0, m)
        counts[v] += 1
        firsts.add(tuple(orc.perm_index(5, i, t, m) for t in range(4)))
    chi2 = ((counts - counts.mean()) ** 2 / counts.mean()).sum()
    assert sps.chi2.sf(chi2, m - 1) > 1e-3
    assert len(firsts) > 2900  # different points, different permutations


def test_without_replacement_exact_at_m_and_cost(orc):
    """Uniform data, where no point is decided before the exact round: with
    replacement each point costs T_{R-1} samples + m exact coordinates, without
    it the exact distance completes the permutation, m in all per point."""
    X, Q = uniform_u8(21, n=600, m=256)
    kw = dict(h=5, delta=0.01, seed=4)
    r1, s1 = orc.adaptive(X, Q[0], 5, orc.make_params(**kw, sampling=1))
    r0, s0 = orc.adaptive(X, Q[0], 5, orc.make_params(**kw, sampling=0))
    d = brute_dists(X, Q[0])
    assert contains_knn(r1, d, 5) and contains_knn(r0, d, 5)
    T = orc.schedule(64, 2.0, 1.0, 256)
    assert s0["exact_points"] == 600 and s1["exact_points"] == 600
    assert s0["coord_evals"] == 600 * (T[-1] + 256)
    assert s1["coord_evals"] == 600 * 256


@pytest.mark.parametrize("seed", range(3))
def test_without_replacement_contains(orc, seed):
    from knn_inputs import gap_family
    X, q = gap_family(400 + seed, n=500, m=256, k=5, near=5, mid=20)
    for ce in (0, 10):
        idx, st = orc.adaptive(X, q, 5, orc.make_params(h=5, delta=0.05, seed=seed, sampling=1, c_exact=ce))
        assert contains_knn(idx, brute_dists(X, q), 5)
    idx, st, T = orc.alg1(X, q, 5, orc.make_params(h=5, delta=0.05, seed=seed, sampling=1))
    assert contains_knn(idx, brute_dists(X, q), 5)
    assert st["coord_evals"] == int(T.sum())  # exact at T = m costs nothing more


# ----------------------------------------------------------------------------
# One coordinate sequence shared by all points (Section 4 writes every
# point's estimator over the same indices j_1, j_2, ...; Lemma 3 needs
# i.i.d. samples per point only)


def test_shared_draw_matches_rocrand_engine(orc):
    """The shared draw of sample t is output t mod 4 of Philox4x32-10 with
    counter (t/4, 0, 0, 2): rocRAND's engine(seed, subsequence = 2^33,
    offset = t).next(), compiled from rocRAND's header as an independent
    implementation."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("rocRAND headers / hipcc not available")
    g = rng(12)
    pairs = [(0, 0), (1, 3), (2**64 - 1, 1000001)]
    for _ in range(200):
        pairs.append((int(g.integers(0, 2**63)), int(g.integers(0, 2**20))))
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "probe")
        subprocess.check_call([hipcc, "-O1", "-I/opt/rocm/include",
                               os.path.join(GOLDEN, "rocrand_philox_probe.cpp"), "-o", exe],
                              stderr=subprocess.DEVNULL)
        inp = "".join(f"{s} {2**33} {t}\n" for s, t in pairs)
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [int(x) for x in out.split()]
    assert [orc.draw_shared(s, t) for s, t in pairs] == ref
    # the coordinate is floor(r m / 2^32) of that draw, the same for every point
    for (s, t), r in list(zip(pairs, ref))[:40]:
        for m in (1, 97, 3072):
            j = (r * m) >> 32
            assert orc.shared_index(s, t, m) == j
            assert orc.coord(2, s, 0, t, m) == j and orc.coord(2, s, 12345, t, m) == j


@pytest.mark.parametrize("m", [1, 2, 5, 100, 3072, 4097])
def test_shared_perm_is_bijection_common_to_points(orc, m):
    for seed in (0, 77, 2**40 + 3):
        vals = [orc.shared_perm_index(seed, t, m) for t in range(m)]
        assert sorted(vals) == list(range(m)), (m, seed)
        assert [orc.coord(3, seed, 9, t, m) for t in range(min(m, 50))] == vals[:50]


def test_shared_round0_sums_over_common_coordinates(orc):
    """After round 0 every point's running sum is the numpy sum of its squared
    (or absolute) differences over the same B0 shared coordinates; two equal
    points therefore keep equal sums in every round, which per-point draws do
    not give."""
    X, Q = uniform_u8(31, n=400, m=512)
    X[17] = X[311]
    for sampling, coords in ((2, [orc.shared_index(8, t, 512) for t in range(64)]),
                             (3, [orc.shared_perm_index(8, t, 512) for t in range(64)])):
        for metric in (0, 1):
            p = orc.make_params(h=5, delta=0.01, seed=8, sampling=sampling)
            _, _, (S, fl, ri) = orc.adaptive(X, Q[0], 5, p, stop_after=1, dump=True, metric=metric)
            diff = X[:, coords].astype(np.int64) - Q[0, coords].astype(np.int64)[None, :]
            want = (np.abs(diff) if metric else diff * diff).sum(axis=1)
            assert np.array_equal(S, want), (sampling, metric)
        for r in (2, 3, 4):
            _, _, (S, fl, ri) = orc.adaptive(X, Q[0], 5, p, stop_after=r, dump=True)
            assert S[17] == S[311] and ri[17] == ri[311]
    _, _, (S0, _, _) = orc.adaptive(X, Q[0], 5, orc.make_params(h=5, seed=8), stop_after=1, dump=True)
    assert S0[17] != S0[311]


def test_shared_unbiased_estimator(orc):
    """E d^ = d over seeds with the shared sequence (Section 4 estimator)."""
    X, Q = uniform_u8(5, n=50, m=256)
    d = brute_dists(X, Q[0]) / (256 * 65025.0)
    est = []
    for s in range(300):
        _, _, (S, _, _) = orc.adaptive(X, Q[0], 3, orc.make_params(seed=s, sampling=2),
                                       stop_after=1, dump=True)
        est.append(S / (64 * 65025.0))
    est = np.array(est)
    z = (est.mean(axis=0) - d) / (est.std(axis=0, ddof=1) / math.sqrt(len(est)))
    assert np.max(np.abs(z)) < 4.5, np.max(np.abs(z))


@pytest.mark.parametrize("sampling", [2, 3])
def test_shared_worked_example_unchanged(orc, sampling):
    """The RNG-free antipodal example decides the same way whatever the
    coordinates: discards at T = 256 in the pure form, 256,000 evaluations;
    74,240 with candidate-exact."""
    X, Q, where = antipodal()
    idx, st = orc.adaptive(X, Q[0], 5, orc.make_params(h=5, delta=0.01, seed=3, sampling=sampling))
    assert sorted(idx.tolist()) == where.tolist()
    assert st == dict(coord_evals=256_000, rounds=3, count=5, exact_points=0)
    idx, st = orc.adaptive(X, Q[0], 5, orc.make_params(h=5, delta=0.01, seed=3, sampling=sampling, c_exact=10))
    assert sorted(idx.tolist()) == where.tolist()
    # without replacement an exact distance costs only the m - T coordinates not yet seen
    want = 64_000 + 10 * (1024 - (64 if sampling == 3 else 0))
    assert st == dict(coord_evals=want, rounds=1, count=5, exact_points=10)


@pytest.mark.parametrize("sampling", [2, 3])
def test_shared_miss_rate_within_delta(orc, sampling):
    """Theorem 1 with the shared sequence: misses <= delta over 1,000 seeds on
    instances decided before the exact round."""
    delta, N = 0.01, 1000
    misses, evals = _miss_count(
        orc, range(N), lambda s: orc.make_params(h=5, delta=delta, seed=20_000 + s, c_exact=10,
                                                 sampling=sampling))
    assert misses <= sps.binom.ppf(0.999, N, delta), misses
    assert np.median(evals) < 600 * 1024


def test_shared_miss_rate_negative_control(orc):
    misses, _ = _miss_count(
        orc, range(200), lambda s: orc.make_params(h=5, delta=0.01, seed=s, alpha_kind=2,
                                                   c_alpha=1e-4, sampling=2))
    assert misses >= 20, misses


@pytest.mark.parametrize("seed", range(4))
def test_shared_contains_knn(orc, seed):
    from knn_inputs import gap_family
    X, q = gap_family(900 + seed, n=500, m=256, k=5, near=5, mid=20)
    d = brute_dists(X, q)
    for sampling in (2, 3):
        for ce in (0, 10):
            idx, st = orc.adaptive(X, q, 5, orc.make_params(h=5, delta=0.05, seed=seed, sampling=sampling,
                                                            c_exact=ce))
            assert contains_knn(idx, d, 5), (sampling, ce)
        idx, st, T = orc.alg1(X, q, 5, orc.make_params(h=5, delta=0.05, seed=seed, sampling=sampling))
        assert contains_knn(idx, d, 5)
