"""Pins for the oracle's l1 distance (Section 3: the results carry over to
l1).  A sample is |x_ij - x_j| instead of (x_ij - x_j)^2; under the
normalisation |x_j| <= 1/2 it lies in [0,1], so the estimator, the widths
and the accept/discard rule are unchanged once samples are divided by
W = 255 (u8) or W = (hi - lo)(1 + 2^-20) 2^F (f32).  Each test ties the
oracle to something outside its own code: numpy brute force, the draws
re-summed in numpy, the worked example derived from the paper's bound, and
the fact that on two-valued data |d| is proportional to d^2, so l1 and l2
runs must make identical decisions."""
from __future__ import annotations

import math

import numpy as np
import pytest

from knn_inputs import antipodal, pm_half, tiny, uniform_u8, rng
from tests.helpers import brute_dists, brute_l1, contains_knn


def _ceil_log2(x: float) -> int:
    f, e = math.frexp(x)
    return e - 1 if f == 0.5 else e


def test_l1_exact_at_m_u8(orc):
    """B0 >= m makes every point exact at once: S is the brute-force l1 sum."""
    X, Q = uniform_u8(3, 300, 64)
    _, st, (S, fl, _) = orc.adaptive(X, Q[0], 5, orc.make_params(b0=64), stop_after=1, dump=True,
                                     metric=orc.L1)
    assert np.array_equal(S, brute_l1(X, Q[0]))
    assert np.all(fl & 1)
    assert st["coord_evals"] == 300 * 64 and st["exact_points"] == 300


def test_l1_scaling(orc):
    """u8: W = 255 (the largest |x - q|); f32: W = R' 2^F with R' = (hi - lo)
    (1 + 2^-20) and F = 61 - ceil(log2 m) - ceil(log2 R'), so that a sum of
    m samples stays below 2^61."""
    X, Q = uniform_u8(5, 10, 33)
    assert orc.scaling(X, Q[0], metric=orc.L1) == (0, 255.0, 0)
    assert orc.scaling(X, Q[0], metric=orc.L2) == (0, 65025.0, 0)
    g = rng(6)
    Xf = (g.standard_normal((50, 40)) * 3).astype(np.float32)
    qf = g.standard_normal(40).astype(np.float32)
    rc, W, F = orc.scaling(Xf, qf, metric=orc.L1)
    lo = min(float(Xf.min()), float(qf.min()))
    hi = max(float(Xf.max()), float(qf.max()))
    Rp = (hi - lo) * (1 + 2**-20)
    assert rc == 0 and F == 61 - _ceil_log2(40) - _ceil_log2(Rp)
    assert W == math.ldexp(Rp, F)
    with pytest.raises(ValueError):
        orc.adaptive(X, Q[0], 2, orc.make_params(), metric=2)
    with pytest.raises(ValueError):
        orc.naive(X, Q[0], 2, metric=-1)


def test_l1_exact_at_m_f32(orc):
    g = rng(4)
    X = g.standard_normal((200, 48)).astype(np.float32)
    q = g.standard_normal((48,)).astype(np.float32)
    rc, W, F = orc.scaling(X, q, metric=orc.L1)
    assert rc == 0 and 30 < F < 62
    _, _, (S, fl, _) = orc.adaptive(X, q, 3, orc.make_params(b0=48), stop_after=1, dump=True,
                                    metric=orc.L1)
    d = brute_l1(X, q)
    lo, hi = min(X.min(), q.min()), max(X.max(), q.max())
    Rp = (float(hi) - float(lo)) * (1 + 2**-20)
    est = S / (48 * W)
    ref = d / (48 * Rp)
    # only the fixed-point truncation and the fp32 rounding of x - q differ
    assert np.max(np.abs(est - ref) / ref) < 1e-6
    assert np.all(est <= 1.0)


@pytest.mark.parametrize("sampling", [0, 1])
def test_l1_round0_sums(orc, sampling):
    """S after round 0 is the sum of |x_ij - x_j| over the point's first B0
    draws, re-summed here in numpy from the draw indices."""
    X, Q = uniform_u8(11, 40, 200)
    q = Q[0].astype(np.int64)
    seed = 77
    _, _, (S, fl, ri) = orc.adaptive(X, Q[0], 3, orc.make_params(seed=seed, b0=32, sampling=sampling),
                                     stop_after=1, dump=True, metric=orc.L1)
    draw = orc.perm_index if sampling else orc.index
    for i in range(40):
        js = np.array([draw(seed, i, t, 200) for t in range(32)])
        ref = int(np.abs(X[i, js].astype(np.int64) - q[js]).sum())
        # points decided in round 0 keep their sums too
        assert S[i] == ref
    if sampling:
        # without replacement the 32 draws of a point are distinct
        assert len({orc.perm_index(seed, 0, t, 200) for t in range(32)}) == 32


def test_l1_worked_example(orc):
    """The worked example of the l2 pins holds unchanged for l1: copies of
    the query give samples 0 and antipodes |0 - 255| = 255 = W, i.e. 1, so
    nothing is decided while alpha > 1/2 (T = 64, 128) and everything at
    T = 256: 1000 * 256 evaluations, the copies returned."""
    X, Q, where = antipodal()
    idx, st = orc.adaptive(X, Q[0], 5, orc.make_params(h=5, delta=0.01, seed=123), metric=orc.L1)
    assert sorted(idx.tolist()) == where.tolist()
    assert st == dict(coord_evals=256_000, rounds=3, count=5, exact_points=0)


@pytest.mark.parametrize("kw", [dict(), dict(c_exact=8), dict(sampling=1), dict(alpha_kind=2, c_alpha=0.05),
                                dict(b0=16, growth=1.5)])
def test_l1_two_valued_u8_equals_l2(orc, kw):
    """On {0, 255} data |d| = d^2 / 255 and W_l1 = W_l2 / 255, so every
    estimate d^ = S / (T W) is the same number under l1 and l2: identical
    sets and statistics, and naive distances in the ratio 255."""
    X, Q, _ = pm_half(21, 700, 256)
    p = orc.make_params(h=4, delta=0.05, seed=5, **kw)
    i1, s1 = orc.adaptive(X, Q[0], 6, p, metric=orc.L1)
    i2, s2 = orc.adaptive(X, Q[0], 6, p, metric=orc.L2)
    assert i1.tolist() == i2.tolist() and s1 == s2
    n1, d1 = orc.naive(X, Q[0], 6, metric=orc.L1)
    n2, d2 = orc.naive(X, Q[0], 6, metric=orc.L2)
    assert n1.tolist() == n2.tolist() and np.array_equal(d1 * 255.0, d2)


def test_l1_two_valued_f32_equals_l2(orc):
    """Float data in {0, 1}: |d| = d^2 and R'_l1 = R'_l2, so l1 and l2 agree
    exactly (with the same F)."""
    X, Q, _ = pm_half(22, 500, 96)
    Xf, qf = (X // 255).astype(np.float32), (Q[0] // 255).astype(np.float32)
    assert orc.scaling(Xf, qf, metric=orc.L1) == orc.scaling(Xf, qf, metric=orc.L2)
    for kw in (dict(), dict(sampling=1, c_exact=4)):
        p = orc.make_params(h=3, delta=0.05, seed=8, **kw)
        i1, s1 = orc.adaptive(Xf, qf, 4, p, metric=orc.L1)
        i2, s2 = orc.adaptive(Xf, qf, 4, p, metric=orc.L2)
        assert i1.tolist() == i2.tolist() and s1 == s2


def test_l1_unbiased_estimator(orc):
    """Lemma 3's premise for l1 samples: E d^(T) = d / (m W)."""
    X, Q = uniform_u8(8, 200, 128)
    d = brute_l1(X, Q[0]) / (128 * 255.0)
    est = []
    for seed in range(300):
        _, _, (S, _, _) = orc.adaptive(X, Q[0], 5, orc.make_params(seed=seed), stop_after=1, dump=True,
                                       metric=orc.L1)
        est.append(S / (64 * 255.0))
    est = np.array(est)
    se = est.std(axis=0, ddof=1) / np.sqrt(est.shape[0])
    z = (est.mean(axis=0) - d) / se
    assert np.max(np.abs(z)) < 5.0
    assert abs(z.mean() * np.sqrt(len(z))) < 4.0


@pytest.mark.parametrize("seed", range(8))
def test_l1_contains_knn_bruteforce(orc, seed):
    g = rng(300 + seed)
    n, m = int(g.integers(50, 400)), int(g.choice([16, 64, 200, 256]))
    k = int(g.integers(1, 8))
    h = int(g.integers(0, 6))
    X, Q, _ = tiny(seed=400 + seed, n=n, m=m, planted=max(1, k), noise=int(g.integers(1, 40)))
    d = brute_l1(X, Q[0])
    for c_exact in (0, k + h):
        for sampling in (0, 1):
            p = orc.make_params(h=h, delta=0.05, seed=seed, b0=4 * int(g.integers(1, 9)),
                                growth=float(g.choice([1.5, 2.0, 3.0])), c_exact=c_exact, sampling=sampling)
            idx, st = orc.adaptive(X, Q[0], k, p, metric=orc.L1)
            assert len(idx) <= k + h and len(set(idx.tolist())) == len(idx)
            assert contains_knn(idx, d, k)
            assert st["coord_evals"] <= n * (2 * m + 4)


def test_l1_f32_contains(orc):
    g = rng(31)
    X = g.uniform(-0.5, 0.5, size=(600, 96)).astype(np.float32)
    q = g.uniform(-0.5, 0.5, size=96).astype(np.float32)
    near = g.choice(600, size=5, replace=False)
    X[near] = np.clip(q + g.uniform(-0.02, 0.02, size=(5, 96)), -0.5, 0.5).astype(np.float32)
    d = brute_l1(X, q)
    for sampling in (0, 1):
        idx, _ = orc.adaptive(X, q, 5, orc.make_params(h=5, delta=0.05, seed=3, sampling=sampling),
                              metric=orc.L1)
        assert contains_knn(idx, d, 5, rtol=1e-9)


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_l1_naive_matches_numpy(orc, dtype):
    g = rng(41)
    if dtype == "u8":
        X = g.integers(0, 256, size=(500, 77), dtype=np.uint8)
        q = g.integers(0, 256, size=77, dtype=np.uint8)
    else:
        X = g.standard_normal((500, 77)).astype(np.float32)
        q = g.standard_normal(77).astype(np.float32)
    d = brute_l1(X, q)
    idx, dist = orc.naive(X, q, 12, metric=orc.L1)
    order = np.lexsort((np.arange(500), d))[:12]
    assert idx.tolist() == order.tolist()
    if dtype == "u8":
        assert np.array_equal(dist, d[order].astype(np.float64))
    else:
        assert np.allclose(dist, d[order], rtol=1e-12, atol=0)
    for i in (0, 17, 499):
        assert orc.exact_dist(X, q, i, metric=orc.L1) == pytest.approx(float(d[i]), rel=1e-12)


def test_l1_one_dimension_orders_like_l2(orc):
    """m = 1: |d| = sqrt(d^2), so the naive l1 and l2 scans rank alike."""
    g = rng(42)
    X = g.integers(0, 256, size=(300, 1), dtype=np.uint8)
    q = np.array([100], dtype=np.uint8)
    i1, d1 = orc.naive(X, q, 20, metric=orc.L1)
    i2, d2 = orc.naive(X, q, 20, metric=orc.L2)
    assert i1.tolist() == i2.tolist() and np.array_equal(d1 * d1, d2)


@pytest.mark.parametrize("seed", range(3))
def test_l1_alg1_contains_knn(orc, seed):
    X, Q, _ = tiny(seed=500 + seed, n=300, m=128, planted=4, noise=10)
    d = brute_l1(X, Q[0])
    idx, st, T = orc.alg1(X, Q[0], 4, orc.make_params(h=4, delta=0.05, seed=seed), metric=orc.L1)
    assert contains_knn(idx, d, 4)
    assert st["coord_evals"] == int(T.sum()) + 128 * st["exact_points"]
