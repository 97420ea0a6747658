"""Workload generators.

Every function returns plain numpy arrays:
  X : (n, m) uint8 or float32, point-major
  Q : (nq, m) same dtype
plus, where it applies, a per-query k array.

The shapes and value distributions follow the paper's experimental setup
(Section 5: subspace data x = c Q y, n = 1000, m = 12288) and the
benchmark configurations below.  Points are drawn in chunks so that the
large configurations do not need float64 copies of the whole matrix.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng", "tiny", "gmm_u8", "gmm_f32", "uniform_u8", "uneven", "antipodal",
    "subspace", "pm_half", "coherent", "gap_family", "planted_corners", "easy_corners", "serving_dbs", "CONFIGS",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def tiny(seed: int = 1000, n: int = 2000, m: int = 256, planted: int = 5, noise: int = 8):
    """n points uniform in {0..255}^m, one query, `planted` points equal to the
    query plus integer noise in [-noise, noise] (clipped), at random indices."""
    g = rng(seed)
    X = g.integers(0, 256, size=(n, m), dtype=np.int64)
    q = g.integers(0, 256, size=(m,), dtype=np.int64)
    where = g.choice(n, size=planted, replace=False)
    for i in where:
        X[i] = np.clip(q + g.integers(-noise, noise + 1, size=m), 0, 255)
    return X.astype(np.uint8), q.astype(np.uint8)[None, :], np.sort(where)


def _mixture_u8(g, count, centres, sigma, chunk=8192):
    out = np.empty((count, centres.shape[1]), dtype=np.uint8)
    comp = g.integers(0, centres.shape[0], size=count)
    for s in range(0, count, chunk):
        e = min(count, s + chunk)
        v = centres[comp[s:e]] + g.standard_normal((e - s, centres.shape[1]), dtype=np.float32) * sigma
        out[s:e] = np.clip(np.rint(v), 0, 255).astype(np.uint8)
    return out


def gmm_u8(seed: int = 2000, n: int = 100_000, m: int = 3072, n_centres: int = 32,
           sigma: float = 30.0, nq: int = 1024):
    """Gaussian mixture in {0..255}^m: centres uniform in [0,255], isotropic
    sigma, rounded and clipped; queries from the same mixture."""
    g = rng(seed)
    centres = g.uniform(0.0, 255.0, size=(n_centres, m)).astype(np.float32)
    X = _mixture_u8(g, n, centres, sigma)
    Q = _mixture_u8(g, nq, centres, sigma)
    return X, Q


def gmm_f32(seed: int = 3000, n: int = 1_000_000, m: int = 128, n_centres: int = 1000,
            sigma: float = 0.1, nq: int = 10_000, chunk: int = 65536):
    """Float mixture: centres N(0, 1)^m, points and queries centre + N(0, sigma^2)."""
    g = rng(seed)
    centres = g.standard_normal((n_centres, m), dtype=np.float32)

    def draw(count):
        out = np.empty((count, m), dtype=np.float32)
        comp = g.integers(0, n_centres, size=count)
        for s in range(0, count, chunk):
            e = min(count, s + chunk)
            out[s:e] = centres[comp[s:e]] + g.standard_normal((e - s, m), dtype=np.float32) * np.float32(sigma)
        return out

    return draw(n), draw(nq)


def uniform_u8(seed: int, n: int, m: int, nq: int = 1):
    g = rng(seed)
    return (g.integers(0, 256, size=(n, m), dtype=np.uint8),
            g.integers(0, 256, size=(nq, m), dtype=np.uint8))


def uneven(seed: int = 4000, n: int = 250_000, m: int = 1024, nq: int = 4096,
           ks=(1, 10, 100), noise: int = 8):
    """Half easy, half hard queries over one shared u8 database.

    Bulk points are random corners of {0,255}^m.  Each easy query is a random
    corner that owns k planted points (the corner moved inwards by integer
    noise in [0, noise]) inserted into the database.  Hard queries are drawn
    from {127,128}^m, so every corner point sits at nearly the same distance.
    k cycles through `ks`."""
    g = rng(seed)
    n_easy = nq // 2
    kq = np.array([ks[i % len(ks)] for i in range(nq)], dtype=np.int32)
    planted_total = int(kq[:n_easy].sum())
    if planted_total > n:
        raise ValueError("database too small for the planted points")
    X = (g.integers(0, 2, size=(n, m), dtype=np.uint8) * np.uint8(255))
    Q = np.empty((nq, m), dtype=np.uint8)
    slots = g.permutation(n)[:planted_total]
    pos = 0
    for qi in range(n_easy):
        c = g.integers(0, 2, size=m, dtype=np.uint8) * np.uint8(255)
        Q[qi] = c
        for _ in range(int(kq[qi])):
            d = g.integers(0, noise + 1, size=m).astype(np.int16)
            v = np.where(c == 255, 255 - d, d).astype(np.uint8)
            X[slots[pos]] = v
            pos += 1
    Q[n_easy:] = 127 + g.integers(0, 2, size=(nq - n_easy, m), dtype=np.uint8)
    return X, Q, kq


def easy_corners(seed: int, n: int, m: int, nq: int, k: int = 10, noise: int = 8, chunk: int = 8192):
    """The easy half of the uneven workload on its own: bulk points are random
    corners of {0,255}^m; each of the nq queries is a random corner that owns
    k planted points (the corner moved inwards by integer noise in
    [0, noise]) at random indices.  Returns (X, Q)."""
    g = rng(seed)
    if nq * k > n:
        raise ValueError("database too small for the planted points")
    X = np.empty((n, m), dtype=np.uint8)
    for s0 in range(0, n, chunk):
        e = min(n, s0 + chunk)
        X[s0:e] = g.integers(0, 2, size=(e - s0, m), dtype=np.uint8) * np.uint8(255)
    Q = g.integers(0, 2, size=(nq, m), dtype=np.uint8) * np.uint8(255)
    slots = g.permutation(n)[:nq * k]
    for qi in range(nq):
        d = g.integers(0, noise + 1, size=(k, m)).astype(np.int16)
        c = Q[qi].astype(np.int16)[None, :]
        X[slots[qi * k:(qi + 1) * k]] = np.where(c == 255, 255 - d, d).astype(np.uint8)
    return X, Q


def antipodal(seed: int = 7, n: int = 1000, m: int = 1024, copies: int = 5):
    """RNG-free worked example: the query is a random corner of {0,255}^m,
    `copies` points equal the query (every sample 0) and the rest are its
    antipode 255 - q (every sample (255)^2, i.e. normalised 1)."""
    g = rng(seed)
    q = g.integers(0, 2, size=m, dtype=np.uint8) * np.uint8(255)
    X = np.repeat((255 - q)[None, :], n, axis=0)
    where = np.sort(g.choice(n, size=copies, replace=False))
    X[where] = q
    return X, q[None, :], where


def subspace(seed: int, n: int = 1000, m: int = 12288, p: int = 10, nq: int = 1):
    """Section 5 synthetic data: x = c Q y with Q an m x p Gaussian matrix with
    unit-norm columns, y uniform on the unit sphere of R^p, and c the largest
    scalar keeping every coordinate within [-1/2, 1/2].  Returned as float32."""
    g = rng(seed)
    Qm = g.standard_normal((m, p))
    Qm /= np.linalg.norm(Qm, axis=0, keepdims=True)
    Y = g.standard_normal((n + nq, p))
    Y /= np.linalg.norm(Y, axis=1, keepdims=True)
    V = Y @ Qm.T
    c = 0.5 / np.abs(V).max()
    V = (c * V).astype(np.float32)
    return V[:n].copy(), V[n:].copy()


def pm_half(seed: int, n: int, m: int, dists=None):
    """Points with coordinates in {-1/2, +1/2} (the data class of Theorem 2),
    encoded as u8 {0, 255}.  If `dists` (length n, values in [0,1]) is given,
    point i differs from the query in round(dists[i] * m) coordinates, so its
    normalised distance is exactly that fraction."""
    g = rng(seed)
    q = g.integers(0, 2, size=m, dtype=np.uint8) * np.uint8(255)
    X = np.repeat(q[None, :], n, axis=0)
    if dists is None:
        dists = g.uniform(0, 1, size=n)
    flips = np.rint(np.asarray(dists) * m).astype(np.int64)
    for i in range(n):
        idx = g.choice(m, size=int(flips[i]), replace=False)
        X[i, idx] = 255 - X[i, idx]
    return X, q[None, :], flips


def planted_corners(seed: int, n: int, m: int, nq: int, near, gaps, mid: int = 3,
                    mid_gap: float = 0.12):
    """Many queries over one database of corners of {0,255}^m, each query with
    its own near points at its own distance.

    Bulk points and queries are random corners, so every bulk point differs
    from every query in about half of the coordinates.  Query j owns near[j]
    points that differ from it in round((gaps[j] + 0.01 t) m) coordinates
    (t = 0, 1, ...) and `mid` points at gaps[j] + mid_gap + 0.05 t, placed at
    random indices.  Returns (X, Q)."""
    g = rng(seed)
    X = g.integers(0, 2, size=(n, m), dtype=np.uint8) * np.uint8(255)
    Q = g.integers(0, 2, size=(nq, m), dtype=np.uint8) * np.uint8(255)
    total = int(np.sum(near)) + mid * nq
    if total > n:
        raise ValueError("database too small for the planted points")
    slots = g.permutation(n)[:total]
    pos = 0
    for j in range(nq):
        fr = [gaps[j] + 0.01 * t for t in range(int(near[j]))]
        fr += [gaps[j] + mid_gap + 0.05 * t for t in range(mid)]
        for f in fr:
            x = Q[j].copy()
            idx = g.choice(m, size=int(np.rint(min(f, 1.0) * m)), replace=False)
            x[idx] = 255 - x[idx]
            X[slots[pos]] = x
            pos += 1
    return X, Q


def coherent(seed: int, n: int, m: int):
    """All points and the query on one coordinate axis (the coherent example
    of Section 4.2): only coordinate 0 varies."""
    g = rng(seed)
    X = np.zeros((n, m), dtype=np.uint8)
    X[:, 0] = g.integers(0, 256, size=n, dtype=np.uint8)
    q = np.zeros((1, m), dtype=np.uint8)
    q[0, 0] = g.integers(0, 256)
    return X, q


def gap_family(seed: int, n: int = 600, m: int = 256, k: int = 5, near: int = 5,
               mid: int = 40, near_noise: int = 40, mid_noise: int = 90):
    """Instances with a spread of gaps: `near` points close to the query, `mid`
    points at intermediate distance, the rest uniform.  Used by the miss-rate
    tests, where decisions must be taken before the exact round."""
    g = rng(seed)
    q = g.integers(0, 256, size=m, dtype=np.int64)
    X = g.integers(0, 256, size=(n, m), dtype=np.int64)
    perm = g.permutation(n)
    for i in perm[:near]:
        X[i] = np.clip(q + g.integers(-near_noise, near_noise + 1, size=m), 0, 255)
    for i in perm[near:near + mid]:
        X[i] = np.clip(q + g.integers(-mid_noise, mid_noise + 1, size=m), 0, 255)
    return X.astype(np.uint8), q.astype(np.uint8)[None, :]


def serving_dbs(seed: int = 5000, scale: float = 1.0):
    """The three resident serving databases (sizes scaled by `scale`):
    A: 50,000 x 784 u8, 10-component mixture, sigma 30;
    B: 500,000 x 256 f32, 1,000 clusters, sigma 0.1;
    C: 2,000,000 x 96 f32, 1,000 clusters, sigma 0.1."""
    nA, nB, nC = (max(64, int(v * scale)) for v in (50_000, 500_000, 2_000_000))
    XA, QA = gmm_u8(seed, n=nA, m=784, n_centres=10, sigma=30.0, nq=256)
    XB, QB = gmm_f32(seed + 1, n=nB, m=256, n_centres=1000, sigma=0.1, nq=256)
    XC, QC = gmm_f32(seed + 2, n=nC, m=96, n_centres=1000, sigma=0.1, nq=256)
    return [(XA, QA), (XB, QB), (XC, QC)]


# The five benchmark configurations (shapes and parameters).
CONFIGS = {
    "tiny": dict(n=2000, m=256, dtype="u8", nq=1, k=5, delta=0.01),
    "batched_int": dict(n=100_000, m=3072, dtype="u8", nq=1024, k=10, delta=0.01),
    "float": dict(n=1_000_000, m=128, dtype="f32", nq=10_000, k=10, delta=0.05),
    "uneven": dict(n=250_000, m=1024, dtype="u8", nq=4096, k=(1, 10, 100), delta=0.01),
    "serving": dict(dbs=((50_000, 784, "u8"), (500_000, 256, "f32"), (2_000_000, 96, "f32"))),
}
