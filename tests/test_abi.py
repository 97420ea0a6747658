"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, and its host-side schedule/widths equal the oracle's."""
from __future__ import annotations

import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def knnlib():
    import paper_1902_09465_amd as P
    try:
        P.lib()
    except ImportError:
        from paper_1902_09465_amd import build
        build.build()
    return P


def test_exports_every_declared_symbol(knnlib):
    hdr = open(os.path.join(ROOT, "include", "knn.h")).read()
    names = sorted(set(re.findall(r"^(?:int|void|const char \*)\s*\*?\s*(knn_\w+)\s*\(", hdr, re.M)))
    assert len(names) >= 14
    L = knnlib.lib()
    missing = [n for n in names if getattr(L, n, None) is None]
    assert not missing, missing


@pytest.mark.parametrize("kind,delta,n,m,b0,g,theta,c", [
    (0, 0.01, 2000, 256, 64, 2.0, 1.0, 0.0), (0, 0.01, 100_000, 3072, 64, 2.0, 1.0, 0.0),
    (0, 0.05, 1_000_000, 128, 16, 1.5, 1.0, 0.0), (1, 0.01, 250_000, 1024, 8, 3.0, 0.7, 0.0),
    (0, 0.9, 1, 500, 4, 2.0, 1.0, 0.0), (2, 0.001, 1000, 12288, 64, 2.0, 1.0, 1e-3),
    (0, 0.001, 1000, 12288, 4, 1.25, 1.0, 0.0)])
def test_schedule_and_widths_equal_oracle(knnlib, orc, kind, delta, n, m, b0, g, theta, c):
    p = knnlib.default_params(delta=delta, alpha_kind=kind, b0=b0, growth=g, theta_exact=theta, c_alpha=c)
    T, A = knnlib.schedule(p, n, m)
    To = orc.schedule(b0, g, theta, m)
    assert T.tolist() == To.tolist()
    for t, a in zip(T, A):
        assert a == orc.alpha(kind, int(t), n, delta, c)  # bit-exact


def test_invalid_params_rejected(knnlib):
    from paper_1902_09465_amd import KnnError
    for kw in (dict(b0=6), dict(delta=0.0), dict(delta=1.0), dict(growth=0.5),
               dict(alpha_kind=2, c_alpha=0.0), dict(alpha_kind=7), dict(b0=4, growth=1.0)):
        with pytest.raises(KnnError):
            knnlib.schedule(knnlib.default_params(**kw), 1000, 1 << 20)
