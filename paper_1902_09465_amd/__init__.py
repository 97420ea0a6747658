"""MI355X-native adaptive k-nearest-neighbour search (LeJeune, Baraniuk,
Heckel, AISTATS 2019): Python binding of libknn.

    from paper_1902_09465_amd import KnnDB, default_params
    db = KnnDB(X)                          # X: cuda uint8/float32 [n, m]
    idx, count, stats = db.adaptive(Q, k=10, params=default_params(delta=0.01))
    nidx, ndist = db.naive(Q, k=10)
"""
from ._lib import (KNN_MAX_KH, KNN_MAX_ROUNDS, KnnError, Params, Stats, default_params,  # noqa: F401
                   lib)
from .api import KnnDB, Session, schedule  # noqa: F401
