"""Exact k-nearest neighbours (oracle ground truth).

The exact top-k of ``||q - x||^2`` over all N rows, ties to the lower id.
Candidates come from a float64 BLAS product (the expansion
``||q||^2 + ||x||^2 - 2 q.x``); the best ``k + extra`` of them are then
re-scored by float64 direct differences and ordered by (distance, id).  The
expansion only preselects: a row is missed only if its float64 expansion
error exceeds the gap to the (k+extra)-th distance, far beyond float64
rounding for these magnitudes.

Pins: a pure-Python double loop on tiny inputs.
"""
from __future__ import annotations

import numpy as np


def knn(X: np.ndarray, Q: np.ndarray, k: int, extra: int = 64, chunk_rows: int = 262144):
    Q64 = np.asarray(Q, dtype=np.float64)
    nq = Q64.shape[0]
    N = X.shape[0]
    m = min(N, k + extra)
    best_d = np.full((nq, m), np.inf)
    best_i = np.full((nq, m), -1, dtype=np.int64)
    qq = np.einsum("ij,ij->i", Q64, Q64)[:, None]
    for s in range(0, N, chunk_rows):
        Xc = np.asarray(X[s:s + chunk_rows], dtype=np.float64)
        xx = np.einsum("ij,ij->i", Xc, Xc)[None, :]
        D = qq + xx - 2.0 * (Q64 @ Xc.T)
        ids = np.arange(s, s + Xc.shape[0])
        allD = np.concatenate([best_d, D], axis=1)
        allI = np.concatenate([best_i, np.broadcast_to(ids, D.shape)], axis=1)
        part = np.argpartition(allD, m - 1, axis=1)[:, :m]
        best_d = np.take_along_axis(allD, part, 1)
        best_i = np.take_along_axis(allI, part, 1)
    ids = np.empty((nq, k), dtype=np.int64)
    dist = np.empty((nq, k))
    for i in range(nq):
        cand = best_i[i][best_i[i] >= 0]
        dd = ((np.asarray(X[cand], dtype=np.float64) - Q64[i][None, :]) ** 2).sum(axis=1)
        o = np.lexsort((cand, dd))[:k]
        ids[i] = cand[o]
        dist[i] = dd[o]
    return ids, dist
