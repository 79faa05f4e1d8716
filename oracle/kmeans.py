"""Grain partitioning by k-means (oracle, FP64).

The paper splits the corpus into local, coherent grains (Sections 1 and 2.2)
without naming the partitioning method; the grains here are k-means clusters:

1. seeding: greedy k-means++ (Arthur & Vassilvitskii 2007) with
   ``2 + floor(ln G)`` local trials per step;
2. Lloyd iterations on a training sample of at most ``train_per_grain * G``
   rows: assign each row to the centroid with the smallest squared Euclidean
   distance (ties to the lower grain index), then move each centroid to the
   mean of its members; an empty grain is re-seeded with the training row
   farthest from its own centroid (ties to the lower row index); stop when no
   assignment changes or after ``max_iter`` iterations;
3. a final assignment of every row, and each centroid set to the exact mean
   of its final members, so that mean centering (eq. 1) is exact.

Parity: the GPU build's k-means is not compared vector by vector (floating
point summation order can change the local optimum it reaches).  It is judged
by inertia and by the invariants of the index it produces.  Pins: recovery of
well-separated clusters, non-increasing inertia, brute-force assignment.
"""
from __future__ import annotations

import math

import numpy as np


def sq_dists(X: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Squared Euclidean distances (n, G) in float64."""
    X = np.asarray(X, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    xx = np.einsum("ij,ij->i", X, X)[:, None]
    cc = np.einsum("ij,ij->i", C, C)[None, :]
    D = xx + cc - 2.0 * (X @ C.T)
    np.maximum(D, 0.0, out=D)
    return D


def assign(X: np.ndarray, C: np.ndarray, chunk: int = 65536):
    """Nearest centroid per row (ties to the lower index) and its distance."""
    n = X.shape[0]
    lab = np.empty(n, dtype=np.int64)
    dmin = np.empty(n, dtype=np.float64)
    for s in range(0, n, chunk):
        D = sq_dists(X[s:s + chunk], C)
        a = np.argmin(D, axis=1)  # argmin returns the first (lowest) index on ties
        lab[s:s + chunk] = a
        dmin[s:s + chunk] = D[np.arange(D.shape[0]), a]
    return lab, dmin


def kmeanspp(X: np.ndarray, G: int, rng: np.random.Generator) -> np.ndarray:
    """Greedy k-means++ seeding; returns G centroids (float64)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    trials = 2 + int(math.log(G))
    first = int(rng.integers(n))
    centers = [X[first].copy()]
    closest = sq_dists(X, X[first:first + 1])[:, 0]
    for _ in range(1, G):
        total = closest.sum()
        if total <= 0.0:
            cand = rng.integers(n, size=trials)
        else:
            u = rng.random(trials) * total
            cand = np.searchsorted(np.cumsum(closest), u, side="right")
            cand = np.minimum(cand, n - 1)
        best_pot, best = None, None
        for c in cand:
            nd = np.minimum(closest, sq_dists(X, X[c:c + 1])[:, 0])
            pot = nd.sum()
            if best_pot is None or pot < best_pot:
                best_pot, best, best_nd = pot, int(c), nd
        centers.append(X[best].copy())
        closest = best_nd
    return np.stack(centers)


def member_means(X: np.ndarray, lab: np.ndarray, G: int, fallback: np.ndarray) -> np.ndarray:
    X = np.asarray(X, dtype=np.float64)
    cnt = np.bincount(lab, minlength=G).astype(np.float64)
    S = np.zeros((G, X.shape[1]), dtype=np.float64)
    np.add.at(S, lab, X)
    out = fallback.astype(np.float64).copy()
    nz = cnt > 0
    out[nz] = S[nz] / cnt[nz, None]
    return out


def lloyd(X: np.ndarray, C0: np.ndarray, max_iter: int = 50):
    """Lloyd iterations from centroids C0.  Returns (centroids, labels, iters, inertia history)."""
    X = np.asarray(X, dtype=np.float64)
    C = np.asarray(C0, dtype=np.float64).copy()
    G = C.shape[0]
    lab, dmin = assign(X, C)
    history = [float(dmin.sum())]
    it = 0
    for it in range(1, max_iter + 1):
        C = member_means(X, lab, G, C)
        cnt = np.bincount(lab, minlength=G)
        if (cnt == 0).any():
            # re-seed each empty grain with the row farthest from its centroid
            taken = set()
            for g in np.nonzero(cnt == 0)[0]:
                order = np.lexsort((np.arange(len(dmin)), -dmin))
                for i in order:
                    if int(i) not in taken:
                        taken.add(int(i))
                        C[g] = X[i]
                        dmin[i] = 0.0
                        break
        new_lab, dmin = assign(X, C)
        history.append(float(dmin.sum()))
        changed = int((new_lab != lab).sum())
        lab = new_lab
        if changed == 0:
            break
    return C, lab, it, history


def kmeans(X: np.ndarray, G: int, seed: int, max_iter: int = 50, train_per_grain: int = 256,
           init: np.ndarray | None = None):
    """Full grain partitioning.  Returns (centroids fp64, labels of all rows)."""
    X = np.asarray(X)
    n = X.shape[0]
    if G < 1 or G > n:
        raise ValueError("need 1 <= G <= N")
    rng = np.random.default_rng(seed)
    n_train = min(n, train_per_grain * G)
    if n_train < n:
        tr = np.sort(rng.choice(n, size=n_train, replace=False))
        Xt = np.asarray(X[tr], dtype=np.float64)
    else:
        Xt = np.asarray(X, dtype=np.float64)
    C0 = kmeanspp(Xt, G, rng) if init is None else np.asarray(init, dtype=np.float64)
    C, _, _, _ = lloyd(Xt, C0, max_iter)
    lab, _ = assign(np.asarray(X, dtype=np.float64), C)
    C = member_means(X, lab, G, C)
    return C, lab


def inertia(X, C, lab) -> float:
    X = np.asarray(X, dtype=np.float64)
    return float(((X - np.asarray(C, dtype=np.float64)[lab]) ** 2).sum())
