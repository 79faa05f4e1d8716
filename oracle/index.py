"""Index construction (oracle, FP64) and the stored index format.

Follows the build side of Section 2.2 for every database vector x_i of grain g:

* eq. (1) mean centering      ``x' = x - mu_g``
* eq. (2) subspace projection ``z = W_g^T x'``        (r coordinates)
* eq. (3) residual            ``e = x' - W_g z``
* eq. (4) residual energy     ``eps = ||e||^2``

(The paper calls the residual energy r and the subspace dimension k; here they
are eps and r.)  The paper's int16 quantisation, eq. (5), is not part of the
FP32 form; FP32 codes are stored.

Stored format (shared contract with the GPU library, all float32 / int):

* ``centroids`` (G, d) f32 - mu_g
* ``basis``     (G, r, d) f32 - row j of grain g is the j-th column of W_g
* ``offsets``   (G+1,) int64 - grain g owns grain-order positions [off[g], off[g+1])
* ``perm``      (N,) int32 - grain-order position -> original row id; inside a
  grain, ids ascend
* ``codes``     (N, r) f32 - z_i in grain order
* ``eps``       (N,) f32 - eps_i in grain order

Pins: orthonormality, Pythagoras ``||x'||^2 = ||z||^2 + eps`` (exact for
orthonormal W), eps >= 0, r = d gives eps = 0.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import kmeans as km
from .pca import local_pca


@dataclass
class OracleIndex:
    centroids: np.ndarray      # (G, d) f64
    W: list                    # per grain (d, r) f64
    labels: np.ndarray         # (N,) grain of each original row
    offsets: np.ndarray        # (G+1,)
    perm: np.ndarray           # (N,)
    codes: np.ndarray          # (N, r) f64, grain order
    eps: np.ndarray            # (N,) f64, grain order
    captured: np.ndarray       # (G,) captured-variance fraction per grain
    evals: list                # per grain eigenvalues (descending)
    r: int

    def stored(self) -> dict:
        G = self.centroids.shape[0]
        d = self.centroids.shape[1]
        basis = np.zeros((G, self.r, d), dtype=np.float32)
        for g in range(G):
            basis[g] = self.W[g].T.astype(np.float32)
        return {
            "centroids": self.centroids.astype(np.float32),
            "basis": basis,
            "offsets": self.offsets.astype(np.int64),
            "perm": self.perm.astype(np.int32),
            "codes": self.codes.astype(np.float32),
            "eps": self.eps.astype(np.float32),
        }


def grain_order(labels: np.ndarray, G: int):
    """Stable grouping by grain: positions of each grain hold ascending ids."""
    perm = np.argsort(labels, kind="stable")
    counts = np.bincount(labels, minlength=G)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return perm, offsets


def encode(x: np.ndarray, mu: np.ndarray, W: np.ndarray):
    """eq. (1)-(4) for a batch of rows of one grain: returns (z, eps) float64."""
    xp = np.asarray(x, dtype=np.float64) - np.asarray(mu, dtype=np.float64)[None, :]   # eq. (1)
    z = xp @ W                                                                           # eq. (2)
    e = xp - z @ W.T                                                                     # eq. (3)
    eps = np.einsum("ij,ij->i", e, e)                                                    # eq. (4)
    return z, eps


def build(X: np.ndarray, G: int, r: int, seed: int, max_iter: int = 50,
          init_centroids: np.ndarray | None = None, labels: np.ndarray | None = None) -> OracleIndex:
    """k-means grains + per-grain local PCA + codes.

    ``labels`` may be given to use a fixed partition (e.g. one grain, or the
    generator's patch labels) instead of k-means; centroids are then the exact
    member means.
    """
    X = np.asarray(X)
    N, d = X.shape
    if not (1 <= r <= d):
        raise ValueError("need 1 <= r <= d")
    if labels is None:
        C, lab = km.kmeans(X, G, seed, max_iter=max_iter, init=init_centroids)
    else:
        lab = np.asarray(labels, dtype=np.int64)
        C = km.member_means(X, lab, G, np.zeros((G, d)))
    perm, offsets = grain_order(lab, G)
    codes = np.zeros((N, r), dtype=np.float64)
    eps = np.zeros(N, dtype=np.float64)
    Ws, evs = [], []
    captured = np.ones(G, dtype=np.float64)
    for g in range(G):
        a, b = int(offsets[g]), int(offsets[g + 1])
        rows = perm[a:b]
        if b > a:
            W, ev, cap = local_pca(X[rows], C[g], r)
        else:
            # empty grain: any orthonormal basis (never probed content)
            W = np.eye(d, r)
            ev, cap = np.zeros(d), 1.0
        Ws.append(W)
        evs.append(ev)
        captured[g] = cap
        if b > a:
            z, e = encode(X[rows], C[g], W)
            codes[a:b] = z
            eps[a:b] = e
    return OracleIndex(C, Ws, lab, offsets, perm, codes, eps, captured, evs, r)


def stored_encode(X: np.ndarray, stored: dict):
    """Recompute codes and eps in FP64 from stored centroids and basis (for
    checking an index whose basis came from elsewhere)."""
    off = stored["offsets"]
    perm = stored["perm"]
    r = stored["basis"].shape[1]
    codes = np.zeros((len(perm), r))
    eps = np.zeros(len(perm))
    for g in range(len(off) - 1):
        a, b = int(off[g]), int(off[g + 1])
        if b > a:
            W = stored["basis"][g].astype(np.float64).T
            z, e = encode(X[perm[a:b]], stored["centroids"][g], W)
            codes[a:b] = z
            eps[a:b] = e
    return codes, eps
