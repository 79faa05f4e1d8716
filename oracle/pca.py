"""Local PCA basis of one grain (oracle, FP64).

Section 2.2: each grain with centroid mu_g gets a local PCA basis W_g whose r
columns span the grain's dominant directions (the paper writes the subspace
dimension as k; here it is r, and k is the number of results).

Definition used: the covariance ``S_g = (1/n_g) * sum_i (x_i - mu_g)(x_i - mu_g)^T``
in float64, its eigen-decomposition by LAPACK ``eigh`` (the library routine),
eigenpairs sorted by descending eigenvalue, and ``W_g`` = the top-r
eigenvectors.  Sign convention (the paper is silent; no distance depends on
it): the entry of largest magnitude in each column is positive, ties to the
lower index.  A grain with n_g <= r has a rank-deficient covariance; ``eigh``
still returns a full orthonormal eigenbasis, so W_g is completed by null-space
vectors automatically.

The captured-variance fraction is ``sum(top-r eigenvalues) / trace(S_g)``
(the quantity of the paper's recall table, "PCA Var. Captured").

Pins: orthonormal columns, eigen-equation residual, the isotropic 6.5% value
of the recall table, the analytic bound for the patch mixture.
"""
from __future__ import annotations

import numpy as np


def covariance(Xg: np.ndarray, mu: np.ndarray) -> np.ndarray:
    Xc = np.asarray(Xg, dtype=np.float64) - np.asarray(mu, dtype=np.float64)[None, :]
    return (Xc.T @ Xc) / max(1, Xc.shape[0])


def fix_signs(W: np.ndarray) -> np.ndarray:
    W = W.copy()
    for j in range(W.shape[1]):
        i = int(np.argmax(np.abs(W[:, j])))  # first index of the maximum
        if W[i, j] < 0:
            W[:, j] = -W[:, j]
    return W


def local_pca(Xg: np.ndarray, mu: np.ndarray, r: int):
    """Returns (W (d, r) float64, eigenvalues (d,) descending, captured fraction)."""
    S = covariance(Xg, mu)
    evals, evecs = np.linalg.eigh(S)
    order = np.argsort(-evals, kind="stable")
    evals = evals[order]
    evecs = evecs[:, order]
    W = fix_signs(evecs[:, :r])
    tr = float(np.trace(S))
    captured = float(evals[:r].sum() / tr) if tr > 0 else 1.0
    return W, evals, captured
