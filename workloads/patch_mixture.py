"""Seeded synthetic inputs: a mixture of local linear patches.

Input generation only.  Nothing here computes any step of the search
method; both the CPU oracle and the GPU path consume these arrays.

Each vector is ``c_g + U_g z + noise`` where

* ``c_g ~ N(0, I_d)`` is the patch centre,
* ``U_g`` is a d x m matrix with orthonormal columns (Q factor of the QR
  decomposition of an N(0,1) matrix, signs fixed so that diag(R) > 0),
* ``z_i ~ N(0, 4 * 0.85**i)`` for i < m (the second argument is the
  variance),
* noise is isotropic with standard deviation 0.05.

Members are drawn and summed in float32 (the stored precision).

Random streams are numpy ``PCG64`` generators keyed by
``SeedSequence(seed, spawn_key=...)`` so any patch (and hence any row) can be
regenerated on its own without materialising the whole data set:

* ``(0, g)``  patch parameters (centre, basis) from the *data* seed
* ``(1, g)``  members of patch g (data seed: corpus, query seed: queries)
* ``(2,)``    patch labels (which patch each row / query belongs to)
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np
from threadpoolctl import threadpool_limits

SIGNAL_VAR_BASE = 4.0
SIGNAL_VAR_DECAY = 0.85
NOISE_STD = 0.05
PATCH_DIM = 32


def _rng(seed: int, *key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=tuple(key))))


def signal_std(m: int = PATCH_DIM) -> np.ndarray:
    return np.sqrt(SIGNAL_VAR_BASE * SIGNAL_VAR_DECAY ** np.arange(m))


def patch_params(seed: int, g: int, d: int, m: int = PATCH_DIM):
    """Centre (d,) and orthonormal basis U (d, m) of patch g, float64."""
    rng = _rng(seed, 0, g)
    centre = rng.standard_normal(d)
    a = rng.standard_normal((d, m))
    q, r = np.linalg.qr(a)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return centre, q * s


def patch_members(seed: int, g: int, n: int, centre, U, noise_std=NOISE_STD) -> np.ndarray:
    """n members of patch g as float32 rows."""
    d, m = U.shape
    rng = _rng(seed, 1, g)
    z = rng.standard_normal((n, m), dtype=np.float32) * signal_std(m).astype(np.float32)
    x = rng.standard_normal((n, d), dtype=np.float32)
    x *= np.float32(noise_std)
    x += centre.astype(np.float32)[None, :]
    x += z @ U.T.astype(np.float32)
    return x


def zipf_sizes(n_total: int, n_patches: int, s: float, lo: int, hi: int, seed: int) -> np.ndarray:
    """Clamped rank-Zipf patch sizes n_j = clamp(c * j**-s, lo, hi) summing to n_total.

    The constant c is found by bisection; largest-remainder rounding makes the
    sizes integers with the exact total.  The patch index is a seeded
    permutation of the rank.
    """
    ranks = np.arange(1, n_patches + 1, dtype=np.float64)
    base = ranks ** (-s)

    def total(c):
        return np.clip(c * base, lo, hi).sum()

    a, b = 0.0, float(n_total) * 10
    for _ in range(200):
        mid = 0.5 * (a + b)
        if total(mid) < n_total:
            a = mid
        else:
            b = mid
    x = np.clip(b * base, lo, hi)
    fl = np.floor(x).astype(np.int64)
    rem = n_total - int(fl.sum())
    if rem > 0:
        frac = x - fl
        # largest remainders first; ties to lower rank; never exceed hi
        order = np.lexsort((ranks, -frac))
        order = [i for i in order if fl[i] < hi]
        for i in order[:rem]:
            fl[i] += 1
    elif rem < 0:
        frac = x - fl
        order = [i for i in np.lexsort((ranks, frac)) if fl[i] > lo]
        for i in order[: -rem]:
            fl[i] -= 1
    perm = _rng(seed, 5).permutation(n_patches)
    sizes = np.empty(n_patches, dtype=np.int64)
    sizes[perm] = fl
    return sizes


@dataclass
class Mixture:
    """A generated corpus: rows X (N, d) float32 and their patch labels."""

    X: np.ndarray
    labels: np.ndarray
    n_patches: int
    seed: int


def _threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def uniform_mixture(n: int, d: int, n_patches: int, seed: int, threads: int | None = None) -> Mixture:
    """Rows with i.i.d. uniform patch labels (corpus of the 10k and 1M workloads)."""
    labels = _rng(seed, 2).integers(0, n_patches, size=n)
    X = np.empty((n, d), dtype=np.float32)
    _fill_from(X, labels, seed, seed, d, n_patches, threads or _threads())
    return Mixture(X, labels, n_patches, seed)


def uniform_queries(nq: int, d: int, n_patches: int, data_seed: int, query_seed: int,
                    threads: int | None = None) -> Mixture:
    """Fresh draws from the same mixture: patch parameters from the data seed,
    labels and members from the query seed."""
    labels = _rng(query_seed, 2).integers(0, n_patches, size=nq)
    Q = np.empty((nq, d), dtype=np.float32)
    _fill_from(Q, labels, data_seed, query_seed, d, n_patches, threads or _threads())
    return Mixture(Q, labels, n_patches, query_seed)


def _fill_from(Y, labels, param_seed, member_seed, d, n_patches, threads, m=PATCH_DIM):
    order = np.argsort(labels, kind="stable")
    counts = np.bincount(labels, minlength=n_patches)
    starts = np.concatenate([[0], np.cumsum(counts)])

    def work(g):
        n = int(counts[g])
        if n == 0:
            return
        centre, U = patch_params(param_seed, g, d, m)
        rows = order[starts[g]:starts[g + 1]]
        Y[rows] = patch_members(member_seed, g, n, centre, U)

    with threadpool_limits(1):
        if threads <= 1:
            for g in range(n_patches):
                work(g)
        else:
            with ThreadPoolExecutor(threads) as ex:
                list(ex.map(work, range(n_patches)))


def zipf_mixture(n: int, d: int, n_patches: int, seed: int, s: float = 1.1, lo: int = 16,
                 hi: int = 20000, threads: int | None = None) -> Mixture:
    """Rows whose patch sizes follow the clamped rank-Zipf rule; row order is a
    seeded shuffle of the labels."""
    sizes = zipf_sizes(n, n_patches, s, lo, hi, seed)
    labels = np.repeat(np.arange(n_patches), sizes)
    labels = labels[_rng(seed, 6).permutation(n)]
    X = np.empty((n, d), dtype=np.float32)
    _fill_from(X, labels, seed, seed, d, n_patches, threads or _threads())
    return Mixture(X, labels, n_patches, seed)


def zipf_queries(nq: int, d: int, sizes: np.ndarray, data_seed: int, query_seed: int,
                 threads: int | None = None) -> Mixture:
    """Queries whose patch is drawn proportionally to the patch size."""
    p = sizes / sizes.sum()
    labels = _rng(query_seed, 2).choice(len(sizes), size=nq, p=p)
    Q = np.empty((nq, d), dtype=np.float32)
    _fill_from(Q, labels, data_seed, query_seed, d, len(sizes), threads or _threads())
    return Mixture(Q, labels, len(sizes), query_seed)


BYTE_SCALE = 32.0
BYTE_OFFSET = 24.0


def byte_valued(m: Mixture) -> Mixture:
    """A SIFT1M-shaped stand-in: the mixture mapped affinely to non-negative
    byte values, x -> clip(rint(32 x + 24), 0, 255), stored as float32 (about
    a quarter of the components clip at 0, as in gradient-histogram
    descriptors)."""
    X = np.clip(np.rint(m.X * BYTE_SCALE + BYTE_OFFSET), 0.0, 255.0).astype(np.float32)
    return Mixture(X, m.labels, m.n_patches, m.seed)


def isotropic(n: int, d: int, seed: int) -> np.ndarray:
    """Isotropic standard Gaussian rows (the isotropic data set of the paper's
    recall table)."""
    return _rng(seed, 7).standard_normal((n, d)).astype(np.float32)


def uniform_rows(n: int, d: int, seed: int, lo=-1.0, hi=1.0) -> np.ndarray:
    """Small unstructured inputs for edge-case tests."""
    return _rng(seed, 8).uniform(lo, hi, size=(n, d)).astype(np.float32)


def uniform_floats(shape, seed: int, key: int = 9, lo=-1.0, hi=1.0, dtype=np.float32):
    return _rng(seed, key).uniform(lo, hi, size=shape).astype(dtype)


def ints(shape, seed: int, lo: int, hi: int, key: int = 10):
    return _rng(seed, key).integers(lo, hi, size=shape)


def log_uniform_batches(total: int, lo: int, hi: int, fixed, seed: int):
    """Uneven query-batch sizes: the fixed sizes first, then log-uniform draws
    in [lo, hi] until ``total`` queries are covered (the last one trimmed)."""
    out = [int(x) for x in fixed]
    rng = _rng(seed, 11)
    while sum(out) < total:
        out.append(int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))))))
    s = sum(out)
    if s > total:
        out[-1] -= s - total
        if out[-1] <= 0:
            out.pop()
    return out
