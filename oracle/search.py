"""HNTL search, step by step (oracle, FP64 on the stored index values).

Query lifecycle of Section 2.1 in Mode B (tiered filter; Mode A, the answer
from the index alone, replaces step 4 by ``answer_mode_a``), with the
hierarchical routing of Section 2.3:

1. ``route``   - squared Euclidean distance from q to every centroid mu_g;
   the P smallest, ordered by (distance, g).
2. ``project`` - for each probed grain: eq. (1) ``q' = q - mu_g``, eq. (2)
   ``z_q = W_g^T q'``, eq. (3) ``e_q = q' - W_g z_q``, eq. (4)
   ``eps_q = ||e_q||^2``.
3. ``scan_pool`` - eq. (6) score ``D_i = ||z_q - z_i||^2 + eps_q + eps_i`` for
   every member i of every probed grain; the candidate pool is the C smallest
   (D, id) over the union of the probed grains (ids are original row ids);
   fewer than C candidates are padded with (id -1, D +inf).
4. ``rerank``  - exact squared L2 ``||q - x_i||^2`` against the raw vectors of
   the pool; the k smallest (distance, id).

Each stage accepts the previous stage's output as an argument, so any stage
can be checked on its own.  The quantisation envelope filter of Section 2.3
prunes grains whose int16 query coordinates saturate; float32 query
coordinates never saturate, so it is the identity here.

Reduced-precision form: the scan reads BF16 or FP8 (per-grain scale) code
values and the projection may run on BF16 inputs; ``project(bf16=True)`` and
``scan_pool(form=...)`` emulate those rounding points exactly and sum in
float64.

Parity: pinned by brute force on tiny inputs (P = G and C = N give the exact
k-NN), by the r = d identity (scan score equals the exact distance), and by
the isotropic rows of the paper's recall table.  The reduced-precision
emulation is pinned by the format tests of ``quant`` and by the identity that
BF16 / FP8 scans of codes that are already exactly representable equal the
FP32 scan.
"""
from __future__ import annotations

import numpy as np

from . import quant

INF = np.inf


def _lexsmallest(dist: np.ndarray, ids: np.ndarray, m: int):
    """The m smallest (dist, id) pairs, ascending; pads with (+inf, -1)."""
    order = np.lexsort((ids, dist))[:m]
    out_d = np.full(m, INF)
    out_i = np.full(m, -1, dtype=np.int64)
    out_d[: len(order)] = dist[order]
    out_i[: len(order)] = ids[order]
    return out_i, out_d


def route(Q: np.ndarray, centroids: np.ndarray, P: int):
    """Probes (nq, P) grain ids and their squared distances, by direct differences."""
    Q = np.asarray(Q, dtype=np.float64)
    M = np.asarray(centroids, dtype=np.float64)
    G = M.shape[0]
    if not 1 <= P <= G:
        raise ValueError("need 1 <= P <= G")
    probes = np.empty((Q.shape[0], P), dtype=np.int64)
    pdist = np.empty((Q.shape[0], P))
    gid = np.arange(G)
    for i, q in enumerate(Q):
        dc = ((q[None, :] - M) ** 2).sum(axis=1)
        probes[i], pdist[i] = _lexsmallest(dc, gid, P)
    return probes, pdist


def project(Q: np.ndarray, probes: np.ndarray, stored: dict, bf16: bool = False):
    """Tangent coordinates z_q (nq, P, r) and residual energies eps_q (nq, P).

    bf16=True emulates the reduced-precision projection: q' = q - mu_g formed in
    float32, q' and W_g rounded to BF16 (nearest even), products summed in
    float64 (exact BF16 products, so only summation order differs from an FP32
    accumulator), and eps_q = max(0, ||q'||^2 - ||z_q||^2) with the unrounded q'.
    """
    Q32 = np.asarray(Q, dtype=np.float32)
    Q = Q32.astype(np.float64)
    M = stored["centroids"].astype(np.float64)
    M32 = stored["centroids"].astype(np.float32)
    B = stored["basis"]
    nq, P = probes.shape
    r = B.shape[1]
    zq = np.zeros((nq, P, r))
    epsq = np.zeros((nq, P))
    for i in range(nq):
        for s in range(P):
            g = int(probes[i, s])
            if g < 0:
                continue
            if bf16:
                qp32 = Q32[i] - M32[g]                                   # eq. (1) in float32
                Wb = quant.bf16_round(B[g]).astype(np.float64)           # (r, d)
                z = Wb @ quant.bf16_round(qp32).astype(np.float64)       # eq. (2)
                qn = float((qp32.astype(np.float64) ** 2).sum())
                zq[i, s] = z
                epsq[i, s] = max(0.0, qn - float(z @ z))                 # eq. (3)-(4), Pythagoras
                continue
            W = B[g].astype(np.float64).T          # (d, r)
            qp = Q[i] - M[g]                       # eq. (1)
            z = W.T @ qp                           # eq. (2)
            e = qp - W @ z                         # eq. (3)
            zq[i, s] = z
            epsq[i, s] = e @ e                     # eq. (4)
    return zq, epsq


def grain_scores(zq: np.ndarray, epsq: float, g: int, stored: dict, codes=None):
    """eq. (6) for every member of grain g: returns (original ids, D).  `codes`
    optionally replaces the stored codes (decoded reduced-precision values)."""
    a, b = int(stored["offsets"][g]), int(stored["offsets"][g + 1])
    Z = (stored["codes"] if codes is None else codes)[a:b].astype(np.float64)
    ei = stored["eps"][a:b].astype(np.float64)
    D = ((zq[None, :] - Z) ** 2).sum(axis=1) + epsq + ei
    return stored["perm"][a:b].astype(np.int64), D


def scan_pool(zq: np.ndarray, epsq: np.ndarray, probes: np.ndarray, stored: dict, C: int, form: str = "fp32"):
    """Candidate pool (nq, C) ids and scores over the union of the probed grains,
    scanning the code values of the given form (fp32, bf16, fp8, int16).  The
    int16 form scores on the integer codes (eq. 5) and applies the
    quantisation envelope filter (Section 2.3): a probed grain in which more
    than a quarter of the query's coordinates saturate contributes nothing."""
    if form == "int16":
        return _scan_pool_int16(zq, epsq, probes, stored, C)
    codes = None if form == "fp32" else quant.decoded_codes(stored["codes"], stored["offsets"], form)
    nq, P = probes.shape
    pool_ids = np.full((nq, C), -1, dtype=np.int64)
    pool_D = np.full((nq, C), INF)
    for i in range(nq):
        ids, Ds = [], []
        for s in range(P):
            g = int(probes[i, s])
            if g < 0:
                continue
            gi, gd = grain_scores(zq[i, s], epsq[i, s], g, stored, codes)
            ids.append(gi)
            Ds.append(gd)
        if ids:
            pool_ids[i], pool_D[i] = _lexsmallest(np.concatenate(Ds), np.concatenate(ids), C)
    return pool_ids, pool_D


def _scan_pool_int16(zq, epsq, probes, stored, C):
    r = stored["basis"].shape[1]
    zh, rh, inv, rinv = quant.int16_grain_codes(stored["codes"], stored["eps"], stored["offsets"], r)
    off = stored["offsets"]
    nq, P = probes.shape
    pool_ids = np.full((nq, C), -1, dtype=np.int64)
    pool_D = np.full((nq, C), INF)
    for i in range(nq):
        ids, Ds = [], []
        for s in range(P):
            g = int(probes[i, s])
            if g < 0:
                continue
            a, b = int(off[g]), int(off[g + 1])
            D, pruned = quant.int16_scores(zq[i, s], epsq[i, s], zh[a:b], rh[a:b], inv[g], rinv[g])
            if pruned or b == a:
                continue
            ids.append(stored["perm"][a:b].astype(np.int64))
            Ds.append(D)
        if ids:
            pool_ids[i], pool_D[i] = _lexsmallest(np.concatenate(Ds), np.concatenate(ids), C)
    return pool_ids, pool_D


def rerank(Q: np.ndarray, pool_ids: np.ndarray, X: np.ndarray, k: int):
    """Exact squared L2 over the pool by direct differences; k smallest (dist, id)."""
    Q = np.asarray(Q, dtype=np.float64)
    nq = Q.shape[0]
    ids = np.full((nq, k), -1, dtype=np.int64)
    dist = np.full((nq, k), INF)
    for i in range(nq):
        cand = pool_ids[i][pool_ids[i] >= 0]
        if len(cand) == 0:
            continue
        xv = np.asarray(X[cand], dtype=np.float64)
        dd = ((xv - Q[i][None, :]) ** 2).sum(axis=1)
        ids[i], dist[i] = _lexsmallest(dd, cand.astype(np.int64), k)
    return ids, dist


def answer_mode_a(zq: np.ndarray, epsq: np.ndarray, probes: np.ndarray, pool_ids: np.ndarray, stored: dict, k: int,
                  form: str = "fp32"):
    """Mode A (Section 2.1): the answer from the index alone.  Every pool member
    i of grain g is reconstructed in the grain's subspace, x_i' = mu_g + W_g z_i,
    and ranked by ||q - x_i'||^2.  With q - x_i' = (q' - W_g z_q) + W_g (z_q - z_i)
    and W_g orthonormal (eq. 2-4) this is ||z_q - z_i||^2 + eps_q, evaluated
    here with the pair's tangent (z_q, eps_q) and the code values of the given
    form; the k smallest (distance, id)."""
    codes = stored["codes"] if form == "fp32" else quant.decoded_codes(stored["codes"], stored["offsets"], form)
    off = np.asarray(stored["offsets"], dtype=np.int64)
    perm = np.asarray(stored["perm"], dtype=np.int64)
    pos_of = np.empty(len(perm), dtype=np.int64)
    pos_of[perm] = np.arange(len(perm))
    nq = probes.shape[0]
    ids = np.full((nq, k), -1, dtype=np.int64)
    dist = np.full((nq, k), INF)
    for i in range(nq):
        cand = pool_ids[i][pool_ids[i] >= 0].astype(np.int64)
        if len(cand) == 0:
            continue
        pos = pos_of[cand]
        g = np.searchsorted(off, pos, side="right") - 1
        slot = np.array([int(np.flatnonzero(probes[i] == gg)[0]) for gg in g])
        Z = np.asarray(codes[pos], dtype=np.float64)
        dd = ((zq[i, slot] - Z) ** 2).sum(axis=1) + epsq[i, slot]
        ids[i], dist[i] = _lexsmallest(dd, cand, k)
    return ids, dist


def search(Q, stored: dict, X, P: int, C: int, k: int, probes=None, zq=None, epsq=None,
           pool_ids=None, form: str = "fp32", bf16_project: bool = False, mode: str = "B"):
    """The whole lifecycle; any stage's input may be supplied to check later stages.
    mode "B": exact rerank against the raw vectors X; mode "A": the answer from
    the index alone (X unused)."""
    G = stored["centroids"].shape[0]
    if not (1 <= P <= G) or k < 1 or C < k:
        raise ValueError("invalid P, C or k")
    out = {}
    if probes is None:
        probes, pdist = route(Q, stored["centroids"], P)
        out["pdist"] = pdist
    out["probes"] = probes
    if zq is None or epsq is None:
        zq, epsq = project(Q, probes, stored, bf16=bf16_project)
    out["zq"], out["epsq"] = zq, epsq
    if pool_ids is None:
        pool_ids, pool_D = scan_pool(zq, epsq, probes, stored, C, form)
        out["pool_D"] = pool_D
    out["pool_ids"] = pool_ids
    if mode == "A":
        out["ids"], out["dist"] = answer_mode_a(zq, epsq, probes, pool_ids, stored, k, form)
    else:
        out["ids"], out["dist"] = rerank(Q, pool_ids, X, k)
    return out


def candidate_recall(pool_ids: np.ndarray, gt: np.ndarray, k: int = 10) -> float:
    """Recall of the approximate top-k (the first k of the pool) against the
    true top-k; the paper's 'Cand. Recall@10' column."""
    hits = [len(set(p[:k].tolist()) & set(t[:k].tolist())) for p, t in zip(pool_ids, gt)]
    return float(np.mean(hits)) / k


def recall(ids: np.ndarray, gt: np.ndarray, k: int = 10) -> float:
    hits = [len(set(a[:k].tolist()) & set(t[:k].tolist())) for a, t in zip(ids, gt)]
    return float(np.mean(hits)) / k
