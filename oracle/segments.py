"""Incremental segments (oracle, FP64): appending vectors to a built index.

Test infrastructure: only the tests, the smoke check and the bench's CPU
baseline use this package.

Section 1 and the SSTable layer of Section 2 (Fig. 1): grains are
self-contained, so adding vectors leaves every other grain and every existing
code untouched; a segment is immutable, so an append yields a new index and
leaves its input as it was.  The paper gives no update rule; the readings
used here:

* a new row x (id N + i) joins the grain of the nearest centroid, squared L2,
  ties to the lower grain (the build's assignment rule), and is encoded with
  that grain's stored mu_g and W_g by eq. (1)-(4);  centroids, bases and the
  codes of existing members stay as stored;
* a grain holding more than ``split_max`` members after the append
  (``split_max`` > 0) is cut into m = ceil(n / split_max) children along its
  leading local principal axis: members ordered by their first code
  coordinate t = z_1 as stored in float32 (ties by id), cut into m runs whose
  sizes differ by at most one (the first n mod m runs one longer).  Child 0
  keeps the grain's number; children 1 .. m - 1 get the numbers G, G + 1, ...
  in ascending order of the grains split.  Each child gets the exact FP64
  mean of its members as centroid, its own local PCA basis (Section 2.2) and
  codes by eq. (1)-(4).

Pins (tests): a row equal to a centroid lands in that grain with z = 0 and
eps = 0; Pythagoras for every new code; existing codes are unchanged; no
split below the threshold; a grain made of two separated clusters along its
leading axis splits exactly into them; every grain ends at or below the
threshold with sibling sizes within one; two appends with no split equal one
append of both batches.
"""
from __future__ import annotations

import numpy as np

from . import kmeans as km
from .index import encode
from .pca import local_pca


def assign_new(X_new: np.ndarray, centroids: np.ndarray):
    """Nearest stored centroid of every new row (ties to the lower grain), its
    distance, and the gap to the second nearest (for checking that a decision
    is not a near tie)."""
    C = np.asarray(centroids, dtype=np.float64)
    D = km.sq_dists(np.asarray(X_new, dtype=np.float64), C)
    lab = np.argmin(D, axis=1)
    best = D[np.arange(len(lab)), lab]
    if C.shape[0] > 1:
        D2 = D.copy()
        D2[np.arange(len(lab)), lab] = np.inf
        gap = D2.min(axis=1) - best
    else:
        gap = np.full(len(lab), np.inf)
    return lab.astype(np.int64), best, gap


def split_runs(n: int, m: int):
    """Sizes of the m runs a grain of n members is cut into."""
    return [n // m + (1 if k < n % m else 0) for k in range(m)]


def append(stored: dict, X_old: np.ndarray | None, X_new: np.ndarray, split_max: int = 0) -> dict:
    """The appended index in stored form (codes and eps in float64), plus the
    new rows' grains, their assignment gaps, the cut gaps of the splits and
    the list of child grains (grain numbers whose basis was recomputed)."""
    C = stored["centroids"].astype(np.float64)
    basis = stored["basis"].astype(np.float64)
    off = np.asarray(stored["offsets"], dtype=np.int64)
    perm = np.asarray(stored["perm"], dtype=np.int64)
    codes_old = np.asarray(stored["codes"])
    eps_old = np.asarray(stored["eps"])
    G, r, d = basis.shape
    N = len(perm)
    X_new = np.asarray(X_new, dtype=np.float64).reshape(-1, d)
    n = X_new.shape[0]
    if split_max and X_old is None:
        raise ValueError("splitting grains needs the raw vectors of the existing rows")

    lab, _, gap = assign_new(X_new, C) if n else (np.zeros(0, np.int64), None, np.zeros(0))
    z_new = np.zeros((n, r))
    e_new = np.zeros(n)
    for g in np.unique(lab):
        rows = np.nonzero(lab == g)[0]
        z, e = encode(X_new[rows], C[g], basis[g].T)          # eq. (1)-(4) with the stored mu_g, W_g
        z_new[rows] = z
        e_new[rows] = e

    # members of every grain: existing ids (ascending) then new ids (ascending)
    members, mcodes, meps = [], [], []
    for g in range(G):
        a, b = int(off[g]), int(off[g + 1])
        nr = np.nonzero(lab == g)[0]
        members.append(np.concatenate([perm[a:b], N + nr]))
        mcodes.append(np.concatenate([codes_old[a:b].astype(np.float64), z_new[nr]]))
        meps.append(np.concatenate([eps_old[a:b].astype(np.float64), e_new[nr]]))

    cents = [C[g] for g in range(G)]
    bases = [basis[g] for g in range(G)]
    children, cut_gaps = [], []
    if split_max:
        X_all = np.vstack([np.asarray(X_old, dtype=np.float64), X_new])
        extra = []
        for g in range(G):
            ids = members[g]
            if len(ids) <= split_max:
                continue
            m = -(-len(ids) // split_max)
            t = mcodes[g][:, 0].astype(np.float32)                # the stored FP32 first coordinate
            order = np.lexsort((ids, t))
            sizes = split_runs(len(ids), m)
            pos = np.concatenate([[0], np.cumsum(sizes)])
            ts = t[order].astype(np.float64)
            cut_gaps.extend((ts[pos[1:-1]] - ts[pos[1:-1] - 1]).tolist())
            for k in range(m):
                cid = np.sort(ids[order[pos[k]:pos[k + 1]]])
                mu = X_all[cid].mean(axis=0)
                W, _, _ = local_pca(X_all[cid], mu, r)
                z, e = encode(X_all[cid], mu, W)
                if k == 0:
                    members[g], mcodes[g], meps[g] = cid, z, e
                    cents[g], bases[g] = mu, W.T
                    children.append(g)
                else:
                    extra.append((cid, z, e, mu, W.T))
        for cid, z, e, mu, Wt in extra:
            children.append(len(members))
            members.append(cid)
            mcodes.append(z)
            meps.append(e)
            cents.append(mu)
            bases.append(Wt)

    G2 = len(members)
    offsets = np.concatenate([[0], np.cumsum([len(x) for x in members])]).astype(np.int64)
    return {
        "centroids": np.asarray(cents).astype(np.float32),
        "basis": np.asarray(bases).astype(np.float32).reshape(G2, r, d),
        "offsets": offsets,
        "perm": np.concatenate(members).astype(np.int32) if G2 else np.zeros(0, np.int32),
        "codes": np.concatenate(mcodes).reshape(-1, r),
        "eps": np.concatenate(meps),
        "new_grain": lab,
        "assign_gap": gap,
        "cut_gaps": np.asarray(cut_gaps, dtype=np.float64),
        "children": np.asarray(children, dtype=np.int64),
    }
