"""Pins of the oracle's incremental-segment append (appending rows to a built
index, with grain splits) against closed forms and invariants."""
import numpy as np

from oracle import index as oi, segments as sg
from workloads import patch_mixture as pm


def _small(n=600, d=16, patches=6, G=6, r=4, seed=11):
    m = pm.uniform_mixture(n, d, patches, seed=seed, threads=1)
    idx = oi.build(m.X, G, r, seed=seed)
    return m.X, idx.stored()


def test_row_at_a_centroid_lands_there_with_zero_code():
    X, st = _small()
    Xn = st["centroids"].copy()              # each new row is exactly a stored centroid
    out = sg.append(st, X, Xn)
    G = len(st["offsets"]) - 1
    np.testing.assert_array_equal(out["new_grain"], np.arange(G))
    N = len(st["perm"])
    pos = {int(i): p for p, i in enumerate(out["perm"])}
    for g in range(G):
        p = pos[N + g]
        assert out["offsets"][g] <= p < out["offsets"][g + 1]
        assert np.all(out["codes"][p] == 0.0) and out["eps"][p] == 0.0


def test_assignment_codes_and_layout_by_definition():
    X, st = _small()
    rng = np.random.default_rng(5)
    Xn = (X[rng.choice(len(X), 50, replace=False)] + rng.normal(scale=0.3, size=(50, X.shape[1]))).astype(np.float32)
    out = sg.append(st, X, Xn)
    C = st["centroids"].astype(np.float64)
    G, N = C.shape[0], len(st["perm"])
    for i in range(len(Xn)):                  # nearest centroid by a plain loop, ties to the lower grain
        best, bg = None, -1
        for g in range(G):
            s = 0.0
            for j in range(Xn.shape[1]):
                t = float(Xn[i, j]) - float(C[g, j])
                s += t * t
            if best is None or s < best:
                best, bg = s, g
        assert out["new_grain"][i] == bg
    off, perm = out["offsets"], out["perm"]
    assert off[-1] == N + len(Xn)
    for g in range(G):
        a, b = int(st["offsets"][g]), int(st["offsets"][g + 1])
        a2, b2 = int(off[g]), int(off[g + 1])
        # existing members first, unchanged, then the new rows of this grain in ascending id order
        np.testing.assert_array_equal(perm[a2:a2 + (b - a)], st["perm"][a:b])
        np.testing.assert_array_equal(out["codes"][a2:a2 + (b - a)], st["codes"][a:b].astype(np.float64))
        new = perm[a2 + (b - a):b2]
        np.testing.assert_array_equal(new, N + np.nonzero(out["new_grain"] == g)[0])
        for p in range(a2 + (b - a), b2):
            x = Xn[perm[p] - N].astype(np.float64) - C[g]
            W = st["basis"][g].astype(np.float64)  # rows are the basis vectors
            z = np.array([sum(W[j, k] * x[k] for k in range(len(x))) for j in range(W.shape[0])])
            np.testing.assert_allclose(out["codes"][p], z, rtol=1e-12, atol=1e-12)
            # Pythagoras up to the FP32 basis' departure from orthonormality
            np.testing.assert_allclose(x @ x, z @ z + out["eps"][p], rtol=1e-6)
            e = x - W.T @ z
            np.testing.assert_allclose(out["eps"][p], e @ e, rtol=1e-9, atol=1e-12)


def test_no_split_at_or_below_the_threshold():
    X, st = _small()
    Xn = X[:40] + 0.01
    plain = sg.append(st, X, Xn)
    cap = int(np.diff(plain["offsets"]).max())
    out = sg.append(st, X, Xn, split_max=cap)
    assert len(out["children"]) == 0
    for k in ("offsets", "perm", "centroids", "basis", "codes", "eps"):
        np.testing.assert_array_equal(out[k], plain[k])


def test_split_separates_two_clusters_along_the_leading_axis():
    rng = np.random.default_rng(2)
    d, n = 5, 40
    A = rng.normal(scale=0.2, size=(n, d))
    A[:, 0] -= 10.0
    Bc = rng.normal(scale=0.2, size=(n, d))
    Bc[:, 0] += 10.0
    X = np.empty((2 * n, d))
    X[0::2], X[1::2] = A, Bc                  # interleaved ids
    X = X.astype(np.float32)
    st = oi.build(X, 1, 2, seed=0, labels=np.zeros(2 * n, np.int64)).stored()
    out = sg.append(st, X, np.zeros((0, d), np.float32), split_max=n)
    np.testing.assert_array_equal(out["offsets"], [0, n, 2 * n])
    kids = [set(out["perm"][:n].tolist()), set(out["perm"][n:].tolist())]
    assert {frozenset(k) for k in kids} == {frozenset(range(0, 2 * n, 2)), frozenset(range(1, 2 * n, 2))}
    for g in range(2):
        ids = out["perm"][out["offsets"][g]:out["offsets"][g + 1]]
        np.testing.assert_allclose(out["centroids"][g], X[ids].astype(np.float64).mean(0), rtol=1e-6, atol=1e-6)
        Wg = out["basis"][g].astype(np.float64)
        np.testing.assert_allclose(Wg @ Wg.T, np.eye(2), atol=1e-6)
    assert (out["eps"] >= 0).all()
    np.testing.assert_array_equal(out["children"], [0, 1])


def test_split_sizes_membership_and_cut_order():
    X, st = _small(n=900, G=5)
    rng = np.random.default_rng(8)
    Xn = (X[rng.choice(len(X), 120, replace=False)] + rng.normal(scale=0.2, size=(120, X.shape[1]))).astype(np.float32)
    plain = sg.append(st, X, Xn)
    sizes = np.diff(plain["offsets"])
    cap = int(sizes.max() // 3 + 7)
    out = sg.append(st, X, Xn, split_max=cap)
    N2 = len(X) + len(Xn)
    G = len(sizes)
    assert sorted(out["perm"].tolist()) == list(range(N2))
    s2 = np.diff(out["offsets"])
    assert s2.max() <= cap
    expect = [(g, -(-int(sizes[g]) // cap)) for g in range(G) if sizes[g] > cap]
    assert len(s2) == G + sum(m - 1 for _, m in expect)
    nxt = G
    for g, m in expect:
        kids = [g] + list(range(nxt, nxt + m - 1))
        nxt += m - 1
        assert sorted(s2[kids].tolist()) == sorted(sg.split_runs(int(sizes[g]), m))
        # the parent's first code coordinate orders the children
        a, b = int(plain["offsets"][g]), int(plain["offsets"][g + 1])
        t = dict(zip(plain["perm"][a:b].tolist(), plain["codes"][a:b, 0].astype(np.float32).tolist()))
        lo = [min(t[int(i)] for i in out["perm"][out["offsets"][k]:out["offsets"][k + 1]]) for k in kids]
        hi = [max(t[int(i)] for i in out["perm"][out["offsets"][k]:out["offsets"][k + 1]]) for k in kids]
        for k in range(m - 1):
            assert hi[k] <= lo[k + 1]
        for k in kids:
            ids = out["perm"][out["offsets"][k]:out["offsets"][k + 1]]
            assert np.all(np.diff(ids) > 0)
    assert sorted(out["children"].tolist()) == sorted(
        [g for g, _ in expect] + list(range(G, len(s2))))
    # unsplit grains keep their stored centroid and basis
    for g in range(G):
        if sizes[g] <= cap:
            np.testing.assert_array_equal(out["centroids"][g], st["centroids"][g])
            np.testing.assert_array_equal(out["basis"][g], st["basis"][g])


def test_two_appends_equal_one_append_of_both():
    X, st = _small()
    rng = np.random.default_rng(4)
    A = (X[:30] + rng.normal(scale=0.1, size=(30, X.shape[1]))).astype(np.float32)
    B = (X[30:70] + rng.normal(scale=0.1, size=(40, X.shape[1]))).astype(np.float32)
    one = sg.append(st, X, np.vstack([A, B]))
    mid = sg.append(st, X, A)
    two = sg.append(mid, np.vstack([X, A]), B)
    np.testing.assert_array_equal(two["offsets"], one["offsets"])
    np.testing.assert_array_equal(two["perm"], one["perm"])
    np.testing.assert_allclose(two["codes"], one["codes"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(two["eps"], one["eps"], rtol=1e-12, atol=1e-12)
