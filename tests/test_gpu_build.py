"""GPU index build (k-means grains, FP64 local PCA, codes) against the oracle's
build and against the invariants of eq. 1-4."""
import numpy as np
import pytest

from oracle import index as oi, kmeans as km, search as osr
from tests.gpu_common import announce, require_gpu, to_dev

pytestmark = pytest.mark.gpu


def _adjusted_rand(a, b):
    from scipy.special import comb
    ca = np.unique(a, return_inverse=True)[1]
    cb = np.unique(b, return_inverse=True)[1]
    M = np.zeros((ca.max() + 1, cb.max() + 1), dtype=np.int64)
    np.add.at(M, (ca, cb), 1)
    s = comb(M, 2).sum()
    sa = comb(M.sum(1), 2).sum()
    sb = comb(M.sum(0), 2).sum()
    e = sa * sb / comb(len(a), 2)
    return (s - e) / (0.5 * (sa + sb) - e)


def _check_invariants(X, st, cap_gpu):
    B = st["basis"].astype(np.float64)
    for g in range(B.shape[0]):
        assert np.abs(B[g] @ B[g].T - np.eye(B.shape[1])).max() < 2e-6
    codes64, eps64 = oi.stored_encode(X, st)
    np.testing.assert_allclose(st["codes"], codes64, atol=2e-5 * np.sqrt(np.abs(codes64).max() + 1))
    assert (st["eps"] >= 0).all()
    np.testing.assert_allclose(st["eps"], eps64, rtol=1e-4, atol=1e-4)
    assert ((cap_gpu > 0) & (cap_gpu <= 1 + 1e-9)).all()


def test_build_from_oracle_centroids(small10k):
    """Seeded with the oracle's converged centroids, the GPU build reproduces the
    oracle's partition; its bases capture the same variance per grain."""
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    W = small10k["W"]
    st = small10k["stored"]
    announce("GPU build 10k x 768 from oracle centroids")
    ix = hntl.hntl_build(to_dev(small10k["X"]), W.G, W.r, init_centroids=to_dev(st["centroids"]), seed=5)
    ex = hntl.hntl_index_export(ix)
    cap = hntl.hntl_index_captured(ix)
    np.testing.assert_array_equal(ex["offsets"], st["offsets"])
    np.testing.assert_array_equal(ex["perm"], st["perm"])
    np.testing.assert_allclose(ex["centroids"], st["centroids"], rtol=0, atol=2e-6)
    np.testing.assert_allclose(cap, st["captured"], rtol=0, atol=1e-6)
    _check_invariants(small10k["X"], ex, cap)
    # same subspace: residual energies agree with the oracle's
    np.testing.assert_allclose(ex["eps"], st["eps"], rtol=2e-3, atol=2e-4)


def test_build_kmeanspp_quality_and_search(small10k):
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    W = small10k["W"]
    announce("GPU build 10k x 768 with device k-means++")
    ix = hntl.hntl_build(to_dev(small10k["X"]), W.G, W.r, seed=W.kmeans_seed)
    ex = hntl.hntl_index_export(ix)
    cap = hntl.hntl_index_captured(ix)
    _check_invariants(small10k["X"], ex, cap)
    lab = np.empty(len(ex["perm"]), np.int64)
    for g in range(W.G):
        lab[ex["perm"][ex["offsets"][g]:ex["offsets"][g + 1]]] = g
    st = small10k["stored"]
    lab_o = np.empty_like(lab)
    for g in range(W.G):
        lab_o[st["perm"][st["offsets"][g]:st["offsets"][g + 1]]] = g
    in_gpu = km.inertia(small10k["X"], ex["centroids"], lab)
    in_orc = km.inertia(small10k["X"], st["centroids"], lab_o)
    assert in_gpu <= in_orc * 1.005
    assert _adjusted_rand(lab, small10k["labels"]) > 0.99
    ids, _ = hntl.hntl_search(ix, to_dev(small10k["Q"]), W.P, W.C, W.k, flags=hntl.HNTL_FLAG_SYNC)
    assert osr.recall(ids.cpu().numpy(), small10k["gt_ids"]) >= 0.99


def test_build_edge_small_grains():
    """Grains smaller than the rank (rank-deficient covariances) still give
    orthonormal bases and eps >= 0."""
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    from workloads import patch_mixture as pm
    X = pm.uniform_mixture(90, 64, 3, seed=3, threads=1).X
    announce("GPU build tiny rank-deficient grains N=90 d=64 G=12 r=16")
    ix = hntl.hntl_build(to_dev(X), 12, 16, seed=1)
    ex = hntl.hntl_index_export(ix)
    _check_invariants(X, ex, hntl.hntl_index_captured(ix))
