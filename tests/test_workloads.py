"""The SIFT1M-shaped stand-in workload: shape and byte-valued components, and
the oracle on it (P = G and C = N reduce to exact k-NN on byte-valued data)."""
import numpy as np

from oracle import brute, index as oi, search as osr
from workloads import SIFTLIKE_1M, SIFTLIKE_20K
from workloads import patch_mixture as pm


def test_siftlike_rows_are_byte_valued():
    m = pm.byte_valued(pm.uniform_mixture(2000, 128, 16, seed=3, threads=1))
    X = m.X
    assert X.shape == (2000, 128) and X.dtype == np.float32
    assert X.min() >= 0 and X.max() <= 255 and np.array_equal(X, np.rint(X))
    assert 0.1 < (X == 0).mean() < 0.4  # a share of components clip at zero
    assert SIFTLIKE_1M.d == 128 and SIFTLIKE_1M.N == 1_000_000 and SIFTLIKE_1M.nq == 10_000
    assert SIFTLIKE_20K.byte_valued and SIFTLIKE_1M.byte_valued


def test_siftlike_full_probe_full_pool_is_exact():
    m = pm.byte_valued(pm.uniform_mixture(400, 128, 8, seed=4, threads=1))
    q = pm.byte_valued(pm.uniform_queries(12, 128, 8, 4, 5, threads=1))
    idx = oi.build(m.X, 6, 16, seed=9)
    out = osr.search(q.X, idx.stored(), m.X, P=6, C=400, k=10)
    ids, dist = brute.knn(m.X, q.X, 10)
    np.testing.assert_array_equal(out["ids"], ids)
    np.testing.assert_allclose(out["dist"], dist, rtol=1e-12)
