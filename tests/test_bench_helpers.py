"""The bench's FP64 measurement helpers (recall ground truth, eq. 6 reference
scores for the reduced-precision report) agree with the oracle."""
import importlib.util
from pathlib import Path

import numpy as np

from oracle import brute, index as oi, search as osr

ROOT = Path(__file__).resolve().parents[1]


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", ROOT / "bench.py")
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_exact_knn_and_recall_match_the_oracle():
    b = _bench()
    rng = np.random.default_rng(0)
    X = rng.standard_normal((5000, 32)).astype(np.float32)
    X[100] = X[7]  # an exact tie: the lower id first
    Q = np.concatenate([rng.standard_normal((19, 32)), X[7:8] + 1e-3]).astype(np.float32)
    got = b.exact_knn(X, Q, 10, chunk=700)
    ref, _ = brute.knn(X, Q, 10)
    np.testing.assert_array_equal(got, ref)
    assert b.recall_at_k(got, ref, 10) == osr.recall(got, ref) == 1.0
    assert abs(b.recall_at_k(got[:, ::-1], ref[:, 5:].repeat(2, 1), 10) - 0.5) < 1e-12


def test_fp64_grain_scores_match_the_oracle():
    b = _bench()
    rng = np.random.default_rng(1)
    X = rng.standard_normal((3000, 24)).astype(np.float32)
    st = oi.build(X, 6, 5, seed=2).stored()
    Q = rng.standard_normal((4, 24)).astype(np.float32)
    probes = np.array([[g, (g + 1) % 6] for g in range(4)])
    zq, eq = osr.project(Q, probes, st)
    for i in range(4):
        for s in range(2):
            gi, gd = osr.grain_scores(zq[i, s], eq[i, s], int(probes[i, s]), st)
            hi, hd = b.fp64_grain_scores(Q[i], int(probes[i, s]), st)
            np.testing.assert_array_equal(hi, gi)
            np.testing.assert_allclose(hd, gd, rtol=1e-12, atol=1e-12)
