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


def test_traffic_entries_apply_only_to_their_sources_and_schedule():
    """A counter-derived traffic figure is reported only while the kernel's
    sources hash as when the counters were taken, and for the scan only under
    the tiles, ranges and passes they were taken with; the bytes are
    FETCH_SIZE x 2 + WRITE_SIZE x 1 KiB."""
    b = _bench()
    wide = {"qt": 8, "nw": 4, "range": 32, "grid": 0, "passes": 1, "proj": 1}
    for t in b.TRAFFIC:
        sched = dict(wide, **t["sched"]) if t["sched"] else wide
        got = b.measured_traffic(t["kernel"], t["workload"], t["form"], t["codes"], t["P"], t["mode"], t["batch"],
                                 sched)
        assert got == round((t["fetch_kib"] * 2.0 + t["write_kib"]) * 1024.0), t["kernel"]
        if t["sched"]:
            assert b.measured_traffic(t["kernel"], t["workload"], t["form"], t["codes"], t["P"], t["mode"],
                                      t["batch"], dict(sched, qt=sched["qt"] * 2)) is None
            assert b.measured_traffic(t["kernel"], t["workload"], t["form"], t["codes"], t["P"], t["mode"],
                                      t["batch"], None) is None
    assert b.measured_traffic("scan", "zipf10M_d768_G8192_r48", "plan", "fp8", 16, "B", 16384, wide) is None
    # a changed source voids the entry
    t0 = b.TRAFFIC[0]
    src = next(iter(t0["sources"]))
    saved = t0["sources"][src]
    try:
        t0["sources"][src] = "0" * 40
        assert b.measured_traffic(t0["kernel"], t0["workload"], t0["form"], t0["codes"], t0["P"], t0["mode"],
                                  t0["batch"], dict(wide, **(t0["sched"] or {}))) is None
    finally:
        t0["sources"][src] = saved
