"""GPU parity of the HNTL search path against the CPU oracle (through the C ABI).

Every stage is checked on its own: the oracle's output of the previous stage
is injected into the GPU stage, so a near-tie in one stage cannot cascade.
The index is the oracle's (imported into the library), so both sides search
the same stored values.
"""
import numpy as np
import pytest

from oracle import brute, index as oi, search as osr
from tests import parity
from tests.gpu_common import (announce, centroid_dist_fn, exact_dist_fn, require_gpu, scan_dist_fn, to_dev)
from workloads import patch_mixture as pm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small(small10k):
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    st = small10k["stored"]
    announce("import oracle index 10k x 768, G=64, r=32")
    ix = hntl.hntl_index_create({k: st[k] for k in ("centroids", "basis", "offsets", "perm", "codes", "eps")},
                                small10k["X"])
    Qd = to_dev(small10k["Q"])
    W = small10k["W"]
    orc = osr.search(small10k["Q"], st, small10k["X"], W.P, W.C, W.k)
    return dict(small10k, ix=ix, Qd=Qd, orc=orc, torch=torch, hntl=hntl)


def test_route_parity(small):
    announce("route parity 1000 queries P=4")
    W, hntl = small["W"], small["hntl"]
    o = hntl.hntl_search_stages(small["ix"], small["Qd"], W.P, W.C, W.k)
    orc = small["orc"]
    nd, n = parity.check_lists(o["probes"].cpu().numpy(), o["pdist"].cpu().numpy(), orc["probes"], orc["pdist"],
                               centroid_dist_fn(small["stored"]["centroids"], small["Q"]), what="probes")
    assert nd <= 0.01 * n


def test_projection_parity(small):
    announce("projection parity with oracle probes injected")
    W, hntl, torch = small["W"], small["hntl"], small["torch"]
    orc = small["orc"]
    probes = to_dev(orc["probes"].astype(np.int32))
    o = hntl.hntl_search_stages(small["ix"], small["Qd"], W.P, W.C, W.k, probes_in=probes)
    zq = o["zq"].cpu().numpy().astype(np.float64)
    eq = o["epsq"].cpu().numpy().astype(np.float64)
    qn2 = (orc["zq"] ** 2).sum(-1) + orc["epsq"]     # ||q'||^2 per pair
    tol = 4e-6 * np.sqrt(qn2)[..., None]
    assert (np.abs(zq - orc["zq"]) <= tol).all(), float(np.abs(zq - orc["zq"]).max())
    assert (np.abs(eq - orc["epsq"]) <= 1e-4 * np.maximum(orc["epsq"], 1e-3 * qn2)).all()
    assert (eq >= 0).all()


def test_scan_pool_parity(small):
    announce("scan/pool parity with oracle probes and tangents injected")
    W, hntl = small["W"], small["hntl"]
    orc = small["orc"]
    o = hntl.hntl_search_stages(small["ix"], small["Qd"], W.P, W.C, W.k,
                                probes_in=to_dev(orc["probes"].astype(np.int32)),
                                tangent_in=to_dev(orc["zq"].astype(np.float32)),
                                epsq_in=to_dev(orc["epsq"].astype(np.float32)))
    nd, n = parity.check_lists(o["pool_ids"].cpu().numpy(), o["pool_D"].cpu().numpy(), orc["pool_ids"],
                               orc["pool_D"], scan_dist_fn(small["stored"], orc["zq"], orc["epsq"], orc["probes"]),
                               what="pool")
    assert nd <= 0.01 * n


def test_rerank_parity(small):
    announce("rerank parity with the oracle pool injected")
    W, hntl = small["W"], small["hntl"]
    orc = small["orc"]
    o = hntl.hntl_search_stages(small["ix"], small["Qd"], W.P, W.C, W.k,
                                pool_in=to_dev(orc["pool_ids"].astype(np.int32)))
    nd, n = parity.check_lists(o["ids"].cpu().numpy(), o["dist"].cpu().numpy(), orc["ids"], orc["dist"],
                               exact_dist_fn(small["X"], small["Q"]), what="rerank")
    assert nd <= 0.01 * n


def test_end_to_end_and_recall(small):
    announce("end-to-end search 1000 queries")
    W, hntl = small["W"], small["hntl"]
    ids, dist = hntl.hntl_search(small["ix"], small["Qd"], W.P, W.C, W.k, flags=hntl.HNTL_FLAG_SYNC)
    ids = ids.cpu().numpy()
    dist = dist.cpu().numpy()
    orc = small["orc"]
    nd, n = parity.check_lists(ids, dist, orc["ids"], orc["dist"], exact_dist_fn(small["X"], small["Q"]),
                               what="final")
    assert nd <= 0.01 * n
    r_gpu = osr.recall(ids, small["gt_ids"])
    r_orc = osr.recall(orc["ids"], small["gt_ids"])
    assert r_gpu >= 0.99 and abs(r_gpu - r_orc) <= 0.002


def test_deterministic_bitwise(small):
    announce("determinism: two runs bitwise equal")
    W, hntl = small["W"], small["hntl"]
    a = hntl.hntl_search_stages(small["ix"], small["Qd"], W.P, W.C, W.k)
    b = hntl.hntl_search_stages(small["ix"], small["Qd"], W.P, W.C, W.k)
    for key in a:
        assert small["torch"].equal(a[key].nan_to_num(0), b[key].nan_to_num(0)), key


# ------------------------------------------------------------------ edge cases

def _edge_index(N, d, G, r, sizes=None, seed=0):
    m = pm.uniform_mixture(N, d, max(2, G // 2), seed=seed, threads=1)
    if sizes is None:
        idx = oi.build(m.X, G, r, seed=seed + 1, max_iter=20)
    else:
        lab = np.repeat(np.arange(G), sizes)
        lab = lab[np.random.default_rng(seed).permutation(N)]
        idx = oi.build(m.X, G, r, 0, labels=lab)
    return m.X, idx.stored()


EDGE = [
    # (name, N, d, G, r, sizes, nq, P, C, k)
    ("ragged-r1", 300, 64, 5, 1, [1, 63, 64, 65, 107], 17, 3, 20, 5),
    ("empty-grain-small-pool", 200, 64, 4, 8, [0, 5, 64, 131], 9, 4, 100, 10),
    ("P=G-full-rank", 250, 64, 4, 64, None, 13, 4, 256, 10),
    ("r48-d768", 700, 768, 6, 48, None, 21, 2, 64, 10),
    ("r32-C=k", 500, 768, 8, 32, None, 33, 3, 10, 10),
    ("single-query-single-grain", 129, 64, 1, 16, None, 1, 1, 128, 7),
]


@pytest.mark.parametrize("case", EDGE, ids=[c[0] for c in EDGE])
def test_edge_cases(case):
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    name, N, d, G, r, sizes, nq, P, C, k = case
    announce(f"edge case {name}: N={N} d={d} G={G} r={r} nq={nq} P={P} C={C} k={k}")
    X, st = _edge_index(N, d, G, r, sizes)
    Q = pm.uniform_queries(nq, d, max(2, G // 2), 0, 99, threads=1).X
    ix = hntl.hntl_index_create(st, X)
    orc = osr.search(Q, st, X, P, C, k)
    Qd = to_dev(Q)
    o = hntl.hntl_search_stages(ix, Qd, P, C, k, probes_in=to_dev(orc["probes"].astype(np.int32)),
                                tangent_in=to_dev(orc["zq"].astype(np.float32)),
                                epsq_in=to_dev(orc["epsq"].astype(np.float32)))
    parity.check_lists(o["pool_ids"].cpu().numpy(), o["pool_D"].cpu().numpy(), orc["pool_ids"], orc["pool_D"],
                       scan_dist_fn(st, orc["zq"], orc["epsq"], orc["probes"]), what=f"{name} pool")
    parity.check_lists(o["ids"].cpu().numpy(), o["dist"].cpu().numpy(), orc["ids"], orc["dist"],
                       exact_dist_fn(X, Q), what=f"{name} final")
    full = hntl.hntl_search_stages(ix, Qd, P, C, k)
    parity.check_lists(full["probes"].cpu().numpy(), full["pdist"].cpu().numpy(), orc["probes"], orc["pdist"],
                       centroid_dist_fn(st["centroids"], Q), what=f"{name} probes")


def test_empty_batch_and_errors():
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    X, st = _edge_index(200, 64, 4, 8, [50, 50, 50, 50])
    ix = hntl.hntl_index_create(st, X)
    Q = to_dev(np.zeros((0, 64), np.float32))
    ids, dist = hntl.hntl_search(ix, Q, 2, 20, 10)
    assert ids.shape == (0, 10)
    Qd = to_dev(pm.uniform_rows(3, 64, 1))
    for P, C, k in [(0, 20, 10), (5, 20, 10), (2, 5, 10), (2, 20, 0)]:
        with pytest.raises(hntl.HNTLError) as e:
            hntl.hntl_search(ix, Qd, P, C, k)
        assert e.value.status == hntl.HNTL_EINVAL
    bad = Qd.clone()
    bad[1, 3] = float("nan")
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_search(ix, bad, 2, 20, 10, flags=hntl.HNTL_FLAG_CHECK_Q)
    assert e.value.status == hntl.HNTL_EINVAL
    # every synchronous call checks (an infinite value this time)
    bad[1, 3] = float("inf")
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_search(ix, bad, 2, 20, 10, flags=hntl.HNTL_FLAG_SYNC)
    assert e.value.status == hntl.HNTL_EINVAL
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_search(ix, Qd, 2, 20, 10, codes="bf16")
    assert e.value.status == hntl.HNTL_ESTATE


def test_export_roundtrip(small):
    announce("index export round trip")
    hntl = small["hntl"]
    ex = hntl.hntl_index_export(small["ix"])
    for key in ("centroids", "basis", "offsets", "perm", "codes", "eps"):
        np.testing.assert_array_equal(ex[key], small["stored"][key].astype(ex[key].dtype), err_msg=key)


def test_pruned_scan_equals_full_scan(small):
    """The slot-0 bound and the grain lower-bound pruning change no pool entry
    and no result (bitwise), and scan strictly fewer members."""
    announce("pruned vs full scan, 1000 queries")
    W, hntl, torch = small["W"], small["hntl"], small["torch"]
    for P, C in ((W.P, W.C), (8, 64), (16, 100)):
        a = hntl.hntl_search_stages(small["ix"], small["Qd"], P, C, W.k,
                                    flags=hntl.HNTL_FLAG_SYNC | hntl.HNTL_FLAG_PROFILE)
        _, _, scored_a = hntl.hntl_profile_read()
        b = hntl.hntl_search_stages(small["ix"], small["Qd"], P, C, W.k,
                                    flags=hntl.HNTL_FLAG_SYNC | hntl.HNTL_FLAG_NO_PRUNE | hntl.HNTL_FLAG_PROFILE)
        _, _, scored_b = hntl.hntl_profile_read()
        for key in ("pool_ids", "pool_D", "ids", "dist"):
            assert torch.equal(a[key], b[key]), (P, C, key)
        sizes = np.diff(small["stored"]["offsets"])
        assert scored_b == int(sizes[b["probes"].cpu().numpy()].sum())
        assert scored_a < scored_b
