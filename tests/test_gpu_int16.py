"""GPU parity of the paper's own int16 form (eq. 5: int16 codes, uint16
residuals, per-grain steps, exact integer squared distance, quantisation
envelope filter, exact code-box pruning) against the oracle's integer
evaluation of the same form, in the staged search and in plans.

The oracle's tangents are injected, so both sides quantise the same float32
query coordinates; the integer sums are then identical and the scores agree to
the float32 rounding of the step products (well inside 1e-4 relative).
"""
import numpy as np
import pytest

from oracle import quant, search as osr
from tests import parity
from tests.gpu_common import announce, require_gpu, to_dev

pytestmark = pytest.mark.gpu

KEYS = ("centroids", "basis", "offsets", "perm", "codes", "eps")


@pytest.fixture(scope="module")
def i16(small10k):
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    st = {k: small10k["stored"][k] for k in KEYS}
    announce("import oracle index 10k x 768 with int16 codes")
    ix = hntl.hntl_index_create(st, small10k["X"], codes=("fp32", "int16"))
    W = small10k["W"]
    orc = osr.search(small10k["Q"], st, small10k["X"], W.P, W.C, W.k)
    return dict(small10k, st=st, ix=ix, Qd=to_dev(small10k["Q"]), orc=orc, torch=torch, hntl=hntl)


def int16_score_fn(st, zq, epsq, probes):
    r = st["basis"].shape[1]
    zh, rh, inv, rinv = quant.int16_grain_codes(st["codes"], st["eps"], st["offsets"], r)
    off = st["offsets"]

    def f(i, ids):
        m = {}
        for s in range(probes.shape[1]):
            g = int(probes[i, s])
            a, b = int(off[g]), int(off[g + 1])
            D, pruned = quant.int16_scores(zq[i, s], epsq[i, s], zh[a:b], rh[a:b], inv[g], rinv[g])
            if not pruned:
                m.update(zip(st["perm"][a:b].tolist(), D.tolist()))
        return np.array([m[int(x)] for x in ids])
    return f


def test_int16_codes_bit_exact(i16):
    """Coordinate codes z_hat, residual codes r_hat and both per-grain steps
    (inv_g, rinv_g) equal the oracle's eq. 5 encoding bit for bit."""
    announce("int16 codes, residual codes and steps bit-exact")
    st = i16["st"]
    codes, inv = i16["hntl"].hntl_index_export_codes(i16["ix"], "int16")
    rcodes, rinv = i16["hntl"].hntl_index_export_codes(i16["ix"], "int16_residuals")
    zh, rh, inv_o, rinv_o = quant.int16_grain_codes(st["codes"], st["eps"], st["offsets"], st["basis"].shape[1])
    np.testing.assert_array_equal(inv, inv_o)
    np.testing.assert_array_equal(rinv, rinv_o)
    np.testing.assert_array_equal(codes.astype(np.int64), zh)
    np.testing.assert_array_equal(rcodes.astype(np.int64), rh)
    assert rh.max() == 65535  # each grain's largest residual sits at the top code


def test_int16_scan_parity(i16):
    announce("int16 scan parity with oracle probes and tangents injected")
    W, hntl, orc, st = i16["W"], i16["hntl"], i16["orc"], i16["st"]
    o = hntl.hntl_search_stages(i16["ix"], i16["Qd"], W.P, W.C, W.k, codes="int16",
                                probes_in=to_dev(orc["probes"].astype(np.int32)),
                                tangent_in=to_dev(orc["zq"].astype(np.float32)),
                                epsq_in=to_dev(orc["epsq"].astype(np.float32)))
    pool_ids, pool_D = osr.scan_pool(orc["zq"], orc["epsq"], orc["probes"], st, W.C, "int16")
    nd, n = parity.check_lists(o["pool_ids"].cpu().numpy(), o["pool_D"].cpu().numpy(), pool_ids, pool_D,
                               int16_score_fn(st, orc["zq"], orc["epsq"], orc["probes"]), what="int16 pool")
    assert nd <= 0.01 * n


def test_int16_envelope_filter_on_gpu(i16):
    """Tangents pushed far outside every probed grain (x 8 of the oracle's) make
    most coordinates saturate: every grain is pruned, nothing is returned."""
    announce("int16 envelope filter: saturated queries get empty pools")
    W, hntl, orc = i16["W"], i16["hntl"], i16["orc"]
    n = 50
    o = hntl.hntl_search_stages(i16["ix"], i16["Qd"][:n].contiguous(), W.P, W.C, W.k, codes="int16",
                                probes_in=to_dev(orc["probes"][:n].astype(np.int32)),
                                tangent_in=to_dev((1e4 * np.sign(orc["zq"][:n]) + 0 * orc["zq"][:n]).astype(np.float32)),
                                epsq_in=to_dev(orc["epsq"][:n].astype(np.float32)))
    assert (o["pool_ids"].cpu().numpy() == -1).all()
    assert (o["ids"].cpu().numpy() == -1).all()


def test_int16_end_to_end(i16):
    """Full int16 search (GPU routing, projection, integer scan with exact box
    pruning, FP32 rerank) against the oracle's int16 lifecycle on the same
    index: probes, pool and final ids under the parity rule, exact final
    distances, and recall."""
    from tests.gpu_common import centroid_dist_fn, exact_dist_fn
    announce("int16 end-to-end search vs the oracle's int16 lifecycle")
    W, hntl, st = i16["W"], i16["hntl"], i16["st"]
    X, Q = i16["X"], i16["Q"]
    orc = osr.search(Q, st, X, W.P, W.C, W.k, form="int16")
    o = hntl.hntl_search_stages(i16["ix"], i16["Qd"], W.P, W.C, W.k, codes="int16")
    parity.check_lists(o["probes"].cpu().numpy(), o["pdist"].cpu().numpy(), orc["probes"], orc["pdist"],
                       centroid_dist_fn(st["centroids"], Q), what="int16 probes")
    nd, n = parity.check_lists(o["pool_ids"].cpu().numpy(), o["pool_D"].cpu().numpy(), orc["pool_ids"],
                               orc["pool_D"], int16_score_fn(st, orc["zq"], orc["epsq"], orc["probes"]),
                               what="int16 pool")
    assert nd <= 0.01 * n
    ids = o["ids"].cpu().numpy()
    parity.check_lists(ids, o["dist"].cpu().numpy(), orc["ids"], orc["dist"], exact_dist_fn(X, Q), what="int16 ids")
    rec = osr.recall(ids, i16["gt_ids"])
    announce(f"int16 Recall@10 {rec:.4f}")
    assert rec >= 0.97
    exact = ((X[ids].astype(np.float64) - Q[:, None, :].astype(np.float64)) ** 2).sum(-1)
    np.testing.assert_allclose(o["dist"].cpu().numpy(), exact, rtol=1e-4)


def test_int16_pruned_equals_unpruned(i16):
    """The exact code-box pruning of the int16 form changes nothing: pools and
    results with and without HNTL_FLAG_NO_PRUNE are identical bit for bit."""
    W, hntl, torch = i16["W"], i16["hntl"], i16["torch"]
    announce("int16: pruned scan equals the full scan")
    for P in (W.P, 8):
        a = hntl.hntl_search_stages(i16["ix"], i16["Qd"], P, W.C, W.k, codes="int16")
        b = hntl.hntl_search_stages(i16["ix"], i16["Qd"], P, W.C, W.k, codes="int16",
                                    flags=hntl.HNTL_FLAG_SYNC | hntl.HNTL_FLAG_NO_PRUNE)
        for k in ("pool_ids", "pool_D", "ids", "dist"):
            assert torch.equal(a[k], b[k]), (P, k)


@pytest.fixture(scope="module")
def r8():
    """A small oracle index with r = 8, so that the envelope's 25% boundary is
    2 of 8 coordinates."""
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    from oracle import index as oi
    from workloads import patch_mixture as pm
    m = pm.uniform_mixture(3000, 32, 4, seed=41, threads=2)
    q = pm.uniform_queries(40, 32, 4, 41, 1041, threads=2)
    st = oi.build(m.X, 4, 8, seed=43).stored()
    st = {k: st[k] for k in KEYS}
    ix = hntl.hntl_index_create(st, m.X, codes=("fp32", "int16"))
    orc = osr.search(q.X, st, m.X, 2, 30, 10)
    return dict(st=st, X=m.X, Q=q.X, ix=ix, orc=orc, hntl=hntl, torch=torch)


def _saturate(zq, inv, ncoords):
    """Copies of the tangents with the first ncoords coordinates of slot 0
    pushed to twice the largest code value (they saturate)."""
    z = zq.copy()
    for i in range(len(z)):
        z[i, 0, :ncoords] = 2.0 * 32767.0 / float(inv[i])
    return z


def test_int16_envelope_boundary_on_gpu(r8):
    """Envelope filter at its 25% boundary (r = 8): with 2 of 8 coordinates of
    the nearest grain saturated the grain is scanned, with 3 of 8 it is pruned;
    the GPU pool equals the oracle's int16 pool on the same injected inputs in
    both cases."""
    hntl, st, orc = r8["hntl"], r8["st"], r8["orc"]
    announce("int16 envelope boundary: 2 of 8 saturated kept, 3 of 8 pruned")
    _, _, inv, _ = quant.int16_grain_codes(st["codes"], st["eps"], st["offsets"], 8)
    probes = orc["probes"]
    inv0 = inv[probes[:, 0]]
    Qd = to_dev(r8["Q"])
    for ns, kept in ((2, True), (3, False)):
        zq = _saturate(orc["zq"], inv0, ns).astype(np.float32)
        o = hntl.hntl_search_stages(r8["ix"], Qd, 2, 30, 10, codes="int16",
                                    probes_in=to_dev(probes.astype(np.int32)), tangent_in=to_dev(zq),
                                    epsq_in=to_dev(orc["epsq"].astype(np.float32)))
        pool_ids, pool_D = osr.scan_pool(zq.astype(np.float64), orc["epsq"], probes, st, 30, "int16")
        gp = o["pool_ids"].cpu().numpy()
        parity.check_lists(gp, o["pool_D"].cpu().numpy(), pool_ids, pool_D,
                           int16_score_fn(st, zq.astype(np.float64), orc["epsq"], probes), what=f"sat {ns}")
        # members of the nearest grain are in the pool only when it is kept
        off = st["offsets"]
        in0 = np.array([np.isin(gp[i], st["perm"][off[probes[i, 0]]:off[probes[i, 0] + 1]]).any()
                        for i in range(len(gp))])
        assert in0.all() if kept else not in0.any(), (ns, in0.mean())


def test_int16_bound_after_pruned_nearest_grain(r8):
    """Only the nearest grain of each query saturates (3 of 8 coordinates, so it
    is pruned) while the other probed grain is scanned: the second scan pass
    must not take a bound from the pruned list, whatever an earlier search
    left in that memory.  A search with ordinary tangents runs first to fill
    the lists; the pool then equals the oracle's int16 pool."""
    hntl, st, orc = r8["hntl"], r8["st"], r8["orc"]
    announce("int16: bound of the second pass after a pruned slot-0 list")
    _, _, inv, _ = quant.int16_grain_codes(st["codes"], st["eps"], st["offsets"], 8)
    probes = orc["probes"]
    Qd = to_dev(r8["Q"])
    pr = to_dev(probes.astype(np.int32))
    hntl.hntl_search_stages(r8["ix"], Qd, 2, 30, 10, codes="int16", probes_in=pr,
                            tangent_in=to_dev(orc["zq"].astype(np.float32)),
                            epsq_in=to_dev(orc["epsq"].astype(np.float32)))
    zq = _saturate(orc["zq"], inv[probes[:, 0]], 3).astype(np.float32)
    o = hntl.hntl_search_stages(r8["ix"], Qd, 2, 30, 10, codes="int16", probes_in=pr, tangent_in=to_dev(zq),
                                epsq_in=to_dev(orc["epsq"].astype(np.float32)))
    pool_ids, pool_D = osr.scan_pool(zq.astype(np.float64), orc["epsq"], probes, st, 30, "int16")
    assert (pool_ids[:, 0] >= 0).all()  # the second grain supplies candidates
    parity.check_lists(o["pool_ids"].cpu().numpy(), o["pool_D"].cpu().numpy(), pool_ids, pool_D,
                       int16_score_fn(st, zq.astype(np.float64), orc["epsq"], probes), what="pruned slot 0")


def test_int16_plan_equals_staged(i16):
    """The batching form runs the int16 codes too (persistent fused kernel,
    quantised tangents, envelope filter, integer distances, code-box pruning):
    a plan's results equal the staged int16 search bit for bit over schedules
    with and without block ranges, two passes and a separate projection."""
    W, hntl, torch = i16["W"], i16["hntl"], i16["torch"]
    announce("int16: plans (several schedules) vs staged search")
    ref = hntl.hntl_search(i16["ix"], i16["Qd"], W.P, W.C, W.k, codes="int16", flags=hntl.HNTL_FLAG_SYNC)
    for sched in (dict(qt=1, nw=4, range=0), dict(qt=4, nw=2, range=1, proj=1), dict(qt=2, nw=4, range=2, passes=2),
                  dict(qt=8, nw=1, range=0, proj=1)):
        plan = hntl.hntl_plan_create(i16["ix"], W.P, W.C, W.k, 1000, codes="int16", sched=sched)
        ids, dist = hntl.hntl_plan_search(plan, i16["Qd"])
        torch.cuda.synchronize()
        assert torch.equal(ids, ref[0]) and torch.equal(dist, ref[1]), sched
        assert hntl.hntl_plan_info_get(plan)["wait_errors"] == 0


def test_int16_unsupported_forms(i16):
    W, hntl = i16["W"], i16["hntl"]
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_plan_create(i16["ix"], W.P, W.C, W.k, 100, codes="int16", flags=hntl.HNTL_FLAG_MODE_A)
    assert e.value.status == hntl.HNTL_EUNSUPPORTED
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_search(i16["ix"], i16["Qd"][:4].contiguous(), W.P, W.C, W.k, codes="int16",
                         flags=hntl.HNTL_FLAG_MODE_A)
    assert e.value.status == hntl.HNTL_EUNSUPPORTED


def test_int16_extreme_range_scores():
    """The integer distance at the ends of the int16 range, at the largest rank
    (r = 64): three quarters of every member's codes and of every query's
    quantised coordinates sit at +-32767 (signs at random), the rest spread
    over the range, so the partial dot products the scan accumulates in 32
    bits reach their largest magnitudes.  Scores, pools and their order match
    the oracle's exact integer evaluation of eq. 5 on the same injected
    tangents."""
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    from oracle import index as oi
    from workloads import patch_mixture as pm
    announce("int16 at the range extremes, r = 64")
    m = pm.uniform_mixture(2400, 96, 4, seed=51, threads=2)
    q = pm.uniform_queries(48, 96, 4, 51, 1051, threads=2)
    st = oi.build(m.X, 4, 64, seed=53).stored()
    st = {k: st[k] for k in KEYS}
    rng = np.random.default_rng(57)
    A = 3.0

    def extreme(shape):
        v = A * rng.choice([-1.0, 1.0], size=shape)
        spread = rng.random(shape) < 0.25
        return np.where(spread, rng.uniform(-A, A, size=shape), v)

    st["codes"] = extreme(st["codes"].shape).astype(st["codes"].dtype)
    ix = hntl.hntl_index_create(st, m.X, codes=("fp32", "int16"))
    P, C, k = 2, 40, 10
    probes = np.stack([np.arange(48) % 4, (np.arange(48) + 1 + np.arange(48) // 4) % 4], axis=1)
    probes[probes[:, 0] == probes[:, 1], 1] = (probes[probes[:, 0] == probes[:, 1], 0] + 1) % 4
    zq = extreme((48, P, 64)).astype(np.float32)
    epsq = rng.uniform(0.0, 1.0, size=(48, P)).astype(np.float32)
    zh, _, inv, _ = quant.int16_grain_codes(st["codes"], st["eps"], st["offsets"], 64)
    assert (np.abs(zh) == 32767).mean() > 0.7  # the codes do sit at the range ends
    o = hntl.hntl_search_stages(ix, to_dev(q.X), P, C, k, codes="int16", probes_in=to_dev(probes.astype(np.int32)),
                                tangent_in=to_dev(zq), epsq_in=to_dev(epsq))
    z64 = zq.astype(np.float64)
    pool_ids, pool_D = osr.scan_pool(z64, epsq.astype(np.float64), probes, st, C, "int16")
    assert (pool_ids >= 0).all()
    parity.check_lists(o["pool_ids"].cpu().numpy(), o["pool_D"].cpu().numpy(), pool_ids, pool_D,
                       int16_score_fn(st, z64, epsq.astype(np.float64), probes), what="int16 extremes")
