"""Full-size checks at the batching workload's shape, in the configuration
bench.py times with --workload zipf10M_d768_G8192_r48 --form plan: 10,000,000
vectors, d = 768, 8,192 Zipf-sized grains, r = 48, batches up to 16,384
queries, P = 16, C = 100, k = 10.

No oracle index exists at this size, so the checks are properties that hold
at any size plus sampled outputs the oracle computes one by one:
* a plan (autotuned schedule, graph replay) returns exactly what the staged
  search returns, at batch sizes 16,384, 1,000 and 1, for FP32 and for BF16
  codes with BF16 projection;
* every returned distance equals the exact squared distance recomputed in
  FP64 from the corpus (1e-4 relative);
* Recall@10 against the oracle's brute force on a query sample is >= 0.95;
* learned routing (router trained briefly here) through a plan equals the
  staged learned search, and tau above 1 equals centroid routing;
* oracle parity on a 48-query sample of the exported index: routing probes,
  the pool and final ids from the oracle's probes, and the plan's final ids;
* the router at full width (8,192 outputs) against the oracle: forward scores,
  every gradient tensor, and the search path's learned probes.
"""
import numpy as np
import pytest

from oracle import brute
from tests.gpu_common import announce, require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def z():
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    from workloads import ZIPF_10M as W
    from workloads.configs import ROUTER_TRAIN_SEED
    announce("generate 10M x 768 Zipf corpus and 16,384 queries")
    m = W.corpus()
    q = W.queries()
    X = torch.from_numpy(m.X).cuda()
    announce("build G=8192 r=48 index (FP32 + BF16 codes)")
    ix = hntl.hntl_build(X, W.G, W.r, seed=W.kmeans_seed, codes=("fp32", "bf16"))
    del X
    torch.cuda.empty_cache()
    Qtr = W.queries(nq=20000, query_seed=ROUTER_TRAIN_SEED).X
    return dict(W=W, X=m.X, Q=q.X, Qd=to_dev(q.X), Qtr=Qtr, ix=ix, hntl=hntl, torch=torch)


def check_exact(z, ids, dist, rows):
    X, Q = z["X"], z["Q"]
    ids = ids[rows]
    ok = ids >= 0
    assert ok.all()
    exact = ((X[ids].astype(np.float64) - Q[rows][:, None, :].astype(np.float64)) ** 2).sum(-1)
    np.testing.assert_allclose(dist[rows], exact, rtol=1e-4)


@pytest.mark.parametrize("codes", ["fp32", "bf16"])
def test_plan_equals_staged_full_size(z, codes):
    W, hntl, torch = z["W"], z["hntl"], z["torch"]
    fl = hntl.HNTL_FLAG_PROJECT_BF16 if codes == "bf16" else 0
    announce(f"10M: autotune + graph plan vs staged search, codes={codes}, batches 16384/1000/1")
    sched, _ = hntl.hntl_tune(z["ix"], z["Qd"], W.P, W.C, W.k, codes=codes, flags=fl)
    plan = hntl.hntl_plan_create(z["ix"], W.P, W.C, W.k, W.nq, codes=codes, flags=fl, sched=sched)
    for nb in (W.nq, 1000, 1):
        Q = z["Qd"][:nb].contiguous()
        a = hntl.hntl_search(z["ix"], Q, W.P, W.C, W.k, codes=codes, flags=fl | hntl.HNTL_FLAG_SYNC)
        b = hntl.hntl_plan_search(plan, Q)
        torch.cuda.synchronize()
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), nb
    assert hntl.hntl_plan_info_get(plan)["wait_errors"] == 0
    ids, dist = (t.cpu().numpy() for t in hntl.hntl_plan_search(plan, z["Qd"]))
    rs = np.random.default_rng(5).choice(W.nq, 64, replace=False)
    check_exact(z, ids, dist, rs)
    gt, _ = brute.knn(z["X"], z["Q"][rs[:32]], W.k)
    rec = np.mean([len(set(ids[r]) & set(g)) / W.k for r, g in zip(rs[:32], gt)])
    announce(f"10M {codes}: Recall@10 on 32 sampled queries {rec:.4f}")
    assert rec >= 0.95


def test_learned_routing_full_size(z):
    W, hntl, torch = z["W"], z["hntl"], z["torch"]
    announce("10M: train router on 20,000 queries (GPU kNN targets), 1 epoch; learned plan vs staged")
    losses = hntl.hntl_router_train(z["ix"], to_dev(z["Qtr"]), hidden=(1024, 1024), epochs=1, batch=1024, seed=3)
    assert np.isfinite(losses).all()
    fl = hntl.HNTL_FLAG_PROJECT_BF16
    Q = z["Qd"][:4096].contiguous()
    a = hntl.hntl_search(z["ix"], Q, 4, W.C, W.k, codes="bf16", flags=fl | hntl.HNTL_FLAG_SYNC, route="learned")
    plan = hntl.hntl_plan_create(z["ix"], 4, W.C, W.k, 4096, codes="bf16", flags=fl, route="learned")
    b = hntl.hntl_plan_search(plan, Q)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    check_exact(z, b[0].cpu().numpy(), b[1].cpu().numpy(), np.arange(0, 4096, 64))
    c = hntl.hntl_search(z["ix"], Q, 4, W.C, W.k, codes="bf16", flags=fl | hntl.HNTL_FLAG_SYNC)
    f = hntl.hntl_search(z["ix"], Q, 4, W.C, W.k, codes="bf16", flags=fl | hntl.HNTL_FLAG_SYNC, route="learned",
                         tau=1.01)
    assert torch.equal(c[0], f[0]) and torch.equal(c[1], f[1])


def test_append_full_size(z):
    """100,000 rows of the same mixture appended to the 10M index with grains
    capped at 16,384 members (the largest Zipf grains hold up to 20,000):
    the result is a permutation of all ids with every grain at or below the
    cap; grains that were not split keep their members, codes, centroid and
    basis bit for bit with the new rows after them; sampled new rows sit in
    their nearest base centroid's grain (or in a child of a split grain) with
    codes and eps equal to the FP64 encoding by the stored centroid and basis;
    children have orthonormal bases and member-mean centroids; an appended
    row searched through the result is its own nearest neighbour."""
    from oracle import index as oi
    W, hntl, torch = z["W"], z["hntl"], z["torch"]
    cap, n = 16384, 100_000
    Xn = W.queries(nq=n, query_seed=4242).X
    announce(f"10M: append {n} rows with split_max {cap}")
    base = hntl.hntl_index_export(z["ix"])
    ix2 = hntl.hntl_index_append(z["ix"], to_dev(Xn), split_max=cap, seed=1)
    ex = hntl.hntl_index_export(ix2)
    N, G = W.N, W.G
    assert ix2.N == N + n and ix2.G > G
    assert np.all(np.bincount(ex["perm"], minlength=N + n) == 1)
    off0, off2 = base["offsets"], ex["offsets"]
    assert np.diff(off2).max() <= cap
    grain = np.empty(N + n, np.int64)
    for g in range(ix2.G):
        grain[ex["perm"][off2[g]:off2[g + 1]]] = g
    unsplit = np.zeros(ix2.G, bool)
    for g in range(G):
        a0, b0, a2, b2 = off0[g], off0[g + 1], off2[g], off2[g + 1]
        if b2 - a2 >= b0 - a0 and np.array_equal(ex["perm"][a2:a2 + (b0 - a0)], base["perm"][a0:b0]):
            unsplit[g] = True
            np.testing.assert_array_equal(ex["codes"][a2:a2 + (b0 - a0)], base["codes"][a0:b0])
            np.testing.assert_array_equal(ex["eps"][a2:a2 + (b0 - a0)], base["eps"][a0:b0])
            np.testing.assert_array_equal(ex["centroids"][g], base["centroids"][g])
            np.testing.assert_array_equal(ex["basis"][g], base["basis"][g])
            tail = ex["perm"][a2 + (b0 - a0):b2]
            assert np.all(tail >= N) and np.all(np.diff(tail) > 0)
    n_split = int(G - unsplit[:G].sum())
    announce(f"10M append: {n_split} grains split into {ix2.G - G + n_split} children")
    assert n_split >= 1
    # sampled new rows: nearest base centroid, codes by the stored centroid and basis
    rs = np.random.default_rng(9).choice(n, 2000, replace=False)
    C0 = base["centroids"].astype(np.float64)
    xs = Xn[rs].astype(np.float64)
    D = (xs ** 2).sum(1)[:, None] + (C0 ** 2).sum(1)[None, :] - 2.0 * xs @ C0.T
    near = np.argmin(D, axis=1)
    gs = grain[N + rs]
    ok_unsplit = unsplit[gs]
    D_sorted = np.sort(D, axis=1)
    clear = (D_sorted[:, 1] - D_sorted[:, 0]) > 1e-4 * np.abs(D_sorted[:, 0])
    np.testing.assert_array_equal(gs[ok_unsplit & clear], near[ok_unsplit & clear])
    assert not np.any(unsplit[near[~ok_unsplit & clear]])  # rows in children came from a split grain
    pos = np.empty(N + n, np.int64)
    pos[ex["perm"]] = np.arange(N + n)
    for g in np.unique(gs):
        rows = rs[gs == g]
        zc, ec = oi.encode(Xn[rows], ex["centroids"][g], ex["basis"][g].astype(np.float64).T)
        p = pos[N + rows]
        np.testing.assert_allclose(ex["codes"][p], zc, rtol=0, atol=2e-5 * np.sqrt(np.abs(zc).max() + 1))
        np.testing.assert_allclose(ex["eps"][p], ec, rtol=1e-4, atol=1e-4)
    for g in np.nonzero(~unsplit)[0][:8]:
        Bg = ex["basis"][g].astype(np.float64)
        assert np.abs(Bg @ Bg.T - np.eye(W.r)).max() < 2e-6
        ids = ex["perm"][off2[g]:off2[g + 1]]
        Xm = np.concatenate([z["X"][ids[ids < N]], Xn[ids[ids >= N] - N]]).astype(np.float64)
        np.testing.assert_allclose(ex["centroids"][g], Xm.mean(0), rtol=0, atol=2e-6 * max(1.0, np.abs(Xm).max()))
    del base, ex
    q = to_dev(Xn[rs[:1000]])
    ids, dist = hntl.hntl_search(ix2, q, W.P, W.C, W.k, flags=hntl.HNTL_FLAG_SYNC)
    np.testing.assert_array_equal(ids.cpu().numpy()[:, 0], N + rs[:1000])
    assert float(dist[:, 0].abs().max()) < 1e-3


def test_full_size_oracle_parity(z):
    """Oracle parity at the full Zipf size on a 48-query sample: the index's
    stored arrays are exported and the oracle searches them (FP64, eq. 1-6) at
    the P = 16, C = 100, k = 10 the plan runs at.  The GPU's own routing probes,
    its pool and final ids from the oracle's probes (stage input injected), and
    the plan's final ids must all meet the parity rule (ids exact except
    near-ties within 1e-5 relative; distances within 1e-4 relative)."""
    from oracle import search as osr
    from tests import parity
    from tests.gpu_common import centroid_dist_fn, exact_dist_fn, scan_dist_fn
    W, hntl, torch = z["W"], z["hntl"], z["torch"]
    rs = np.random.default_rng(21).choice(W.nq, 48, replace=False)
    Qs = z["Q"][rs]
    announce("10M: oracle search of 48 sampled queries on the exported index, P=16 C=100 k=10")
    ex = hntl.hntl_index_export(z["ix"])
    orc = osr.search(Qs, ex, z["X"], W.P, W.C, W.k)
    Qd = to_dev(Qs)
    announce("10M: GPU routing, pool (oracle probes injected) and plan ids vs the oracle")
    own = hntl.hntl_search_stages(z["ix"], Qd, W.P, W.C, W.k, flags=hntl.HNTL_FLAG_SYNC | hntl.HNTL_FLAG_ROUTE_BF16)
    parity.check_lists(own["probes"].cpu().numpy(), own["pdist"].cpu().numpy(), orc["probes"], orc["pdist"],
                       centroid_dist_fn(ex["centroids"], Qs), what="10M probes")
    inj = hntl.hntl_search_stages(z["ix"], Qd, W.P, W.C, W.k, probes_in=to_dev(orc["probes"].astype(np.int32)))
    parity.check_lists(inj["pool_ids"].cpu().numpy(), inj["pool_D"].cpu().numpy(), orc["pool_ids"], orc["pool_D"],
                       scan_dist_fn(ex, orc["zq"], orc["epsq"], orc["probes"]), what="10M pool")
    parity.check_lists(inj["ids"].cpu().numpy(), inj["dist"].cpu().numpy(), orc["ids"], orc["dist"],
                       exact_dist_fn(z["X"], Qs), what="10M ids (oracle probes)")
    plan = hntl.hntl_plan_create(z["ix"], W.P, W.C, W.k, 48, flags=hntl.HNTL_FLAG_ROUTE_BF16)
    ids, dist = hntl.hntl_plan_search(plan, Qd)
    torch.cuda.synchronize()
    parity.check_lists(ids.cpu().numpy(), dist.cpu().numpy(), orc["ids"], orc["dist"], exact_dist_fn(z["X"], Qs),
                       what="10M plan ids")


def _check_top_scores(gpu_probes, s, P, what, rel=2e-3):
    """gpu_probes (rows x P) against full oracle scores s (rows x G): the P
    largest scores, ties to the lower grain, up to near-ties within
    rel * max |s| of the row.  The window covers the GPU's score error against
    the oracle's BF16 emulation: FP32 and FP64 accumulation can round a hidden
    activation to neighbouring BF16 values (2^-8 relative), which moves scores
    by about 1e-4 of their scale (the forward test bounds the whole error at
    1e-3 relative)."""
    for i in range(len(s)):
        order = np.lexsort((np.arange(s.shape[1]), -s[i]))[:P]
        thr = s[i, order[-1]]
        tol = rel * float(np.abs(s[i]).max())
        g = gpu_probes[i]
        assert len(set(g.tolist())) == P, (what, i)
        assert (s[i, g] >= thr - tol).all(), (what, i, g, order)
        missing = set(order.tolist()) - set(g.tolist())
        assert all(s[i, m] <= thr + tol for m in missing), (what, i)
        assert (np.diff(s[i, g]) <= tol).all(), (what, i)  # descending within the tie window


def test_router_parity_full_width(z):
    """The router at its full width, 768-1024-1024-8192 (the logits layer spans
    32 column tiles of 256): forward scores of 1,024 queries and every
    gradient tensor of a 256-query batch against the oracle's BF16 emulation
    (1e-3 relative Frobenius), and the search path's learned probes (1,024
    rows through the staged search, and the plan's results) against the
    oracle's route_learned on the same weights."""
    from oracle import router as orr
    W, hntl, torch = z["W"], z["hntl"], z["torch"]
    announce("10M: router 768-1024-1024-8192 with oracle weights: forward, gradients, search probes")
    dims = (W.d, 1024, 1024, W.G)
    params = orr.init_params(dims, seed=8)
    mean = z["Qtr"].astype(np.float64).mean(0)
    std = z["Qtr"].astype(np.float64).std(0)
    hntl.hntl_router_set(z["ix"], {k: v.astype(np.float32) for k, v in params.items()}, mean.astype(np.float32),
                         std.astype(np.float32))
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in params.items()}
    m, sd = mean.astype(np.float32).astype(np.float64), std.astype(np.float32).astype(np.float64)
    Q = z["Q"][:1024]  # 1,024 rows: the large-tile GEMM (from 512 rows on)
    s_gpu = hntl.hntl_router_forward(z["ix"], to_dev(Q)).cpu().numpy().astype(np.float64)
    s_orc, cache = orr.forward(p, Q, m, sd, bf16=True)
    err = np.linalg.norm(s_gpu - s_orc) / np.linalg.norm(s_orc)
    announce(f"forward rel Frobenius error {err:.2e}")
    assert err < 1e-3
    # gradients against seeded targets (10 grain ids per row)
    tg = np.random.default_rng(3).integers(0, W.G, size=(256, 10)).astype(np.int32)
    loss_gpu, g_gpu = hntl.hntl_router_grad(z["ix"], to_dev(z["Qtr"][:256]), to_dev(tg))
    s2, c2 = orr.forward(p, z["Qtr"][:256], m, sd, bf16=True)
    y = orr.grain_targets(tg, np.arange(W.G), W.G)
    loss_orc, ds = orr.loss_and_dlogits(s2, y)
    g_orc = orr.backward(p, c2, ds, bf16=True)
    assert abs(loss_gpu - loss_orc) <= 1e-4 * abs(loss_orc), (loss_gpu, loss_orc)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        e = np.linalg.norm(np.asarray(g_gpu[k], np.float64) - g_orc[k]) / np.linalg.norm(g_orc[k])
        assert e < 1e-3, (k, e)
    # the search path's probes (learned routing, 1,024 rows) against route_learned
    Qd = to_dev(Q)
    o = hntl.hntl_search_stages(z["ix"], Qd, W.P, W.C, W.k, route="learned")
    gp = o["probes"].cpu().numpy()
    # exactly the P largest of the GPU's own forward scores (ties: lower grain)
    own = np.lexsort((np.broadcast_to(np.arange(W.G), s_gpu.shape), -s_gpu), axis=1)[:, :W.P]
    np.testing.assert_array_equal(gp, own)
    lp, _ = orr.route_learned(p, Q, m, sd, W.P)
    _check_top_scores(gp, s_orc, W.P, "learned probes")
    announce(f"learned probes equal to route_learned in {(gp == lp).all(1).mean():.4f} of rows")
    # and the plan's results equal the staged learned search on those rows
    plan = hntl.hntl_plan_create(z["ix"], W.P, W.C, W.k, 1024, route="learned")
    ids, dist = hntl.hntl_plan_search(plan, Qd)
    torch.cuda.synchronize()
    assert torch.equal(ids, o["ids"]) and torch.equal(dist, o["dist"])


def test_bf16_routing_forms_full_size(z):
    """At G = 8,192 and 2,048 rows (the large-tile GEMM with its direct LDS
    loads), the plain and split BF16 shortlists give the same probes and
    distances as FP32 MFMA routing: the P = 16 winners are FP32 direct
    differences in every form."""
    W, hntl, torch = z["W"], z["hntl"], z["torch"]
    announce("10M: BF16 / split-BF16 / FP32 routing forms agree at 2,048 rows")
    Q = z["Qd"][:2048].contiguous()
    ref = hntl.hntl_search_stages(z["ix"], Q, W.P, W.C, W.k)
    for fl in (hntl.HNTL_FLAG_ROUTE_BF16, hntl.HNTL_FLAG_ROUTE_BF16X3):
        o = hntl.hntl_search_stages(z["ix"], Q, W.P, W.C, W.k, flags=hntl.HNTL_FLAG_SYNC | fl)
        assert torch.equal(o["probes"], ref["probes"]), fl
        assert torch.equal(o["pdist"], ref["pdist"]), fl
        assert torch.equal(o["ids"], ref["ids"]) and torch.equal(o["dist"], ref["dist"]), fl
