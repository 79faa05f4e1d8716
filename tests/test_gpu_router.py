"""GPU tests of the learned router: forward, gradients and one Adam step
against the oracle (which emulates the BF16 rounding points), the
brute-force kNN that labels the training queries, learned routing in the
search (staged and plan), the centroid fallback, and what training gains.

The weights under test come from the oracle's initialisation; the oracle never
reads a GPU output.  Tolerances: 1e-3 relative Frobenius error per gradient
tensor (BF16 operands, FP32 against FP64 accumulation).
"""
import numpy as np
import pytest

from oracle import brute, router as orr
from tests import parity
from tests.gpu_common import announce, exact_dist_fn, require_gpu, to_dev

pytestmark = pytest.mark.gpu

DIMS_H = (1024, 1024)


def rel_fro(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def rt(small10k):
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    st = small10k["stored"]
    announce("import oracle index 10k x 768 for the router tests")
    ix = hntl.hntl_index_create({k: st[k] for k in ("centroids", "basis", "offsets", "perm", "codes", "eps")},
                                small10k["X"])
    W = small10k["W"]
    dims = (768,) + DIMS_H + (W.G,)
    params = orr.init_params(dims, seed=5)
    Qtr = W.queries(nq=4096, query_seed=3005).X
    mean = Qtr.astype(np.float64).mean(0)
    std = Qtr.astype(np.float64).std(0)
    # grain of every original row from the oracle index
    lab = np.empty(len(small10k["X"]), np.int64)
    off = st["offsets"]
    for g in range(W.G):
        lab[st["perm"][off[g]:off[g + 1]]] = g
    return dict(small10k, ix=ix, torch=torch, hntl=hntl, params=params, mean=mean, std=std, Qtr=Qtr, lab=lab)


def set_weights(rt):
    p = rt["params"]
    rt["hntl"].hntl_router_set(rt["ix"], {k: p[k].astype(np.float32) for k in p}, rt["mean"].astype(np.float32),
                               rt["std"].astype(np.float32))


def oracle_params32(rt):
    """The oracle's weights as the GPU holds them (FP32 masters, FP32 mean/std)."""
    p = {k: v.astype(np.float32).astype(np.float64) for k, v in rt["params"].items()}
    return p, rt["mean"].astype(np.float32).astype(np.float64), rt["std"].astype(np.float32).astype(np.float64)


def test_router_forward_parity(rt):
    announce("router forward 256 queries, 768-1024-1024-64, vs oracle (BF16 emulation)")
    set_weights(rt)
    Q = rt["Q"][:256]
    s_gpu = rt["hntl"].hntl_router_forward(rt["ix"], to_dev(Q)).cpu().numpy()
    p, m, sd = oracle_params32(rt)
    s_orc, _ = orr.forward(p, Q, m, sd, bf16=True)
    assert rel_fro(s_gpu, s_orc) < 1e-3, rel_fro(s_gpu, s_orc)


def test_knn_parity(rt):
    announce("brute-force kNN k=10 for 300 queries vs oracle")
    hntl = rt["hntl"]
    Q = rt["Q"][:300]
    ids, dist = hntl.hntl_knn(rt["ix"], to_dev(Q), 10)
    gt_ids, gt_dist = rt["gt_ids"][:300], rt["gt_dist"][:300]
    nd, n = parity.check_lists(ids.cpu().numpy(), dist.cpu().numpy(), gt_ids, gt_dist,
                               exact_dist_fn(rt["X"], Q), what="knn ids")
    assert nd <= 0.01 * n


def knn_targets(rt, Q, k=10):
    ids, _ = brute.knn(rt["X"], Q, k)
    return rt["lab"][ids].astype(np.int32)


def test_router_gradient_parity(rt):
    announce("router gradients of a 256-query batch vs oracle backward (BF16 emulation)")
    hntl = rt["hntl"]
    set_weights(rt)
    X = rt["Qtr"][:256]
    tg = knn_targets(rt, X)
    loss_gpu, g_gpu = hntl.hntl_router_grad(rt["ix"], to_dev(X), to_dev(tg))
    p, m, sd = oracle_params32(rt)
    s, cache = orr.forward(p, X, m, sd, bf16=True)
    y = orr.grain_targets(tg, np.arange(rt["W"].G), rt["W"].G)
    loss_orc, ds = orr.loss_and_dlogits(s, y)
    g_orc = orr.backward(p, cache, ds, bf16=True)
    assert abs(loss_gpu - loss_orc) <= 1e-4 * abs(loss_orc), (loss_gpu, loss_orc)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert rel_fro(g_gpu[k], g_orc[k]) < 1e-3, (k, rel_fro(g_gpu[k], g_orc[k]))


def test_router_adam_step_parity(rt):
    """One training step (one batch, no shuffling) from the oracle's weights:
    the GPU's weight change equals the oracle's Adam step on its own gradients,
    except where a gradient is so small that its sign is rounding noise (the
    first Adam step moves every weight by about lr * sign(g))."""
    announce("one Adam step on one batch vs oracle")
    hntl = rt["hntl"]
    set_weights(rt)
    X = rt["Qtr"][:256]
    tg = knn_targets(rt, X)
    lr = 1e-3
    hntl.hntl_router_train(rt["ix"], to_dev(X), targets=to_dev(tg), hidden=DIMS_H, epochs=1, batch=256, knn=10,
                           lr=lr, flags=hntl.HNTL_ROUTER_KEEP_WEIGHTS | hntl.HNTL_ROUTER_NO_SHUFFLE)
    after = hntl.hntl_router_export(rt["ix"])
    p, m, sd = oracle_params32(rt)
    s, cache = orr.forward(p, X, m, sd, bf16=True)
    y = orr.grain_targets(tg, np.arange(rt["W"].G), rt["W"].G)
    _, ds = orr.loss_and_dlogits(s, y)
    g = orr.backward(p, cache, ds, bf16=True)
    new = orr.adam_step(dict(p), g, {}, 1, lr=lr)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        d_gpu = after[k].astype(np.float64) - p[k]
        d_orc = new[k] - p[k]
        bad = np.abs(d_gpu - d_orc) > 1e-2 * lr
        small = np.abs(g[k]) < 1e-2 * np.abs(g[k]).max()
        assert not (bad & ~small).any(), (k, int((bad & ~small).sum()))
        assert bad.mean() < 0.02, (k, float(bad.mean()))


def test_router_adam_two_steps_parity(rt):
    """Two Adam steps (two batches of 128 rows in input order: t = 1, then
    t = 2, where the moments mix both gradients and the bias corrections no
    longer cancel) move the weights as the oracle's `adam_step` does when fed
    the GPU's own gradients at the GPU's own weights: `hntl_router_grad` (whose
    parity with the oracle's backward is tested above) at the starting weights
    on the first batch, and at the weights after a one-step run on the second.
    This isolates the optimiser's arithmetic from the BF16 gradient noise that
    a second step amplifies where two gradients nearly cancel."""
    announce("two Adam steps on two batches vs the oracle's Adam on the GPU's gradients")
    hntl = rt["hntl"]
    X = rt["Qtr"][:256]
    tg = knn_targets(rt, X)
    lr = 1e-3
    flags = hntl.HNTL_ROUTER_KEEP_WEIGHTS | hntl.HNTL_ROUTER_NO_SHUFFLE
    keys = ("W1", "b1", "W2", "b2", "W3", "b3")
    set_weights(rt)
    _, g1 = hntl.hntl_router_grad(rt["ix"], to_dev(X[:128]), to_dev(tg[:128]))
    hntl.hntl_router_train(rt["ix"], to_dev(X[:128]), targets=to_dev(tg[:128]), hidden=DIMS_H, epochs=1, batch=128,
                           knn=10, lr=lr, flags=flags)
    p1 = hntl.hntl_router_export(rt["ix"])
    hntl.hntl_router_set(rt["ix"], {k: p1[k] for k in keys}, p1["mean"], p1["std"])
    _, g2 = hntl.hntl_router_grad(rt["ix"], to_dev(X[128:]), to_dev(tg[128:]))
    set_weights(rt)
    hntl.hntl_router_train(rt["ix"], to_dev(X), targets=to_dev(tg), hidden=DIMS_H, epochs=1, batch=128, knn=10,
                           lr=lr, flags=flags)
    after = hntl.hntl_router_export(rt["ix"])
    p, _, _ = oracle_params32(rt)
    state = {}
    cur = orr.adam_step(dict(p), {k: g1[k].astype(np.float64) for k in keys}, state, 1, lr=lr)
    d1 = {k: cur[k] - p[k] for k in keys}
    cur = orr.adam_step(dict(cur), {k: g2[k].astype(np.float64) for k in keys}, state, 2, lr=lr)
    for k in keys:
        # the first step alone, then both: FP32 masters and moments against
        # FP64, far inside 1e-3 lr
        np.testing.assert_allclose(p1[k].astype(np.float64) - p[k], d1[k], rtol=0, atol=1e-3 * lr, err_msg=k)
        np.testing.assert_allclose(after[k].astype(np.float64) - p[k], cur[k] - p[k], rtol=0, atol=1e-3 * lr,
                                   err_msg=k)
        assert np.abs(cur[k] - p[k]).max() > 0.5 * lr  # the steps moved the weights


def probe_recall(probes, gt_ids, lab):
    """Fraction of the true top-10 neighbours whose grain is probed."""
    hit = 0
    for i in range(len(probes)):
        ps = set(probes[i].tolist())
        hit += sum(int(lab[j]) in ps for j in gt_ids[i])
    return hit / gt_ids.size


@pytest.fixture(scope="module")
def trained(rt):
    """The router trained on 4,096 generated queries with brute-force kNN targets
    (computed on the GPU), 6 epochs."""
    hntl = rt["hntl"]
    announce("train router 768-1024-1024-64 on 4096 queries, 6 epochs, GPU kNN targets")
    losses = hntl.hntl_router_train(rt["ix"], to_dev(rt["Qtr"]), hidden=DIMS_H, epochs=6, batch=256, knn=10,
                                    lr=1e-3, seed=7)
    return losses


def test_training_reduces_loss(rt, trained):
    announce(f"training losses {np.round(trained, 4).tolist()}")
    assert trained[-1] < 0.8 * trained[0]


def test_learned_probe_recall_at_equal_p(rt, trained):
    """Probe recall (true neighbours inside the probed grains) on held-out
    queries, learned against centroid routing at equal P: the trained router
    loses at most 0.01 (on this mixture the nearest centroids are already
    near-perfect probes; the router's gain is the probe budget below)."""
    hntl, W = rt["hntl"], rt["W"]
    Qh = W.queries(nq=1000, query_seed=3006).X
    gt, _ = brute.knn(rt["X"], Qh, 10)
    Qd = to_dev(Qh)
    rec = {}
    for route in ("centroid", "learned"):
        for P in (1, 2, 4):
            o = hntl.hntl_search_stages(rt["ix"], Qd, P, W.C, W.k, route=route)
            rec[(route, P)] = probe_recall(o["probes"].cpu().numpy(), gt, rt["lab"])
    announce("probe recall " + ", ".join(f"{r} P={p}: {v:.4f}" for (r, p), v in sorted(rec.items())))
    for P in (1, 2, 4):
        assert rec[("learned", P)] >= rec[("centroid", P)] - 0.01, (P, rec)


def test_mass_budget_parity(rt, trained):
    """The probability-mass probe budget on the GPU against the oracle's
    mass_cut, on the oracle's weights with the output layer scaled by 12 (so
    the softmax is peaked and cuts happen): the kept probes are a prefix of the
    uncut learned probes, and the number kept equals the oracle's except where
    the oracle's cumulative probability at the cut lies within 1e-3 of the
    mass (the GPU's scores differ from the BF16 emulation by about 1e-4)."""
    hntl, W = rt["hntl"], rt["W"]
    announce("mass budget: GPU cut vs oracle mass_cut")
    saved = hntl.hntl_router_export(rt["ix"])  # the trained router, put back afterwards
    params = {k: v.copy() for k, v in rt["params"].items()}
    params["W3"] *= 12.0
    hntl.hntl_router_set(rt["ix"], {k: v.astype(np.float32) for k, v in params.items()},
                         rt["mean"].astype(np.float32), rt["std"].astype(np.float32))
    try:
        p = {k: v.astype(np.float32).astype(np.float64) for k, v in params.items()}
        m, sd = rt["mean"].astype(np.float32).astype(np.float64), rt["std"].astype(np.float32).astype(np.float64)
        Q = rt["Q"][:512]
        Qd = to_dev(Q)
        P = 6
        full = hntl.hntl_search_stages(rt["ix"], Qd, P, W.C, W.k, route="learned")["probes"].cpu().numpy()
        s_orc, _ = orr.forward(p, Q, m, sd, bf16=True)
        cuts = 0
        for mass in (0.5, 0.9, 0.99):
            cut = hntl.hntl_search_stages(rt["ix"], Qd, P, W.C, W.k, route="learned",
                                          mass=mass)["probes"].cpu().numpy()
            kept = (cut >= 0).sum(1)
            assert (kept >= 1).all()
            for i in range(len(Q)):
                assert (cut[i, :kept[i]] == full[i, :kept[i]]).all() and (cut[i, kept[i]:] == -1).all()
            ref = orr.mass_cut(s_orc, full, mass)
            kref = (ref >= 0).sum(1)
            for i in np.nonzero(kept != kref)[0]:
                e = np.exp(s_orc[i] - s_orc[i].max())
                c = np.cumsum(e[full[i]] / e.sum())
                j = min(kept[i], kref[i]) - 1
                assert abs(c[j] - mass) < 1e-3, (mass, i, kept[i], kref[i], c)
            cuts += int((kept < P).sum())
            announce(f"mass {mass}: mean probes {kept.mean():.3f}, rows differing from the oracle "
                     f"{int((kept != kref).sum())}")
        assert cuts > 0
    finally:
        hntl.hntl_router_set(rt["ix"], {k: saved[k] for k in ("W1", "b1", "W2", "b2", "W3", "b3")},
                             saved["mean"], saved["std"])


def test_learned_probe_budget_gain():
    """What the trained router gains over centroid routing: its softmax
    probabilities are a calibrated confidence, so a probability-mass budget
    spends probes only on uncertain queries.  Index: the 10k patch mixture
    split into 256 grains (4 per patch, so neighbours straddle grains), router
    trained on 20,000 generated queries with brute-force kNN targets.  On
    1,000 held-out queries (C = 20, k = 10), the budget reaches the Recall@10
    of centroid routing at some fixed P with fewer probed (query, grain)
    pairs: the measured gain is asserted > 0 and stated."""
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    from workloads import SMALL_10K as W
    announce("router gain: 10k corpus in 256 grains, router trained on 20,000 queries")
    X = W.corpus().X
    ix = hntl.hntl_build(to_dev(X), 256, 32, seed=W.kmeans_seed)
    Qtr = W.queries(nq=20000, query_seed=3005).X
    hntl.hntl_router_train(ix, to_dev(Qtr), hidden=DIMS_H, epochs=8, batch=512, knn=10, lr=1e-3, seed=7)
    Qh = W.queries(nq=1000, query_seed=3006).X
    gt, _ = brute.knn(X, Qh, 10)
    Qd = to_dev(Qh)
    C, k = 20, 10

    def recall(o):
        ids = o["ids"].cpu().numpy()
        return float(np.mean([len(set(a.tolist()) & set(b.tolist())) / k for a, b in zip(ids, gt)]))

    cen = {}
    for P in (1, 2, 3, 4, 6, 8):
        o = hntl.hntl_search_stages(ix, Qd, P, C, k)
        cen[P] = (recall(o), P * len(Qh))
    lrn = {}
    for mass in (0.9, 0.99, 0.999):
        o = hntl.hntl_search_stages(ix, Qd, 8, C, k, route="learned", mass=mass)
        lrn[mass] = (recall(o), int((o["probes"] >= 0).sum()))
    announce("centroid (Recall@10, pairs): " + ", ".join(f"P={P}: {v[0]:.4f} {v[1]}" for P, v in cen.items()))
    announce("learned budget (Recall@10, pairs): " + ", ".join(f"mass={m}: {v[0]:.4f} {v[1]}" for m, v in lrn.items()))
    gains = []
    for mass, (rl, pl) in lrn.items():
        matched = [pairs for rc, pairs in cen.values() if rc >= rl]
        if matched:
            gains.append((min(matched) / pl, mass, rl))
    assert gains, "no centroid P reaches the learned budget's recall"
    best = max(gains)
    announce(f"gain: {best[0]:.2f}x fewer probed pairs at Recall@10 {best[2]:.4f} (mass {best[1]})")
    assert best[0] > 1.0, gains


def test_learned_plan_equals_staged(rt, trained):
    hntl, W, torch = rt["hntl"], rt["W"], rt["torch"]
    announce("learned routing: plan (graph) vs staged search")
    Qd = to_dev(rt["Q"])
    a = hntl.hntl_search(rt["ix"], Qd, W.P, W.C, W.k, route="learned", flags=hntl.HNTL_FLAG_SYNC)
    plan = hntl.hntl_plan_create(rt["ix"], W.P, W.C, W.k, 1000, route="learned", sched=dict(qt=2, nw=4, range=1))
    b = hntl.hntl_plan_search(plan, Qd)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    for nb in (1, 37):
        c = hntl.hntl_plan_search(plan, Qd[:nb].contiguous())
        torch.cuda.synchronize()
        assert torch.equal(c[0], a[0][:nb]) and torch.equal(c[1], a[1][:nb])


def test_fallback_to_centroids(rt, trained):
    """tau above any probability sends every query to centroid routing (results
    equal the centroid search bit for bit); tau = 0 never falls back."""
    hntl, W, torch = rt["hntl"], rt["W"], rt["torch"]
    announce("fallback: tau 1.01 equals centroid routing; plan likewise")
    Qd = to_dev(rt["Q"])
    cen = hntl.hntl_search_stages(rt["ix"], Qd, W.P, W.C, W.k)
    fb = hntl.hntl_search_stages(rt["ix"], Qd, W.P, W.C, W.k, route="learned", tau=1.01)
    assert torch.equal(cen["probes"], fb["probes"])
    assert torch.equal(cen["ids"], fb["ids"]) and torch.equal(cen["dist"], fb["dist"])
    plan = hntl.hntl_plan_create(rt["ix"], W.P, W.C, W.k, 1000, route="learned", tau=1.01)
    ids, dist = hntl.hntl_plan_search(plan, Qd)
    torch.cuda.synchronize()
    assert torch.equal(ids, cen["ids"]) and torch.equal(dist, cen["dist"])
    # part fallback: probes are either the learned ones or the centroid ones, row by row
    le = hntl.hntl_search_stages(rt["ix"], Qd, W.P, W.C, W.k, route="learned")
    s = hntl.hntl_router_forward(rt["ix"], Qd).cpu().numpy().astype(np.float64)
    pmax = 1.0 / np.exp(s - s.max(1, keepdims=True)).sum(1)
    tau = float(np.median(pmax))
    mix = hntl.hntl_search_stages(rt["ix"], Qd, W.P, W.C, W.k, route="learned", tau=tau)
    lo = pmax < tau * (1 - 1e-4)
    hi = pmax > tau * (1 + 1e-4)
    mp = mix["probes"].cpu().numpy()
    assert (mp[lo] == cen["probes"].cpu().numpy()[lo]).all()
    assert (mp[hi] == le["probes"].cpu().numpy()[hi]).all()


def test_learned_route_requires_router(small10k):
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    st = small10k["stored"]
    ix = hntl.hntl_index_create({k: st[k] for k in ("centroids", "basis", "offsets", "perm", "codes", "eps")},
                                small10k["X"][:])
    W = small10k["W"]
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_search(ix, to_dev(small10k["Q"][:4]), W.P, W.C, W.k, route="learned")
    assert e.value.status == hntl.HNTL_ESTATE
