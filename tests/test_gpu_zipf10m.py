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
  staged learned search, and tau above 1 equals centroid routing.
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
