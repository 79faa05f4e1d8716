"""GPU parity on the SIFT1M-shaped stand-in (d = 128, r = 16, byte-valued
components): the staged search and a plan against the oracle on the oracle's
index, at a rank (16) and dimension the other workloads do not use."""
import numpy as np
import pytest

from oracle import search as osr
from tests import parity
from tests.conftest import cached_oracle_index
from tests.gpu_common import announce, exact_dist_fn, require_gpu, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sl():
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    from oracle import brute, index as oi
    from workloads import SIFTLIKE_20K as W
    m, q = W.corpus(), W.queries()

    def mk():
        return oi.build(m.X, W.G, W.r, W.kmeans_seed).stored()
    st = cached_oracle_index("siftlike20k", mk)
    st = {k: st[k] for k in ("centroids", "basis", "offsets", "perm", "codes", "eps")}
    announce("import oracle index 20k x 128 (byte-valued), G=64, r=16")
    ix = hntl.hntl_index_create(st, m.X)
    orc = osr.search(q.X, st, m.X, W.P, W.C, W.k)
    gt, _ = brute.knn(m.X, q.X, W.k)
    return dict(W=W, X=m.X, Q=q.X, Qd=to_dev(q.X), st=st, ix=ix, orc=orc, gt=gt, hntl=hntl, torch=torch)


def test_siftlike_staged_parity_and_recall(sl):
    W, hntl, orc = sl["W"], sl["hntl"], sl["orc"]
    announce("siftlike 20k: staged search vs oracle")
    ids, dist = hntl.hntl_search(sl["ix"], sl["Qd"], W.P, W.C, W.k, flags=hntl.HNTL_FLAG_SYNC)
    nd, n = parity.check_lists(ids.cpu().numpy(), dist.cpu().numpy(), orc["ids"], orc["dist"],
                               exact_dist_fn(sl["X"], sl["Q"]), what="siftlike ids")
    assert nd <= 0.01 * n
    assert osr.recall(ids.cpu().numpy(), sl["gt"]) >= 0.95


def test_siftlike_plan_equals_staged(sl):
    W, hntl, torch = sl["W"], sl["hntl"], sl["torch"]
    announce("siftlike 20k: plans vs staged")
    a = hntl.hntl_search(sl["ix"], sl["Qd"], W.P, W.C, W.k, flags=hntl.HNTL_FLAG_SYNC)
    for sched in (dict(qt=4, nw=2, range=0), dict(qt=1, nw=4, range=2, proj=1)):
        plan = hntl.hntl_plan_create(sl["ix"], W.P, W.C, W.k, W.nq, sched=sched)
        b = hntl.hntl_plan_search(plan, sl["Qd"])
        torch.cuda.synchronize()
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), sched
