"""GPU tests of the batching form: search plans around the persistent fused
project-scan-select kernel, HIP-graph replay, and the schedule autotuner.

A plan's pool is the exact top C of (eq. 6 score, id) over the probed grains,
computed with the same arithmetic as the staged search, so its results must
equal hntl_search's bit for bit, for every schedule (tile shape, waves per
workgroup, block ranges), batch size, code form and projection precision.
The final results are also checked against the oracle on the oracle's own
index.
"""
import numpy as np
import pytest

from oracle import search as osr
from tests import parity
from tests.gpu_common import announce, exact_dist_fn, require_gpu, to_dev

pytestmark = pytest.mark.gpu

SCHEDULES = [
    dict(qt=1, nw=1, range=0),
    dict(qt=1, nw=4, range=1),   # every grain split into one-block ranges
    dict(qt=2, nw=2, range=2),
    dict(qt=2, nw=1, range=3),
    dict(qt=4, nw=4, range=0),
    dict(qt=4, nw=8, range=1),
    dict(qt=8, nw=2, range=0),
    dict(qt=8, nw=1, range=2),
    dict(qt=4, nw=4, range=0, passes=2),
    dict(qt=2, nw=2, range=1, passes=2),
    dict(qt=4, nw=4, range=0, proj=1),           # separate projection launch
    dict(qt=2, nw=2, range=1, passes=2, proj=1),
    dict(qt=1, nw=8, range=3, proj=1),
]


@pytest.fixture(scope="module")
def bt(small10k):
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    st = {k: small10k["stored"][k] for k in ("centroids", "basis", "offsets", "perm", "codes", "eps")}
    announce("import oracle index 10k x 768 (FP32, BF16, FP8 codes) for plans")
    ix = hntl.hntl_index_create(st, small10k["X"], codes=("fp32", "bf16", "fp8"))
    W = small10k["W"]
    orc = osr.search(small10k["Q"], st, small10k["X"], W.P, W.C, W.k)
    return dict(small10k, st=st, ix=ix, Qd=to_dev(small10k["Q"]), orc=orc, torch=torch, hntl=hntl)


def staged(bt, Q, codes="fp32", flags=0):
    W, hntl = bt["W"], bt["hntl"]
    ids, dist = hntl.hntl_search(bt["ix"], Q, W.P, W.C, W.k, codes=codes, flags=flags | hntl.HNTL_FLAG_SYNC)
    return ids, dist


def assert_same(a, b, what):
    torch = __import__("torch")
    assert torch.equal(a[0], b[0]), f"{what}: ids differ"
    assert torch.equal(a[1], b[1]), f"{what}: distances differ"


@pytest.mark.parametrize("sched", SCHEDULES,
                         ids=lambda s: f"qt{s['qt']}-nw{s['nw']}-range{s['range']}-passes{s.get('passes', 1)}"
                                       f"-proj{s.get('proj', 0)}")
def test_plan_equals_staged_search(bt, sched):
    W, hntl = bt["W"], bt["hntl"]
    announce(f"plan (eager) {sched} vs staged search, batches 1..1000")
    plan = hntl.hntl_plan_create(bt["ix"], W.P, W.C, W.k, 1000, sched=sched, graph=False,
                                 flags=hntl.HNTL_FLAG_SYNC)
    for nb in (1000, 1, 7, 256):
        Q = bt["Qd"][:nb].contiguous()
        assert_same(hntl.hntl_plan_search(plan, Q), staged(bt, Q), f"{sched} nq={nb}")
    assert hntl.hntl_plan_info_get(plan)["wait_errors"] == 0


@pytest.mark.parametrize("codes,bf16proj", [("bf16", True), ("fp8", True), ("bf16", False), ("fp8", False)])
def test_plan_reduced_precision_equals_staged(bt, codes, bf16proj):
    W, hntl = bt["W"], bt["hntl"]
    fl = hntl.HNTL_FLAG_PROJECT_BF16 if bf16proj else 0
    announce(f"plan codes={codes} bf16 projection={bf16proj} vs staged search")
    for sched in (dict(qt=2, nw=4, range=1), dict(qt=4, nw=2, range=0), dict(qt=4, nw=2, range=0, proj=1)):
        plan = hntl.hntl_plan_create(bt["ix"], W.P, W.C, W.k, 1000, codes=codes, flags=fl | hntl.HNTL_FLAG_SYNC,
                                     sched=sched)
        assert_same(hntl.hntl_plan_search(plan, bt["Qd"]), staged(bt, bt["Qd"], codes, fl), f"{codes} {sched}")


def test_plan_no_prune_equals_pruned(bt):
    W, hntl = bt["W"], bt["hntl"]
    announce("plan with and without exact pruning")
    sched = dict(qt=2, nw=2, range=1)
    a = hntl.hntl_plan_create(bt["ix"], W.P, W.C, W.k, 1000, sched=sched, flags=hntl.HNTL_FLAG_SYNC)
    b = hntl.hntl_plan_create(bt["ix"], W.P, W.C, W.k, 1000, sched=sched,
                              flags=hntl.HNTL_FLAG_SYNC | hntl.HNTL_FLAG_NO_PRUNE)
    assert_same(hntl.hntl_plan_search(a, bt["Qd"]), hntl.hntl_plan_search(b, bt["Qd"]), "prune vs no prune")


def test_graph_replays_match_eager(bt):
    """Replays of one captured graph with different batch sizes, with unrelated
    eager GPU work and synchronisations between them; every replay must equal
    the eager result of the same batch."""
    W, hntl, torch = bt["W"], bt["hntl"], bt["torch"]
    announce("graph replay: 6 replays of one plan, nq 1000/1/333/7/1000/64")
    plan = hntl.hntl_plan_create(bt["ix"], W.P, W.C, W.k, 1000, sched=dict(qt=2, nw=4, range=2), graph=True)
    assert hntl.hntl_plan_info_get(plan)["graph"]
    x = torch.randn(512, 512, device="cuda")
    for nb in (1000, 1, 333, 7, 1000, 64):
        Q = bt["Qd"][:nb].contiguous()
        got = hntl.hntl_plan_search(plan, Q)
        torch.cuda.synchronize()
        y = (x @ x).sum()  # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(y)
        assert_same(got, staged(bt, Q), f"replay nq={nb}")
    assert hntl.hntl_plan_info_get(plan)["wait_errors"] == 0


def test_plan_buffers_run(bt):
    """Queries written straight into the plan's buffer; results read from its buffers."""
    W, hntl, torch = bt["W"], bt["hntl"], bt["torch"]
    announce("plan_run on the plan's own buffers")
    plan = hntl.hntl_plan_create(bt["ix"], W.P, W.C, W.k, 1000, sched=dict(qt=1, nw=2, range=0))
    qa, ia, da = hntl.hntl_plan_buffers(plan)
    assert qa and ia and da
    ref = staged(bt, bt["Qd"][:100].contiguous())
    ids, dist = hntl.hntl_plan_search(plan, bt["Qd"][:100].contiguous())
    torch.cuda.synchronize()
    assert_same((ids, dist), ref, "plan_search")
    hntl.hntl_plan_run(plan, 100)  # same queries are still in the plan's buffer
    torch.cuda.synchronize()
    ids2, dist2 = hntl.hntl_plan_search(plan, bt["Qd"][:100].contiguous())
    assert_same((ids2, dist2), ref, "plan_run then plan_search")


def test_plan_oracle_parity(bt):
    """Final results of a graph-replayed plan against the oracle (ids up to
    near-ties within 1e-5 relative, distances within 1e-4 relative)."""
    W, hntl = bt["W"], bt["hntl"]
    announce("plan final ids/distances vs oracle")
    plan = hntl.hntl_plan_create(bt["ix"], W.P, W.C, W.k, 1000, sched=dict(qt=2, nw=4, range=1), graph=True)
    ids, dist = hntl.hntl_plan_search(plan, bt["Qd"])
    orc = bt["orc"]
    nd, n = parity.check_lists(ids.cpu().numpy(), dist.cpu().numpy(), orc["ids"], orc["dist"],
                               exact_dist_fn(bt["X"], bt["Q"]), what="plan ids")
    assert nd <= 0.01 * n


def test_autotuner_and_lookup(bt, tmp_path):
    W, hntl = bt["W"], bt["hntl"]
    announce("autotuner on 256 queries, tuning file round trip")
    db = tmp_path / "tune.txt"
    Q = bt["Qd"][:256].contiguous()
    best, ms = hntl.hntl_tune(bt["ix"], Q, W.P, W.C, W.k, db_path=db)
    assert ms > 0 and best["qt"] in (1, 2, 4, 8) and 1 <= best["nw"] <= 8 and best["proj"] in (0, 1)
    assert hntl.hntl_schedule_lookup(bt["ix"], W.P, W.C, W.k, 256, db) == best
    text = db.read_text()
    assert text.count("\n") == 1 and "nq=256" in text
    best2, _ = hntl.hntl_tune(bt["ix"], Q, W.P, W.C, W.k, db_path=db)  # replaces its own line
    assert db.read_text().count("\n") == 1
    with pytest.raises(hntl.HNTLError):
        hntl.hntl_schedule_lookup(bt["ix"], W.P, W.C, W.k, 999, db)
    plan = hntl.hntl_plan_create(bt["ix"], W.P, W.C, W.k, 256, sched=best2)
    assert_same(hntl.hntl_plan_search(plan, Q), staged(bt, Q), "tuned schedule")


def test_plan_errors(bt):
    W, hntl = bt["W"], bt["hntl"]
    announce("plan argument errors")
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_plan_create(bt["ix"], W.P, W.C, W.k, 100, sched=dict(qt=3, nw=1, range=0))
    assert e.value.status == hntl.HNTL_EINVAL
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_plan_create(bt["ix"], W.P, W.C, W.k, 100, sched=dict(qt=1, nw=9, range=0))
    assert e.value.status == hntl.HNTL_EINVAL
    with pytest.raises(hntl.HNTLError) as e:  # C beyond the compiled pool size
        hntl.hntl_plan_create(bt["ix"], W.P, 512, W.k, 100, sched=dict(qt=4, nw=8, range=0))
    assert e.value.status == hntl.HNTL_EUNSUPPORTED
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_plan_create(bt["ix"], W.P, W.C, W.k, 0)
    assert e.value.status == hntl.HNTL_EINVAL
    plan = hntl.hntl_plan_create(bt["ix"], W.P, W.C, W.k, 10)
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_plan_search(plan, bt["Qd"][:11].contiguous())
    assert e.value.status == hntl.HNTL_EINVAL


def test_plan_unequal_grains(bt):
    """An index built on the GPU with G = 100 grains over 64 patches: grain sizes
    differ, so the plans' size-ordered item lists (rank -> grain map) are not
    the identity; every schedule form must still equal the staged search."""
    W, hntl, torch = bt["W"], bt["hntl"], bt["torch"]
    announce("G=100 GPU-built index: plans (fused and separate projection) vs staged search")
    ix = hntl.hntl_build(torch.from_numpy(bt["X"]).cuda(), 100, 32, seed=11, codes=("fp32", "bf16"))
    sizes = np.diff(hntl.hntl_index_export(ix)["offsets"])
    assert len(set(sizes.tolist())) > 1
    Q = bt["Qd"]
    for codes, fl in (("fp32", 0), ("bf16", hntl.HNTL_FLAG_PROJECT_BF16)):
        ref = hntl.hntl_search(ix, Q, W.P, W.C, W.k, codes=codes, flags=fl | hntl.HNTL_FLAG_SYNC)
        for sched in (dict(qt=4, nw=2, range=0), dict(qt=4, nw=2, range=0, proj=1),
                      dict(qt=2, nw=4, range=1, passes=2, proj=1), dict(qt=1, nw=8, range=2)):
            plan = hntl.hntl_plan_create(ix, W.P, W.C, W.k, 1000, codes=codes, flags=fl, sched=sched)
            assert_same(hntl.hntl_plan_search(plan, Q), ref, f"G=100 {codes} {sched}")
            assert hntl.hntl_plan_info_get(plan)["wait_errors"] == 0


def test_bf16_routing_forms(bt):
    """Routing's shortlist from plain BF16 or split-BF16 MFMA products (own
    kernels) picks the same probes as FP32 MFMA products: the P winners are
    decided on FP32 direct differences in every form, inside each form's error
    window, so the whole search is unchanged; plans honour the flags."""
    W, hntl, torch = bt["W"], bt["hntl"], bt["torch"]
    announce("BF16 and split-BF16 routing vs FP32 routing (staged and plan)")
    for fl in (hntl.HNTL_FLAG_ROUTE_BF16X3, hntl.HNTL_FLAG_ROUTE_BF16):
        for nb in (1000, 9):  # 9 rows take the direct-difference path
            Q = bt["Qd"][:nb].contiguous()
            a = hntl.hntl_search_stages(bt["ix"], Q, W.P, W.C, W.k)
            b = hntl.hntl_search_stages(bt["ix"], Q, W.P, W.C, W.k, flags=hntl.HNTL_FLAG_SYNC | fl)
            assert torch.equal(a["probes"], b["probes"]), (fl, nb)
            assert torch.equal(a["ids"], b["ids"]) and torch.equal(a["dist"], b["dist"]), (fl, nb)
        plan = hntl.hntl_plan_create(bt["ix"], W.P, W.C, W.k, 1000, flags=fl, sched=dict(qt=2, nw=4, range=1, proj=1))
        assert_same(hntl.hntl_plan_search(plan, bt["Qd"]), staged(bt, bt["Qd"], flags=fl), f"plan, routing {fl}")


def test_routing_forms_reject_both_flags(bt):
    """The two BF16 routing forms are exclusive: asking for both is EINVAL."""
    W, hntl = bt["W"], bt["hntl"]
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_search_stages(bt["ix"], bt["Qd"][:8].contiguous(), W.P, W.C, W.k,
                                flags=hntl.HNTL_FLAG_ROUTE_BF16X3 | hntl.HNTL_FLAG_ROUTE_BF16)
    assert e.value.status == hntl.HNTL_EINVAL


def test_results_do_not_depend_on_the_batch(bt):
    """Every routing product is computed by one kernel whatever the row count
    (a row's output tile and depth order do not depend on the batch), so a
    query's probes and results are the same whatever batch it is searched in:
    rows of batches of 1000, 300, 100 and 64 queries (MFMA products) and of 9
    (direct differences) agree bit for bit, in all three routing forms."""
    W, hntl, torch = bt["W"], bt["hntl"], bt["torch"]
    announce("batch independence of routing and results: 1000 / 300 / 100 / 64 / 9 queries")
    for fl in (0, hntl.HNTL_FLAG_ROUTE_BF16X3, hntl.HNTL_FLAG_ROUTE_BF16):
        full = hntl.hntl_search_stages(bt["ix"], bt["Qd"], W.P, W.C, W.k, flags=hntl.HNTL_FLAG_SYNC | fl)
        for nb in (300, 100, 64, 9):
            part = hntl.hntl_search_stages(bt["ix"], bt["Qd"][:nb].contiguous(), W.P, W.C, W.k,
                                           flags=hntl.HNTL_FLAG_SYNC | fl)
            for k in ("probes", "ids", "dist"):
                assert torch.equal(part[k], full[k][:nb]), (fl, nb, k)


def test_plan_profile_stages(bt):
    """hntl_plan_profile reports five stages; the projection launch has time only
    with a separate projection launch (schedule proj = 1)."""
    W, hntl = bt["W"], bt["hntl"]
    announce("plan profile stages with and without a separate projection launch")
    for proj in (0, 1):
        plan = hntl.hntl_plan_create(bt["ix"], W.P, W.C, W.k, 1000, sched=dict(qt=2, nw=4, range=0, proj=proj))
        hntl.hntl_plan_search(plan, bt["Qd"])
        st, scored = hntl.hntl_plan_profile(plan, 1000, reps=2)
        assert list(st) == ["route", "bucket", "project", "fused", "rerank"]
        assert all(v >= 0 for v in st.values()) and st["fused"] > 0 and st["rerank"] > 0 and scored > 0
        if proj:
            assert st["project"] > 0.005
        else:
            assert st["project"] < 0.05
