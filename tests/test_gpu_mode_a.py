"""GPU tests of Mode A (the paper's self-contained mode, Section 2.1): the
answer is the k smallest reconstruction distances ||z_q - z_i||^2 + eps_q over
the pool, with no raw vectors read.

Checked against the oracle's Mode A (which evaluates the reconstruction
distance from the pair's tangent and the code values) on the oracle's own
index, with the parity rule of tests/parity.py (ids up to near-ties within
1e-5, distances within 1e-4 relative); plans must equal the staged search bit
for bit; an index imported without raw vectors answers Mode A searches and
refuses the others.
"""
import numpy as np
import pytest

from oracle import brute, search as osr
from tests import parity
from tests.gpu_common import announce, require_gpu, to_dev

pytestmark = pytest.mark.gpu

KEYS = ("centroids", "basis", "offsets", "perm", "codes", "eps")


@pytest.fixture(scope="module")
def ma(small10k):
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    st = {k: small10k["stored"][k] for k in KEYS}
    announce("import oracle index 10k x 768 with and without raw vectors (Mode A)")
    ix = hntl.hntl_index_create(st, small10k["X"], codes=("fp32", "bf16"))
    ix_noraw = hntl.hntl_index_create(st, None, codes=("fp32", "bf16"))
    W = small10k["W"]
    return dict(small10k, st=st, ix=ix, ix_noraw=ix_noraw, Qd=to_dev(small10k["Q"]), torch=torch, hntl=hntl)


def mode_a_dist_fn(st, out):
    """oracle_dist_of(row, ids) for Mode A: ||z_q,s - z_i||^2 + eps_q,s, s the probe slot of i's grain."""
    perm = np.asarray(st["perm"], dtype=np.int64)
    off = np.asarray(st["offsets"], dtype=np.int64)
    pos_of = np.empty(len(perm), dtype=np.int64)
    pos_of[perm] = np.arange(len(perm))

    def f(i, ids):
        pos = pos_of[np.asarray(ids, dtype=np.int64)]
        g = np.searchsorted(off, pos, side="right") - 1
        slot = np.array([int(np.flatnonzero(out["probes"][i] == gg)[0]) for gg in g])
        Z = np.asarray(st["codes"][pos], dtype=np.float64)
        return ((out["zq"][i, slot] - Z) ** 2).sum(1) + out["epsq"][i, slot]
    return f


def test_mode_a_oracle_parity(ma):
    W, hntl = ma["W"], ma["hntl"]
    announce("Mode A staged search vs oracle Mode A, 1000 queries")
    orc = osr.search(ma["Q"], ma["st"], None, W.P, W.C, W.k, mode="A")
    ids, dist = hntl.hntl_search(ma["ix"], ma["Qd"], W.P, W.C, W.k, flags=hntl.HNTL_FLAG_SYNC | hntl.HNTL_FLAG_MODE_A)
    nd, n = parity.check_lists(ids.cpu().numpy(), dist.cpu().numpy(), orc["ids"], orc["dist"],
                               mode_a_dist_fn(ma["st"], orc), what="Mode A ids")
    assert nd <= 0.01 * n
    gt = ma["gt_ids"]
    rec = osr.recall(ids.cpu().numpy(), gt, W.k)
    rec_b = osr.recall(hntl.hntl_search(ma["ix"], ma["Qd"], W.P, W.C, W.k,
                                        flags=hntl.HNTL_FLAG_SYNC)[0].cpu().numpy(), gt, W.k)
    announce(f"Recall@10 Mode A {rec:.4f}, Mode B {rec_b:.4f}")
    assert rec >= 0.8 and rec <= rec_b + 1e-9


@pytest.mark.parametrize("sched", [dict(qt=4, nw=2, range=0), dict(qt=2, nw=4, range=1, proj=1)],
                         ids=["fused", "split-projection"])
def test_mode_a_plan_equals_staged(ma, sched):
    W, hntl, torch = ma["W"], ma["hntl"], ma["torch"]
    announce(f"Mode A plan {sched} vs staged")
    fl = hntl.HNTL_FLAG_MODE_A
    a = hntl.hntl_search(ma["ix"], ma["Qd"], W.P, W.C, W.k, flags=hntl.HNTL_FLAG_SYNC | fl)
    plan = hntl.hntl_plan_create(ma["ix"], W.P, W.C, W.k, 1000, flags=fl, sched=sched)
    b = hntl.hntl_plan_search(plan, ma["Qd"])
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_mode_a_bf16_codes(ma):
    """BF16 codes (FP32 projection): the reconstruction uses the decoded code values."""
    W, hntl = ma["W"], ma["hntl"]
    announce("Mode A with BF16 codes vs oracle (decoded BF16 code values)")
    orc = osr.search(ma["Q"], ma["st"], None, W.P, W.C, W.k, mode="A", form="bf16")
    ids, dist = hntl.hntl_search(ma["ix"], ma["Qd"], W.P, W.C, W.k, codes="bf16",
                                 flags=hntl.HNTL_FLAG_SYNC | hntl.HNTL_FLAG_MODE_A)
    from oracle import quant
    st_dec = dict(ma["st"], codes=quant.decoded_codes(ma["st"]["codes"], ma["st"]["offsets"], "bf16"))
    nd, n = parity.check_lists(ids.cpu().numpy(), dist.cpu().numpy(), orc["ids"], orc["dist"],
                               mode_a_dist_fn(st_dec, orc), what="Mode A bf16 ids")
    assert nd <= 0.01 * n


def test_index_without_raw_vectors(ma):
    W, hntl, torch = ma["W"], ma["hntl"], ma["torch"]
    announce("index without raw vectors: Mode A works, Mode B refused")
    fl = hntl.HNTL_FLAG_SYNC | hntl.HNTL_FLAG_MODE_A
    a = hntl.hntl_search(ma["ix"], ma["Qd"], W.P, W.C, W.k, flags=fl)
    b = hntl.hntl_search(ma["ix_noraw"], ma["Qd"], W.P, W.C, W.k, flags=fl)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_search(ma["ix_noraw"], ma["Qd"], W.P, W.C, W.k, flags=hntl.HNTL_FLAG_SYNC)
    assert e.value.status == hntl.HNTL_ESTATE
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_plan_create(ma["ix_noraw"], W.P, W.C, W.k, 100)
    assert e.value.status == hntl.HNTL_ESTATE
    plan = hntl.hntl_plan_create(ma["ix_noraw"], W.P, W.C, W.k, 1000, flags=hntl.HNTL_FLAG_MODE_A)
    c = hntl.hntl_plan_search(plan, ma["Qd"])
    torch.cuda.synchronize()
    assert torch.equal(a[0], c[0]) and torch.equal(a[1], c[1])
