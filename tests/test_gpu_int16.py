"""GPU parity of the paper's own int16 form (eq. 5: int16 codes, uint16
residuals, per-grain steps, exact integer squared distance, quantisation
envelope filter) against the oracle's integer evaluation of the same form.

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
    announce("int16 codes and steps bit-exact")
    st = i16["st"]
    codes, inv = i16["hntl"].hntl_index_export_codes(i16["ix"], "int16")
    zh, rh, inv_o, rinv_o = quant.int16_grain_codes(st["codes"], st["eps"], st["offsets"], st["basis"].shape[1])
    np.testing.assert_array_equal(inv, inv_o)
    np.testing.assert_array_equal(codes.astype(np.int64), zh)


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
    """Full int16 search with exact FP32 rerank: parity of the final results
    with the oracle's int16 lifecycle, and recall."""
    announce("int16 end-to-end search")
    W, hntl = i16["W"], i16["hntl"]
    o = hntl.hntl_search_stages(i16["ix"], i16["Qd"], W.P, W.C, W.k, codes="int16")
    ids = o["ids"].cpu().numpy()
    rec = osr.recall(ids, i16["gt_ids"])
    announce(f"int16 Recall@10 {rec:.4f}")
    assert rec >= 0.97
    X, Q = i16["X"], i16["Q"]
    exact = ((X[ids].astype(np.float64) - Q[:, None, :].astype(np.float64)) ** 2).sum(-1)
    np.testing.assert_allclose(o["dist"].cpu().numpy(), exact, rtol=1e-4)


def test_int16_unsupported_forms(i16):
    W, hntl = i16["W"], i16["hntl"]
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_plan_create(i16["ix"], W.P, W.C, W.k, 100, codes="int16")
    assert e.value.status == hntl.HNTL_EUNSUPPORTED
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_search(i16["ix"], i16["Qd"][:4].contiguous(), W.P, W.C, W.k, codes="int16",
                         flags=hntl.HNTL_FLAG_MODE_A)
    assert e.value.status == hntl.HNTL_EUNSUPPORTED
