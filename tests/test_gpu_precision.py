"""GPU parity of the reduced-precision form (BF16 / FP8 codes, BF16 projection)
against the oracle's emulation of the same rounding points."""
import numpy as np
import pytest

from oracle import quant, search as osr
from tests import parity
from tests.gpu_common import announce, require_gpu, scan_dist_fn, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lowp(small10k):
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    st = {k: small10k["stored"][k] for k in ("centroids", "basis", "offsets", "perm", "codes", "eps")}
    announce("import oracle index 10k x 768 with BF16 and FP8 codes")
    ix = hntl.hntl_index_create(st, small10k["X"], codes=("fp32", "bf16", "fp8"))
    W = small10k["W"]
    orc = osr.search(small10k["Q"], st, small10k["X"], W.P, W.C, W.k)
    return dict(small10k, st=st, ix=ix, Qd=to_dev(small10k["Q"]), orc=orc, torch=torch, hntl=hntl)


def test_codes_bit_exact(lowp):
    announce("BF16 / FP8 codes and scales bit-exact")
    hntl, st = lowp["hntl"], lowp["st"]
    b16, _ = hntl.hntl_index_export_codes(lowp["ix"], "bf16")
    np.testing.assert_array_equal(b16, quant.bf16_bits(st["codes"]))
    f8, sc = hntl.hntl_index_export_codes(lowp["ix"], "fp8")
    c, sc_o = quant.fp8_grain_codes(st["codes"], st["offsets"])
    np.testing.assert_array_equal(sc, sc_o)
    np.testing.assert_array_equal(f8, quant.fp8_encode_byte(c))


@pytest.mark.parametrize("form", ["bf16", "fp8"])
def test_lowp_scan_parity(lowp, form):
    announce(f"{form} scan parity with oracle probes and tangents injected")
    W, hntl = lowp["W"], lowp["hntl"]
    orc = lowp["orc"]
    st = lowp["st"]
    o = hntl.hntl_search_stages(lowp["ix"], lowp["Qd"], W.P, W.C, W.k, codes=form,
                                probes_in=to_dev(orc["probes"].astype(np.int32)),
                                tangent_in=to_dev(orc["zq"].astype(np.float32)),
                                epsq_in=to_dev(orc["epsq"].astype(np.float32)))
    dec = dict(st, codes=quant.decoded_codes(st["codes"], st["offsets"], form))
    pool_ids, pool_D = osr.scan_pool(orc["zq"], orc["epsq"], orc["probes"], st, W.C, form)
    nd, n = parity.check_lists(o["pool_ids"].cpu().numpy(), o["pool_D"].cpu().numpy(), pool_ids, pool_D,
                               scan_dist_fn(dec, orc["zq"], orc["epsq"], orc["probes"]), what=f"{form} pool")
    assert nd <= 0.01 * n


def test_bf16_projection_parity(lowp):
    announce("BF16 projection parity with oracle probes injected")
    W, hntl = lowp["W"], lowp["hntl"]
    orc = lowp["orc"]
    o = hntl.hntl_search_stages(lowp["ix"], lowp["Qd"], W.P, W.C, W.k, codes="bf16",
                                flags=hntl.HNTL_FLAG_SYNC | hntl.HNTL_FLAG_PROJECT_BF16,
                                probes_in=to_dev(orc["probes"].astype(np.int32)))
    zb, eb = osr.project(lowp["Q"], orc["probes"], lowp["st"], bf16=True)
    zq = o["zq"].cpu().numpy().astype(np.float64)
    eq = o["epsq"].cpu().numpy().astype(np.float64)
    qn2 = (zb ** 2).sum(-1) + eb
    assert (np.abs(zq - zb) <= 4e-6 * np.sqrt(qn2)[..., None]).all(), float(np.abs(zq - zb).max())
    assert (np.abs(eq - eb) <= 1e-4 * np.maximum(eb, 1e-3 * qn2)).all()


@pytest.mark.parametrize("form", ["bf16", "fp8"])
def test_lowp_end_to_end(lowp, form):
    """Full reduced-precision search: recall stays at the FP32 level, the
    pruned scan equals the full scan bitwise, and the final distances are the
    exact FP32 ones (rerank never uses codes)."""
    announce(f"{form} end-to-end search with BF16 projection")
    W, hntl, torch = lowp["W"], lowp["hntl"], lowp["torch"]
    fl = hntl.HNTL_FLAG_SYNC | hntl.HNTL_FLAG_PROJECT_BF16
    a = hntl.hntl_search_stages(lowp["ix"], lowp["Qd"], W.P, W.C, W.k, codes=form, flags=fl)
    b = hntl.hntl_search_stages(lowp["ix"], lowp["Qd"], W.P, W.C, W.k, codes=form, flags=fl | hntl.HNTL_FLAG_NO_PRUNE)
    for key in ("pool_ids", "pool_D", "ids", "dist"):
        assert torch.equal(a[key], b[key]), key
    ids = a["ids"].cpu().numpy()
    assert osr.recall(ids, lowp["gt_ids"]) >= 0.99
    X, Q = lowp["X"], lowp["Q"]
    exact = ((X[ids].astype(np.float64) - Q[:, None, :].astype(np.float64)) ** 2).sum(-1)
    np.testing.assert_allclose(a["dist"].cpu().numpy(), exact, rtol=1e-4)
