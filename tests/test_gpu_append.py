"""GPU tests of incremental segments (hntl_index_append): rows appended to an
index imported from the oracle's build, against the oracle's append.

* without splits: new rows' grains equal the oracle's wherever the oracle's
  nearest and second-nearest centroids are not a near tie (and are valid
  there), layout and ids equal, existing codes and every centroid and basis
  bit for bit, new codes and eps within FP32 rounding of the FP64 values;
* with splits: the same partition (cut positions decided on the same FP32
  code values), child centroids within FP32 rounding, child bases capturing
  the same variance and giving the same residual energies as the oracle's
  eigendecomposition (tolerances of the build's own test), codes consistent
  with the stored bases;
* the base index is unchanged, two appends equal one, an appended row is its
  own nearest neighbour, recall of searches on the result.
"""
import numpy as np
import pytest

from oracle import brute, index as oi, pca, search as osr, segments as sg
from tests.gpu_common import announce, require_gpu, to_dev

pytestmark = pytest.mark.gpu

KEYS = ("centroids", "basis", "offsets", "perm", "codes", "eps")


@pytest.fixture(scope="module")
def ap(small10k):
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    st = {k: small10k["stored"][k] for k in KEYS}
    announce("import oracle index 10k x 768 for appends")
    ix0 = hntl.hntl_index_create(st, small10k["X"])
    # 1,000 new rows from the same patch mixture (the workload's query rows)
    Xn = np.ascontiguousarray(small10k["Q"], dtype=np.float32)
    return dict(small10k, st=st, ix0=ix0, Xn=Xn, torch=torch, hntl=hntl)


def _grain_of(ex):
    lab = np.empty(len(ex["perm"]), np.int64)
    for g in range(len(ex["offsets"]) - 1):
        lab[ex["perm"][ex["offsets"][g]:ex["offsets"][g + 1]]] = g
    return lab


def _check_assignment(ex, orc, st, Xn, N):
    lab = _grain_of(ex)[N:]
    C = st["centroids"].astype(np.float64)
    D = ((Xn.astype(np.float64)[:, None, :] - C[None]) ** 2).sum(-1)
    dmin = D.min(1)
    sure = orc["assign_gap"] > 1e-4 * np.maximum(dmin, 1e-12)
    np.testing.assert_array_equal(lab[sure], orc["new_grain"][sure])
    # near ties: the GPU's grain is one of the nearest within the tie window
    got = D[np.arange(len(lab)), lab]
    assert np.all(got <= dmin * (1 + 1e-4) + 1e-9)
    return bool(sure.all())


def _export(hntl, ix):
    return hntl.hntl_index_export(ix)


def test_append_without_split(ap):
    hntl, st, Xn = ap["hntl"], ap["st"], ap["Xn"]
    N = len(st["perm"])
    announce("append 1000 rows to the 10k index, no split")
    before = _export(hntl, ap["ix0"])
    ix1 = hntl.hntl_index_append(ap["ix0"], Xn)
    ex = _export(hntl, ix1)
    assert ix1.N == N + len(Xn) and ix1.G == len(st["offsets"]) - 1
    orc = sg.append(st, ap["X"], Xn)
    assert _check_assignment(ex, orc, st, Xn, N)
    np.testing.assert_array_equal(ex["offsets"], orc["offsets"])
    np.testing.assert_array_equal(ex["perm"], orc["perm"])
    np.testing.assert_array_equal(ex["centroids"], st["centroids"])
    np.testing.assert_array_equal(ex["basis"], st["basis"])
    old = ex["perm"] < N
    np.testing.assert_array_equal(ex["codes"][old], orc["codes"][old].astype(np.float32))
    np.testing.assert_array_equal(ex["eps"][old], orc["eps"][old].astype(np.float32))
    scale = np.abs(orc["codes"][~old]).max()
    np.testing.assert_allclose(ex["codes"][~old], orc["codes"][~old], rtol=0, atol=2e-6 * scale)
    np.testing.assert_allclose(ex["eps"][~old], orc["eps"][~old], rtol=1e-5, atol=1e-6 * scale ** 2)
    after = _export(hntl, ap["ix0"])
    for k in KEYS:
        np.testing.assert_array_equal(after[k], before[k])


def test_two_appends_equal_one_and_empty_append(ap):
    hntl, Xn = ap["hntl"], ap["Xn"]
    announce("append 400 then 600 rows vs 1000 at once; empty append")
    one = _export(hntl, hntl.hntl_index_append(ap["ix0"], Xn))
    two = _export(hntl, hntl.hntl_index_append(hntl.hntl_index_append(ap["ix0"], Xn[:400]), ap["torch"].from_numpy(Xn[400:]).cuda()))
    for k in KEYS:
        np.testing.assert_array_equal(two[k], one[k])
    same = _export(hntl, hntl.hntl_index_append(ap["ix0"], np.zeros((0, Xn.shape[1]), np.float32)))
    base = _export(hntl, ap["ix0"])
    for k in KEYS:
        np.testing.assert_array_equal(same[k], base[k])


def test_append_with_split(ap):
    hntl, st, Xn, X = ap["hntl"], ap["st"], ap["Xn"], ap["X"]
    N = len(st["perm"])
    plain = sg.append(st, X, Xn)
    sizes = np.diff(plain["offsets"])
    cap = int(np.percentile(sizes, 70))
    announce(f"append 1000 rows with split_max={cap}")
    ix2 = hntl.hntl_index_append(ap["ix0"], Xn, split_max=cap, seed=3)
    ex = _export(hntl, ix2)
    orc = sg.append(st, X, Xn, split_max=cap)
    # the new rows' grains before the split are checked without splits above;
    # here the final partitions must match, so no assignment may be a near tie
    D = ((Xn.astype(np.float64)[:, None, :] - st["centroids"].astype(np.float64)[None]) ** 2).sum(-1)
    assert np.all(orc["assign_gap"] > 1e-4 * D.min(1))
    assert len(orc["children"]) > 0 and np.all(orc["cut_gaps"] > 0)
    assert ix2.G == len(orc["offsets"]) - 1
    np.testing.assert_array_equal(ex["offsets"], orc["offsets"])
    np.testing.assert_array_equal(ex["perm"], orc["perm"])
    assert np.diff(ex["offsets"]).max() <= cap
    kids = set(orc["children"].tolist())
    Xall = np.vstack([X, Xn])
    cap_gpu = hntl.hntl_index_captured(ix2)
    for g in range(ix2.G):
        a, b = int(ex["offsets"][g]), int(ex["offsets"][g + 1])
        if g not in kids:
            np.testing.assert_array_equal(ex["centroids"][g], st["centroids"][g])
            np.testing.assert_array_equal(ex["basis"][g], st["basis"][g])
            continue
        np.testing.assert_allclose(ex["centroids"][g], orc["centroids"][g], rtol=0, atol=2e-6)
        Bg = ex["basis"][g].astype(np.float64)
        assert np.abs(Bg @ Bg.T - np.eye(Bg.shape[0])).max() < 2e-6
        ids = ex["perm"][a:b]
        _, _, cap_o = pca.local_pca(Xall[ids], Xall[ids].astype(np.float64).mean(0), Bg.shape[0])
        assert abs(cap_gpu[g] - cap_o) < 1e-6
        np.testing.assert_allclose(ex["eps"][a:b], orc["eps"][a:b], rtol=2e-3, atol=2e-4)
    # every code against the stored centroid and basis it was made with
    codes64, eps64 = oi.stored_encode(Xall, ex)
    np.testing.assert_allclose(ex["codes"], codes64, atol=2e-5 * np.sqrt(np.abs(codes64).max() + 1))
    np.testing.assert_allclose(ex["eps"], eps64, rtol=1e-4, atol=1e-4)
    # searches on the result: an appended row is its own nearest neighbour; recall
    torch, W = ap["torch"], ap["W"]
    q = to_dev(Xn[:200])
    ids, dist = hntl.hntl_search(ix2, q, W.P, 100, W.k, flags=hntl.HNTL_FLAG_SYNC)
    np.testing.assert_array_equal(ids.cpu().numpy()[:, 0], N + np.arange(200))
    assert float(dist[:, 0].abs().max()) < 1e-3
    Qn = Xn[200:400] + np.float32(0.05)
    gt, _ = brute.knn(Xall, Qn, W.k)
    ids, _ = hntl.hntl_search(ix2, to_dev(np.ascontiguousarray(Qn)), W.P, W.C, W.k, flags=hntl.HNTL_FLAG_SYNC)
    rec = osr.recall(ids.cpu().numpy(), gt)
    orc_ids = osr.search(Qn, orc, Xall, W.P, W.C, W.k)["ids"]
    assert rec >= osr.recall(orc_ids, gt) - 0.01


def test_append_to_index_without_raw_vectors(ap):
    hntl, st, Xn = ap["hntl"], ap["st"], ap["Xn"]
    announce("append to an index imported without raw vectors (Mode A), bf16 codes")
    ixa = hntl.hntl_index_create(st, None, codes=("fp32", "bf16"))
    with pytest.raises(hntl.HNTLError):
        hntl.hntl_index_append(ixa, Xn, split_max=100)
    ixb = hntl.hntl_index_append(ixa, Xn)
    ex = _export(hntl, ixb)
    full = _export(hntl, hntl.hntl_index_append(ap["ix0"], Xn))
    for k in KEYS:
        np.testing.assert_array_equal(ex[k], full[k])
    assert hntl.hntl_index_info_get(ixb)["codes_mask"] == (1 | (1 << hntl.HNTL_CODES_BF16))
    W = ap["W"]
    ids, _ = hntl.hntl_search(ixb, to_dev(Xn[:100]), W.P, 100, W.k, flags=hntl.HNTL_FLAG_SYNC | hntl.HNTL_FLAG_MODE_A)
    np.testing.assert_array_equal(ids.cpu().numpy()[:, 0], len(st["perm"]) + np.arange(100))
