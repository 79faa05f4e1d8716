"""GPU tests of index files (hntl_index_save / hntl_index_load): NumPy reads
the arrays directly and they equal the exported index; a loaded index equals
the saved one array for array and answers searches bit for bit alike; the
learned router, the captured-variance record and indexes without raw vectors
survive the round trip; missing or corrupted files give HNTL_EIO."""
import json

import numpy as np
import pytest

from tests.gpu_common import announce, require_gpu, to_dev

pytestmark = pytest.mark.gpu

KEYS = ("centroids", "basis", "offsets", "perm", "codes", "eps")


@pytest.fixture(scope="module")
def io(small10k):
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    st = {k: small10k["stored"][k] for k in KEYS}
    return dict(small10k, st=st, torch=torch, hntl=hntl)


def test_save_load_roundtrip_and_search(io, tmp_path):
    hntl, W = io["hntl"], io["W"]
    announce("save / load the 10k index (FP32 + BF16 codes, raw vectors)")
    ix = hntl.hntl_index_create(io["st"], io["X"], codes=("fp32", "bf16"))
    d = tmp_path / "ix10k"
    hntl.hntl_index_save(ix, d)
    ex = hntl.hntl_index_export(ix)
    for k in KEYS:  # plain NumPy reads every array
        np.testing.assert_array_equal(np.load(d / f"{k}.npy", allow_pickle=False), ex[k])
    np.testing.assert_array_equal(np.load(d / "X.npy", allow_pickle=False), io["X"])
    meta = json.loads((d / "meta.json").read_text())
    assert meta["N"] == W.N and meta["G"] == W.G and meta["raw_vectors"] == 1
    ix2 = hntl.hntl_index_load(d)
    ex2 = hntl.hntl_index_export(ix2)
    for k in KEYS:
        np.testing.assert_array_equal(ex2[k], ex[k])
    assert hntl.hntl_index_info_get(ix2)["codes_mask"] == hntl.hntl_index_info_get(ix)["codes_mask"]
    Q = to_dev(io["Q"])
    for codes in ("fp32", "bf16"):
        a = hntl.hntl_search(ix, Q, W.P, W.C, W.k, codes=codes, flags=hntl.HNTL_FLAG_SYNC)
        b = hntl.hntl_search(ix2, Q, W.P, W.C, W.k, codes=codes, flags=hntl.HNTL_FLAG_SYNC)
        assert io["torch"].equal(a[0], b[0]) and io["torch"].equal(a[1], b[1])


def test_router_captured_and_no_raw_vectors(io, tmp_path):
    hntl, W = io["hntl"], io["W"]
    announce("save / load: built index with captured record, random router; index without raw vectors")
    ix = hntl.hntl_build(to_dev(io["X"]), W.G, W.r, init_centroids=to_dev(io["st"]["centroids"]), seed=5)
    rng = np.random.default_rng(1)
    d_, h = io["X"].shape[1], 64
    p = {"W1": rng.standard_normal((h, d_), dtype=np.float32) * 0.05, "b1": rng.standard_normal(h, dtype=np.float32),
         "W2": rng.standard_normal((h, h), dtype=np.float32) * 0.1, "b2": rng.standard_normal(h, dtype=np.float32),
         "W3": rng.standard_normal((W.G, h), dtype=np.float32) * 0.1, "b3": rng.standard_normal(W.G, dtype=np.float32)}
    mean = rng.standard_normal(d_, dtype=np.float32)
    std = rng.uniform(0.5, 2.0, d_).astype(np.float32)
    hntl.hntl_router_set(ix, p, mean, std)
    hntl.hntl_index_save(ix, tmp_path / "b")
    ix2 = hntl.hntl_index_load(tmp_path / "b")
    np.testing.assert_array_equal(hntl.hntl_index_captured(ix2), hntl.hntl_index_captured(ix))
    r1, r2 = hntl.hntl_router_export(ix), hntl.hntl_router_export(ix2)
    for k in r1:
        np.testing.assert_array_equal(np.asarray(r2[k]), np.asarray(r1[k]))
    Q = to_dev(io["Q"])
    a = hntl.hntl_search(ix, Q, W.P, W.C, W.k, route="learned", flags=hntl.HNTL_FLAG_SYNC)
    b = hntl.hntl_search(ix2, Q, W.P, W.C, W.k, route="learned", flags=hntl.HNTL_FLAG_SYNC)
    assert io["torch"].equal(a[0], b[0]) and io["torch"].equal(a[1], b[1])
    # an index without raw vectors stays one: Mode A answers, Mode B refuses
    ixa = hntl.hntl_index_create(io["st"], None)
    hntl.hntl_index_save(ixa, tmp_path / "a")
    assert not (tmp_path / "a" / "X.npy").exists()
    ixa2 = hntl.hntl_index_load(tmp_path / "a")
    fa = hntl.HNTL_FLAG_SYNC | hntl.HNTL_FLAG_MODE_A
    a = hntl.hntl_search(ixa, Q, W.P, W.C, W.k, flags=fa)
    b = hntl.hntl_search(ixa2, Q, W.P, W.C, W.k, flags=fa)
    assert io["torch"].equal(a[0], b[0]) and io["torch"].equal(a[1], b[1])
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_search(ixa2, Q, W.P, W.C, W.k, flags=hntl.HNTL_FLAG_SYNC)
    assert e.value.status == hntl.HNTL_ESTATE


def test_load_errors(io, tmp_path):
    hntl = io["hntl"]
    announce("load: missing directory, missing file, corrupted data, wrong shape")
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_index_load(tmp_path / "nothing-here")
    assert e.value.status == hntl.HNTL_EIO
    ix = hntl.hntl_index_create(io["st"], None)
    d = tmp_path / "c"
    hntl.hntl_index_save(ix, d)
    raw = bytearray((d / "codes.npy").read_bytes())
    raw[-5] ^= 0x40  # one bit of the last code
    (d / "codes.npy").write_bytes(bytes(raw))
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_index_load(d)
    assert e.value.status == hntl.HNTL_EIO and "checksum" in str(e.value)
    hntl.hntl_index_save(ix, d)
    np.save(d / "eps.npy", np.zeros(7, np.float32))  # a valid .npy of the wrong shape
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_index_load(d)
    assert e.value.status == hntl.HNTL_EIO and "shape" in str(e.value)
    hntl.hntl_index_save(ix, d)
    (d / "perm.npy").unlink()
    with pytest.raises(hntl.HNTLError) as e:
        hntl.hntl_index_load(d)
    assert e.value.status == hntl.HNTL_EIO
