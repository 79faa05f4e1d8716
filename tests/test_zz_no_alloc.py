"""GPU test of hntl_search_noalloc, the entry point for callers that cannot
allocate device memory: through the C ABI its results equal hntl_search's bit
for bit (the same kernels on the same inputs), on two calls in a row, the
second with a smaller batch, so the static scratch array's leftover contents
from the first call must not leak into the second."""
import ctypes as C

import numpy as np
import pytest

from tests.gpu_common import announce, require_gpu, to_dev

pytestmark = pytest.mark.gpu


def _call(hntl, fn, ix, Q, P, Cc, k, flags=0, route=0, tau=0.0, codes=0):
    import torch
    nq = Q.shape[0]
    ids = torch.full((nq, k), -7, dtype=torch.int32, device=Q.device)
    dist = torch.full((nq, k), float("nan"), dtype=torch.float32, device=Q.device)
    sp = hntl.hntl_search_params(P, Cc, k, codes, flags | hntl.HNTL_FLAG_SYNC, route, tau)
    st = getattr(hntl.lib(), fn)(ix.handle, Q.data_ptr(), nq, C.byref(sp), ids.data_ptr(), dist.data_ptr(), None)
    return st, ids, dist


def test_noalloc_equals_search_on_two_calls(small10k):
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    st = small10k["stored"]
    W = small10k["W"]
    ix = hntl.hntl_index_create({k: st[k] for k in ("centroids", "basis", "offsets", "perm", "codes", "eps")},
                                small10k["X"], codes=("fp32", "bf16"))
    Qd = to_dev(small10k["Q"])
    cases = [(1000, W.P, W.C, 0), (137, W.P + 2, W.C + 11, 0),
             (1000, W.P, W.C, hntl.HNTL_FLAG_ROUTE_BF16), (61, 2, 33, hntl.HNTL_FLAG_ROUTE_BF16)]
    # the BF16 routing form derives the split centroids in its first hntl_search
    for nq, P, Cc, fl in cases:
        announce(f"no-alloc search vs hntl_search: nq={nq} P={P} C={Cc} flags={fl}")
        Q = Qd[:nq].contiguous()
        s0, i0, d0 = _call(hntl, "hntl_search", ix, Q, P, Cc, W.k, fl)
        s1, i1, d1 = _call(hntl, "hntl_search_noalloc", ix, Q, P, Cc, W.k, fl)
        assert s0 == hntl.HNTL_OK and s1 == hntl.HNTL_OK, (s0, s1, hntl.hntl_last_error())
        assert torch.equal(i0, i1) and torch.equal(d0, d1), (nq, P, Cc, fl)
    # BF16 codes with BF16 projection, then a smaller FP32 call after it
    for nq, codes, fl in ((1000, 1, hntl.HNTL_FLAG_PROJECT_BF16), (300, 0, 0)):
        Q = Qd[:nq].contiguous()
        s0, i0, d0 = _call(hntl, "hntl_search", ix, Q, W.P, W.C, W.k, fl, codes=codes)
        s1, i1, d1 = _call(hntl, "hntl_search_noalloc", ix, Q, W.P, W.C, W.k, fl, codes=codes)
        assert s0 == hntl.HNTL_OK and s1 == hntl.HNTL_OK
        assert torch.equal(i0, i1) and torch.equal(d0, d1), (nq, codes)


def test_noalloc_limits_and_errors(small10k):
    torch = require_gpu()
    from paper_2606_08813_amd import hntl
    st = small10k["stored"]
    W = small10k["W"]
    ix = hntl.hntl_index_create({k: st[k] for k in ("centroids", "basis", "offsets", "perm", "codes", "eps")},
                                small10k["X"])
    announce("no-alloc search: size limit, refused profile flag, missing derived data")
    # 40,000 queries x P = 16 x C = 256 candidate keys alone need 1.3 GB: refused, nothing written
    big = torch.zeros((40000, W.d), dtype=torch.float32, device="cuda")
    s, ids, _ = _call(hntl, "hntl_search_noalloc", ix, big, 16, 256, W.k)
    assert s == hntl.HNTL_EINVAL and "HNTL_NOALLOC_SCRATCH_BYTES" in hntl.hntl_last_error()
    assert (ids == -7).all()
    Q = to_dev(small10k["Q"][:50])
    s, _, _ = _call(hntl, "hntl_search_noalloc", ix, Q, W.P, W.C, W.k, hntl.HNTL_FLAG_PROFILE)
    assert s == hntl.HNTL_EINVAL
    # this fresh index has no split centroids yet: the BF16 routing form is refused until made
    s, _, _ = _call(hntl, "hntl_search_noalloc", ix, Q, W.P, W.C, W.k, hntl.HNTL_FLAG_ROUTE_BF16X3)
    assert s == hntl.HNTL_ESTATE
    s0, i0, d0 = _call(hntl, "hntl_search", ix, Q, W.P, W.C, W.k, hntl.HNTL_FLAG_ROUTE_BF16X3)
    s1, i1, d1 = _call(hntl, "hntl_search_noalloc", ix, Q, W.P, W.C, W.k, hntl.HNTL_FLAG_ROUTE_BF16X3)
    assert s0 == s1 == hntl.HNTL_OK and torch.equal(i0, i1) and torch.equal(d0, d1)
