"""Python binding of the HNTL C ABI (``include/hntl.h``).

Argument marshalling only: every step of the search runs in the HIP library.
PyTorch supplies device memory (tensors) and streams.  The functions keep the
C names; array arguments are torch CUDA tensors (or, where the C ABI accepts
host memory, contiguous numpy arrays).

Loading fails loudly when the shared library has not been built.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from pathlib import Path

import numpy as np

LIB_PATH = Path(__file__).resolve().parent / "libhntl.so"

HNTL_OK, HNTL_EINVAL, HNTL_ENOMEM, HNTL_EDEVICE, HNTL_ESTATE, HNTL_EIO, HNTL_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
HNTL_CODES_FP32, HNTL_CODES_BF16, HNTL_CODES_FP8_E4M3, HNTL_CODES_INT16 = 0, 1, 2, 3
HNTL_FLAG_SYNC, HNTL_FLAG_CHECK_Q, HNTL_FLAG_PROFILE, HNTL_FLAG_NO_PRUNE, HNTL_FLAG_PROJECT_BF16 = 1, 2, 4, 8, 16
HNTL_FLAG_ROUTE_BF16X3 = 32
HNTL_FLAG_ROUTE_BF16 = 128
HNTL_FLAG_MODE_A = 64
HNTL_ROUTE_CENTROID, HNTL_ROUTE_LEARNED = 0, 1
HNTL_ROUTER_KEEP_WEIGHTS, HNTL_ROUTER_NO_SHUFFLE = 1, 2
ROUTES = {"centroid": HNTL_ROUTE_CENTROID, "learned": HNTL_ROUTE_LEARNED}
STAGES = ("route", "bucket", "project", "scan", "rerank")
HNTL_MAX_R, HNTL_MAX_C, HNTL_MAX_P, HNTL_BLOCK = 64, 256, 48, 64
CODES = {"fp32": HNTL_CODES_FP32, "bf16": HNTL_CODES_BF16, "fp8": HNTL_CODES_FP8_E4M3, "int16": HNTL_CODES_INT16}


class hntl_build_params(C.Structure):
    _fields_ = [("G", C.c_uint32), ("r", C.c_uint32), ("kmeans_iters", C.c_uint32),
                ("train_per_grain", C.c_uint32), ("eig_iters", C.c_uint32), ("codes_mask", C.c_uint32),
                ("seed", C.c_uint64), ("init_centroids", C.c_void_p)]


class hntl_append_params(C.Structure):
    _fields_ = [("split_max", C.c_uint32), ("eig_iters", C.c_uint32), ("seed", C.c_uint64)]


class hntl_search_params(C.Structure):
    _fields_ = [("P", C.c_uint32), ("C", C.c_uint32), ("k", C.c_uint32), ("codes", C.c_uint32),
                ("flags", C.c_uint32), ("route", C.c_uint32), ("tau", C.c_float),
                ("mass", C.c_float)]


class hntl_router_params(C.Structure):
    _fields_ = [("hidden1", C.c_uint32), ("hidden2", C.c_uint32), ("epochs", C.c_uint32), ("batch", C.c_uint32),
                ("knn", C.c_uint32), ("flags", C.c_uint32), ("lr", C.c_float), ("seed", C.c_uint64)]


class hntl_index_info(C.Structure):
    _fields_ = [("N", C.c_uint64), ("d", C.c_uint32), ("G", C.c_uint32), ("r", C.c_uint32),
                ("block", C.c_uint32), ("codes_mask", C.c_uint32), ("n_blocks", C.c_uint64),
                ("device_bytes", C.c_uint64), ("captured_variance", C.c_double),
                ("kmeans_iters_run", C.c_uint32), ("max_grain", C.c_uint32)]


class hntl_schedule(C.Structure):
    _fields_ = [("qt", C.c_uint32), ("nw", C.c_uint32), ("range", C.c_uint32), ("grid", C.c_uint32),
                ("passes", C.c_uint32), ("proj", C.c_uint32)]


class hntl_plan_info(C.Structure):
    _fields_ = [("max_nq", C.c_uint32), ("sched", hntl_schedule), ("graph", C.c_uint32),
                ("device_bytes", C.c_uint64), ("list_slots", C.c_uint64), ("wait_errors", C.c_uint32)]


HNTL_PLAN_GRAPH = 1


class HNTLError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hntl status {status}: {msg}")
        self.status = status


_lib = None

EXPORTS = {
    "hntl_build": (C.c_int, [C.c_void_p, C.c_uint64, C.c_uint32, C.POINTER(hntl_build_params), C.c_void_p,
                             C.POINTER(C.c_void_p)]),
    "hntl_index_create": (C.c_int, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32] + [C.c_void_p] * 7
                          + [C.c_uint32, C.POINTER(C.c_void_p)]),
    "hntl_index_export": (C.c_int, [C.c_void_p] * 8),
    "hntl_index_append": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.POINTER(hntl_append_params), C.c_void_p,
                                    C.POINTER(C.c_void_p)]),
    "hntl_index_save": (C.c_int, [C.c_void_p, C.c_char_p]),
    "hntl_index_load": (C.c_int, [C.c_char_p, C.POINTER(C.c_void_p)]),
    "hntl_index_export_codes": (C.c_int, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]),
    "hntl_index_info_get": (C.c_int, [C.c_void_p, C.POINTER(hntl_index_info)]),
    "hntl_index_captured": (C.c_int, [C.c_void_p, C.c_void_p]),
    "hntl_index_free": (None, [C.c_void_p]),
    "hntl_search": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.POINTER(hntl_search_params), C.c_void_p,
                              C.c_void_p, C.c_void_p]),
    "hntl_search_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.POINTER(hntl_search_params), C.c_void_p,
                                      C.c_void_p, C.c_void_p]),
    "hntl_search_stages": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.POINTER(hntl_search_params)]
                           + [C.c_void_p] * 13),
    "hntl_profile_read": (C.c_int, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]),
    "hntl_plan_create": (C.c_int, [C.c_void_p, C.POINTER(hntl_search_params), C.c_uint32, C.c_void_p, C.c_uint32,
                                   C.c_void_p, C.POINTER(C.c_void_p)]),
    "hntl_plan_buffers": (C.c_int, [C.c_void_p] + [C.POINTER(C.c_void_p)] * 3),
    "hntl_plan_run": (C.c_int, [C.c_void_p, C.c_uint32, C.c_void_p]),
    "hntl_plan_search": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "hntl_plan_info_get": (C.c_int, [C.c_void_p, C.POINTER(hntl_plan_info)]),
    "hntl_plan_free": (None, [C.c_void_p]),
    "hntl_plan_profile": (C.c_int, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "hntl_tune": (C.c_int, [C.c_void_p, C.POINTER(hntl_search_params), C.c_void_p, C.c_uint32, C.c_char_p,
                            C.POINTER(hntl_schedule), C.POINTER(C.c_float), C.c_void_p]),
    "hntl_schedule_lookup": (C.c_int, [C.c_void_p, C.POINTER(hntl_search_params), C.c_uint32, C.c_char_p,
                                       C.POINTER(hntl_schedule)]),
    "hntl_router_train": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.POINTER(hntl_router_params),
                                    C.c_void_p, C.c_void_p]),
    "hntl_router_set": (C.c_int, [C.c_void_p, C.c_uint32, C.c_uint32] + [C.c_void_p] * 8),
    "hntl_router_export": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)] + [C.c_void_p] * 8),
    "hntl_router_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]),
    "hntl_router_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint32] + [C.c_void_p] * 7
                         + [C.c_void_p]),
    "hntl_knn": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "hntl_last_error": (C.c_char_p, []),
    "hntl_version": (C.c_char_p, []),
}


def lib():
    """The loaded shared library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"HNTL HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build() or paper_2606_08813_amd/build_lib.py)")
        L = C.CDLL(str(LIB_PATH))
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != HNTL_OK:
        raise HNTLError(status, lib().hntl_last_error().decode())


def hntl_last_error() -> str:
    return lib().hntl_last_error().decode()


def hntl_version() -> str:
    return lib().hntl_version().decode()


def _ptr(x):
    """Device or host address of a tensor / ndarray (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        assert x.flags["C_CONTIGUOUS"]
        return x.ctypes.data
    assert x.is_contiguous(), "tensors passed to the library must be contiguous"
    return x.data_ptr()


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _cuda_f32(x, name):
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    return x


@dataclass
class Index:
    """An index handle (freed when garbage collected or by ``hntl_index_free``)."""

    handle: C.c_void_p
    N: int
    d: int
    G: int
    r: int

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.hntl_index_free(self.handle)
            self.handle = None


def hntl_build(X, G: int, r: int, *, kmeans_iters=0, train_per_grain=0, eig_iters=0, codes=("fp32",), seed=0,
               init_centroids=None, stream=None) -> Index:
    """Build an index from X (N x d float32 CUDA tensor)."""
    _cuda_f32(X, "X")
    N, d = X.shape
    mask = 0
    for c in codes:
        mask |= 1 << CODES[c]
    p = hntl_build_params(G, r, kmeans_iters, train_per_grain, eig_iters, mask, seed,
                          _ptr(init_centroids))
    out = C.c_void_p()
    _check(lib().hntl_build(X.data_ptr(), N, d, C.byref(p), _stream(stream), C.byref(out)))
    return Index(out, N, d, G, r)


def hntl_index_create(stored: dict, X, codes=("fp32",)) -> Index:
    """Index from stored-format arrays (numpy host arrays or CUDA tensors).  X = None
    gives an index without raw vectors, which answers Mode A searches only."""
    def prep(a, dt):
        if isinstance(a, np.ndarray):
            return np.ascontiguousarray(a, dtype=dt)
        return a.contiguous()
    cen = prep(stored["centroids"], np.float32)
    bas = prep(stored["basis"], np.float32)
    off = prep(stored["offsets"], np.int64)
    per = prep(stored["perm"], np.int32)
    cod = prep(stored["codes"], np.float32)
    eps = prep(stored["eps"], np.float32)
    Xc = None if X is None else prep(X, np.float32)
    G, d = cen.shape
    r = bas.shape[1]
    N = per.shape[0]
    mask = 0
    for c in codes:
        mask |= 1 << CODES[c]
    out = C.c_void_p()
    _check(lib().hntl_index_create(N, d, G, r, _ptr(cen), _ptr(bas), _ptr(off), _ptr(per), _ptr(cod), _ptr(eps),
                                   None if Xc is None else _ptr(Xc), mask, C.byref(out)))
    return Index(out, N, d, G, r)


def hntl_index_append(base: Index, X, *, split_max=0, eig_iters=0, seed=0, stream=None) -> Index:
    """A new index holding base's rows plus the rows of X (n x d float32, numpy
    or CUDA tensor; ids N .. N + n - 1).  base is left as it was."""
    if isinstance(X, np.ndarray):
        X = np.ascontiguousarray(X, dtype=np.float32)
        n = X.shape[0]
    else:
        import torch
        if X.dtype != torch.float32:
            raise TypeError("X must be float32")
        X = X.contiguous()
        n = X.shape[0]
    if X.ndim != 2 or X.shape[1] != base.d:
        raise ValueError(f"X must be n x {base.d}")
    p = hntl_append_params(split_max, eig_iters, seed)
    out = C.c_void_p()
    _check(lib().hntl_index_append(base.handle, _ptr(X) if n else None, n, C.byref(p), _stream(stream),
                                   C.byref(out)))
    info = hntl_index_info()
    _check(lib().hntl_index_info_get(out, C.byref(info)))
    return Index(out, info.N, info.d, info.G, info.r)


def hntl_index_save(index: Index, path) -> None:
    """Write the index to the directory `path` (.npy arrays + meta.json)."""
    _check(lib().hntl_index_save(index.handle, str(path).encode()))


def hntl_index_load(path) -> Index:
    """Read an index written by hntl_index_save."""
    out = C.c_void_p()
    _check(lib().hntl_index_load(str(path).encode(), C.byref(out)))
    info = hntl_index_info()
    _check(lib().hntl_index_info_get(out, C.byref(info)))
    return Index(out, info.N, info.d, info.G, info.r)


def hntl_index_export(index: Index, with_scales=False) -> dict:
    G, d, r, N = index.G, index.d, index.r, index.N
    o = dict(centroids=np.empty((G, d), np.float32), basis=np.empty((G, r, d), np.float32),
             offsets=np.empty(G + 1, np.int64), perm=np.empty(N, np.int32), codes=np.empty((N, r), np.float32),
             eps=np.empty(N, np.float32))
    sc = np.empty(G, np.float32) if with_scales else None
    _check(lib().hntl_index_export(index.handle, _ptr(o["centroids"]), _ptr(o["basis"]), _ptr(o["offsets"]),
                                   _ptr(o["perm"]), _ptr(o["codes"]), _ptr(o["eps"]), _ptr(sc)))
    if with_scales:
        o["scales"] = sc
    return o


HNTL_EXPORT_RESIDUALS = 0x100


def hntl_index_export_codes(index: Index, codes: str):
    """Reduced-precision codes (N x r bit patterns, grain order) and, for FP8, the
    per-grain scales; for int16, the signed codes and the per-grain inv_g; for
    "int16_residuals", the N uint16 residual codes r_hat and the per-grain rinv_g."""
    if codes == "int16_residuals":
        out = np.empty(index.N, np.uint16)
        sc = np.empty(index.G, np.float32)
        _check(lib().hntl_index_export_codes(index.handle, HNTL_CODES_INT16 | HNTL_EXPORT_RESIDUALS,
                                             out.ctypes.data, sc.ctypes.data))
        return out, sc
    if codes == "int16":
        out = np.empty((index.N, index.r), np.int16)
        sc = np.empty(index.G, np.float32)
        _check(lib().hntl_index_export_codes(index.handle, HNTL_CODES_INT16, out.ctypes.data, sc.ctypes.data))
        return out, sc
    if codes == "bf16":
        out = np.empty((index.N, index.r), np.uint16)
        _check(lib().hntl_index_export_codes(index.handle, HNTL_CODES_BF16, out.ctypes.data, None))
        return out, None
    out = np.empty((index.N, index.r), np.uint8)
    sc = np.empty(index.G, np.float32)
    _check(lib().hntl_index_export_codes(index.handle, HNTL_CODES_FP8_E4M3, out.ctypes.data, sc.ctypes.data))
    return out, sc


def hntl_index_info_get(index: Index) -> dict:
    info = hntl_index_info()
    _check(lib().hntl_index_info_get(index.handle, C.byref(info)))
    return {k: getattr(info, k) for k, _ in info._fields_}


def hntl_index_captured(index: Index) -> np.ndarray:
    out = np.empty(index.G, np.float64)
    _check(lib().hntl_index_captured(index.handle, out.ctypes.data))
    return out


def hntl_index_free(index: Index):
    if index.handle:
        lib().hntl_index_free(index.handle)
        index.handle = None


def _params(P, C_, k, codes, flags, route="centroid", tau=0.0, mass=0.0):
    return hntl_search_params(P, C_, k, CODES[codes] if isinstance(codes, str) else codes, flags,
                              ROUTES[route] if isinstance(route, str) else route, tau, mass)


def hntl_search(index: Index, Q, P: int, C_: int, k: int, codes="fp32", flags=0, out=None, stream=None,
                route="centroid", tau=0.0, mass=0.0):
    """Top-k ids (int32) and squared distances (float32) per query, as CUDA tensors."""
    import torch
    _cuda_f32(Q, "Q")
    nq = Q.shape[0]
    if out is None:
        ids = torch.empty((nq, k), dtype=torch.int32, device=Q.device)
        dist = torch.empty((nq, k), dtype=torch.float32, device=Q.device)
    else:
        ids, dist = out
    sp = _params(P, C_, k, codes, flags, route, tau, mass)
    _check(lib().hntl_search(index.handle, Q.data_ptr(), nq, C.byref(sp), ids.data_ptr(), dist.data_ptr(),
                             _stream(stream)))
    return ids, dist


def hntl_search_noalloc(index: Index, Q, P: int, C_: int, k: int, codes="fp32", flags=0, out=None, stream=None,
                        route="centroid", tau=0.0, mass=0.0):
    """hntl_search with its scratch in the library's static per-GPU array (no device
    allocation by the library); out = (ids, dist) CUDA tensors, else new ones."""
    import torch
    _cuda_f32(Q, "Q")
    nq = Q.shape[0]
    if out is None:
        ids = torch.empty((nq, k), dtype=torch.int32, device=Q.device)
        dist = torch.empty((nq, k), dtype=torch.float32, device=Q.device)
    else:
        ids, dist = out
    sp = _params(P, C_, k, codes, flags, route, tau, mass)
    _check(lib().hntl_search_noalloc(index.handle, Q.data_ptr(), nq, C.byref(sp), ids.data_ptr(), dist.data_ptr(),
                                     _stream(stream)))
    return ids, dist


HNTL_NOALLOC_SCRATCH_BYTES = 64 << 20


def hntl_profile_read():
    """Summed per-stage milliseconds of profiled searches since the last read, their
    count, and the number of eq. 6 scores they computed."""
    ms = np.zeros(len(STAGES), np.float64)
    calls = C.c_uint32(0)
    scored = C.c_uint64(0)
    _check(lib().hntl_profile_read(ms.ctypes.data, len(STAGES), C.byref(calls), C.byref(scored)))
    return dict(zip(STAGES, ms.tolist())), calls.value, scored.value


def hntl_search_stages(index: Index, Q, P: int, C_: int, k: int, codes="fp32", flags=HNTL_FLAG_SYNC,
                       probes_in=None, tangent_in=None, epsq_in=None, pool_in=None, stream=None,
                       route="centroid", tau=0.0, mass=0.0):
    """Run the lifecycle with stage outputs returned and optional stage inputs (CUDA tensors)."""
    import torch
    _cuda_f32(Q, "Q")
    nq = Q.shape[0]
    dev = Q.device
    r = index.r
    o = {}
    if pool_in is None:
        if probes_in is None:
            o["probes"] = torch.full((nq, P), -7, dtype=torch.int32, device=dev)
            o["pdist"] = torch.full((nq, P), float("nan"), dtype=torch.float32, device=dev)
        if tangent_in is None:
            o["zq"] = torch.full((nq, P, r), float("nan"), dtype=torch.float32, device=dev)
            o["epsq"] = torch.full((nq, P), float("nan"), dtype=torch.float32, device=dev)
        o["pool_ids"] = torch.full((nq, C_), -7, dtype=torch.int32, device=dev)
        o["pool_D"] = torch.full((nq, C_), float("nan"), dtype=torch.float32, device=dev)
    o["ids"] = torch.full((nq, k), -7, dtype=torch.int32, device=dev)
    o["dist"] = torch.full((nq, k), float("nan"), dtype=torch.float32, device=dev)
    sp = _params(P, C_, k, codes, flags, route, tau, mass)
    _check(lib().hntl_search_stages(
        index.handle, Q.data_ptr(), nq, C.byref(sp), _ptr(probes_in), _ptr(o.get("probes")), _ptr(o.get("pdist")),
        _ptr(tangent_in), _ptr(epsq_in), _ptr(o.get("zq")), _ptr(o.get("epsq")), _ptr(pool_in),
        _ptr(o.get("pool_ids")), _ptr(o.get("pool_D")), _ptr(o["ids"]), _ptr(o["dist"]), _stream(stream)))
    return o


# ---------------------------------------------------------------- batching form
@dataclass
class Plan:
    """A search plan handle (freed when garbage collected or by ``hntl_plan_free``).
    Keeps its index alive."""

    handle: C.c_void_p
    index: Index
    max_nq: int
    k: int

    def __del__(self):
        if self.handle and _lib is not None:
            _lib.hntl_plan_free(self.handle)
            self.handle = None


def _sched(sched):
    if sched is None:
        return None
    if isinstance(sched, hntl_schedule):
        return sched
    if isinstance(sched, dict):
        return hntl_schedule(sched["qt"], sched["nw"], sched["range"], sched.get("grid", 0), sched.get("passes", 1),
                             sched.get("proj", 0))
    return hntl_schedule(*sched)


def sched_dict(s: hntl_schedule) -> dict:
    return {"qt": s.qt, "nw": s.nw, "range": s.range, "grid": s.grid, "passes": s.passes, "proj": s.proj}


def hntl_plan_create(index: Index, P: int, C_: int, k: int, max_nq: int, codes="fp32", flags=0, sched=None,
                     graph=True, stream=None, route="centroid", tau=0.0, mass=0.0) -> Plan:
    sp = _params(P, C_, k, codes, flags, route, tau, mass)
    sc = _sched(sched)
    h = C.c_void_p()
    _check(lib().hntl_plan_create(index.handle, C.byref(sp), max_nq, C.byref(sc) if sc is not None else None,
                                  HNTL_PLAN_GRAPH if graph else 0, _stream(stream), C.byref(h)))
    return Plan(h, index, max_nq, k)


def hntl_plan_buffers(plan: Plan):
    """Device addresses (ints) of the plan's Q, ids and dist buffers."""
    q, i, d = C.c_void_p(), C.c_void_p(), C.c_void_p()
    _check(lib().hntl_plan_buffers(plan.handle, C.byref(q), C.byref(i), C.byref(d)))
    return q.value, i.value, d.value


def hntl_plan_run(plan: Plan, nq: int, stream=None):
    _check(lib().hntl_plan_run(plan.handle, nq, _stream(stream)))


def hntl_plan_search(plan: Plan, Q, out=None, stream=None):
    """Search the rows of Q (nq <= max_nq) with the plan; returns (ids, dist) CUDA tensors."""
    import torch
    _cuda_f32(Q, "Q")
    nq = Q.shape[0]
    if out is None:
        ids = torch.empty((nq, plan.k), dtype=torch.int32, device=Q.device)
        dist = torch.empty((nq, plan.k), dtype=torch.float32, device=Q.device)
    else:
        ids, dist = out
    _check(lib().hntl_plan_search(plan.handle, Q.data_ptr(), nq, ids.data_ptr(), dist.data_ptr(), _stream(stream)))
    return ids, dist


def hntl_plan_info_get(plan: Plan) -> dict:
    info = hntl_plan_info()
    _check(lib().hntl_plan_info_get(plan.handle, C.byref(info)))
    return {"max_nq": info.max_nq, "sched": sched_dict(info.sched), "graph": bool(info.graph),
            "device_bytes": info.device_bytes, "list_slots": info.list_slots, "wait_errors": info.wait_errors}


PLAN_STAGES = ("route", "bucket", "project", "fused", "rerank")


def hntl_plan_profile(plan: Plan, nq: int, reps=3, stream=None):
    """Mean device ms per plan stage over reps eager runs of the queries already in
    the plan's buffer, and the eq. 6 scores of the last run."""
    ms = np.zeros(len(PLAN_STAGES), np.float64)
    sc = C.c_uint64(0)
    _check(lib().hntl_plan_profile(plan.handle, nq, reps, ms.ctypes.data, C.byref(sc), _stream(stream)))
    return dict(zip(PLAN_STAGES, ms.tolist())), sc.value


def hntl_plan_free(plan: Plan):
    if plan.handle:
        lib().hntl_plan_free(plan.handle)
        plan.handle = None


def hntl_tune(index: Index, Q, P: int, C_: int, k: int, codes="fp32", flags=0, db_path=None, stream=None,
              route="centroid", tau=0.0, mass=0.0):
    """Autotune the fused kernel's schedule on the batch Q; returns (schedule dict, median ms)."""
    _cuda_f32(Q, "Q")
    sp = _params(P, C_, k, codes, flags, route, tau, mass)
    best = hntl_schedule()
    ms = C.c_float(0.0)
    _check(lib().hntl_tune(index.handle, C.byref(sp), Q.data_ptr(), Q.shape[0],
                           str(db_path).encode() if db_path else None, C.byref(best), C.byref(ms), _stream(stream)))
    return sched_dict(best), ms.value


def hntl_schedule_lookup(index: Index, P: int, C_: int, k: int, max_nq: int, db_path, codes="fp32", flags=0,
                         route="centroid", tau=0.0, mass=0.0):
    sp = _params(P, C_, k, codes, flags, route, tau, mass)
    out = hntl_schedule()
    _check(lib().hntl_schedule_lookup(index.handle, C.byref(sp), max_nq, str(db_path).encode(), C.byref(out)))
    return sched_dict(out)


# ----------------------------------------------------------------- learned router
def hntl_router_train(index: Index, Qtrain, targets=None, hidden=(1024, 1024), epochs=1, batch=1024, knn=10,
                      lr=1e-3, seed=0, flags=0, stream=None):
    """Train the index's router on Qtrain (CUDA float32, n x d); returns the per-epoch mean losses."""
    _cuda_f32(Qtrain, "Qtrain")
    rp = hntl_router_params(hidden[0], hidden[1], epochs, batch, knn, flags, lr, seed)
    losses = np.zeros(max(1, epochs), np.float32)
    _check(lib().hntl_router_train(index.handle, Qtrain.data_ptr(), Qtrain.shape[0], _ptr(targets), C.byref(rp),
                                   losses.ctypes.data, _stream(stream)))
    return losses


def hntl_router_set(index: Index, params: dict, mean, std):
    """Import router weights (numpy float32: W1, b1, W2, b2, W3, b3) and the input standardisation."""
    a = {k: np.ascontiguousarray(params[k], dtype=np.float32) for k in ("W1", "b1", "W2", "b2", "W3", "b3")}
    m = np.ascontiguousarray(mean, dtype=np.float32)
    s = np.ascontiguousarray(std, dtype=np.float32)
    _check(lib().hntl_router_set(index.handle, a["W1"].shape[0], a["W2"].shape[0], *(a[k].ctypes.data for k in
                                 ("W1", "b1", "W2", "b2", "W3", "b3")), m.ctypes.data, s.ctypes.data))


def hntl_router_export(index: Index) -> dict:
    h1, h2 = C.c_uint32(), C.c_uint32()
    _check(lib().hntl_router_export(index.handle, C.byref(h1), C.byref(h2), *([None] * 8)))
    d, G = index.d, index.G
    out = {"W1": np.empty((h1.value, d), np.float32), "b1": np.empty(h1.value, np.float32),
           "W2": np.empty((h2.value, h1.value), np.float32), "b2": np.empty(h2.value, np.float32),
           "W3": np.empty((G, h2.value), np.float32), "b3": np.empty(G, np.float32),
           "mean": np.empty(d, np.float32), "std": np.empty(d, np.float32)}
    _check(lib().hntl_router_export(index.handle, None, None, *(out[k].ctypes.data for k in
                                    ("W1", "b1", "W2", "b2", "W3", "b3", "mean", "std"))))
    return out


def hntl_router_forward(index: Index, Q, stream=None):
    import torch
    _cuda_f32(Q, "Q")
    s = torch.empty((Q.shape[0], index.G), dtype=torch.float32, device=Q.device)
    _check(lib().hntl_router_forward(index.handle, Q.data_ptr(), Q.shape[0], s.data_ptr(), _stream(stream)))
    return s


def hntl_router_grad(index: Index, X, targets):
    """Loss and gradients (numpy float32 dict) of the router at its current weights."""
    _cuda_f32(X, "X")
    w = hntl_router_export(index)
    g = {k: np.empty_like(w[k]) for k in ("W1", "b1", "W2", "b2", "W3", "b3")}
    loss = np.zeros(1, np.float32)
    _check(lib().hntl_router_grad(index.handle, X.data_ptr(), X.shape[0], targets.data_ptr(), targets.shape[1],
                                  loss.ctypes.data, *(g[k].ctypes.data for k in ("W1", "b1", "W2", "b2", "W3", "b3")),
                                  _stream(None)))
    return float(loss[0]), g


def hntl_knn(index: Index, Q, k: int, stream=None):
    import torch
    _cuda_f32(Q, "Q")
    ids = torch.empty((Q.shape[0], k), dtype=torch.int32, device=Q.device)
    dist = torch.empty((Q.shape[0], k), dtype=torch.float32, device=Q.device)
    _check(lib().hntl_knn(index.handle, Q.data_ptr(), Q.shape[0], k, ids.data_ptr(), dist.data_ptr(), _stream(stream)))
    return ids, dist
