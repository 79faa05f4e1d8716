"""Shared helpers of the GPU tests: device checks and oracle reference callables."""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_08813_amd import hntl
    hntl.lib()  # raises when a GPU is present but the HIP library is missing
    return torch


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def exact_dist_fn(X, Q):
    """oracle_dist_of(row, ids): exact squared L2 in float64 by direct differences."""
    def f(i, ids):
        return ((X[np.asarray(ids)].astype(np.float64) - Q[i].astype(np.float64)[None, :]) ** 2).sum(1)
    return f


def centroid_dist_fn(M, Q):
    def f(i, ids):
        return ((M[np.asarray(ids)].astype(np.float64) - Q[i].astype(np.float64)[None, :]) ** 2).sum(1)
    return f


def scan_dist_fn(stored, zq, epsq, probes):
    """eq. 6 score of arbitrary ids of query i from the oracle's tangents."""
    from oracle import search as osr
    cache = {}

    def f(i, ids):
        if i not in cache:
            m = {}
            for s in range(probes.shape[1]):
                g = int(probes[i, s])
                if g < 0:
                    continue
                gi, gd = osr.grain_scores(zq[i, s], epsq[i, s], g, stored)
                m.update(zip(gi.tolist(), gd.tolist()))
            cache.clear()
            cache[i] = m
        return np.array([cache[i].get(int(x), np.inf) for x in ids])
    return f
