"""Learned router: MLP forward/backward, softmax cross-entropy, Adam (oracle).

The paper routes by centroid distance (Section 2.3) and lists learned
partitioning as future work (Section 4).  The learned router maps a query to
one score per grain; its top-P grains replace centroid routing.

Network (float64 here; the GPU runs BF16 GEMM inputs with FP32 accumulation,
which ``bf16=True`` emulates by rounding at the same points):

* input standardisation ``xh = (x - mean) / std`` (training-set statistics)
* ``h1 = gelu(W1 xh + b1)``, ``h2 = gelu(W2 h1 + b2)``, ``s = W3 h2 + b3``
* GELU is the exact form ``0.5 x (1 + erf(x / sqrt(2)))`` (Hendrycks & Gimpel)
* loss: softmax cross-entropy against a target distribution y over grains,
  ``L = mean_b [ -sum_g y_bg log softmax(s_b)_g ]``
* Adam (Kingma & Ba) with bias correction on float64 master weights.

Training targets: the grain distribution of a query's exact top-10
neighbours (the fraction of them that lies in each grain).

Rounding points when ``bf16=True``: the standardised input, every weight
matrix, and every activation that enters a GEMM are rounded to BF16 (RNE);
GEMMs accumulate in float64 (the GPU in float32); bias, GELU, softmax stay in
float64.  In the backward pass the upstream gradient entering each GEMM is
rounded to BF16 as well.

Pins: central finite differences of the loss on a tiny network in float64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from .quant import bf16_round


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def _r(a, on):
    return bf16_round(a).astype(np.float64) if on else np.asarray(a, dtype=np.float64)


def init_params(dims, seed: int):
    """He-style uniform init for each layer; biases zero.  dims = (d, h1, h2, G)."""
    rng = np.random.default_rng(seed)
    params = {}
    for li in range(3):
        fan_in, fan_out = dims[li], dims[li + 1]
        bound = math.sqrt(6.0 / fan_in) if li < 2 else math.sqrt(3.0 / fan_in)
        params[f"W{li + 1}"] = rng.uniform(-bound, bound, size=(fan_out, fan_in))
        params[f"b{li + 1}"] = np.zeros(fan_out)
    return params


def forward(params, x, mean, std, bf16=False):
    xh = _r((np.asarray(x, dtype=np.float64) - mean) / std, bf16)
    W1, W2, W3 = (_r(params[k], bf16) for k in ("W1", "W2", "W3"))
    a1 = xh @ W1.T + params["b1"]
    h1 = gelu(a1)
    h1r = _r(h1, bf16)
    a2 = h1r @ W2.T + params["b2"]
    h2 = gelu(a2)
    h2r = _r(h2, bf16)
    s = h2r @ W3.T + params["b3"]
    cache = dict(xh=xh, a1=a1, h1r=h1r, a2=a2, h2r=h2r, W1=W1, W2=W2, W3=W3)
    return s, cache


def softmax(s):
    m = s.max(axis=1, keepdims=True)
    e = np.exp(s - m)
    return e / e.sum(axis=1, keepdims=True)


def loss_and_dlogits(s, y):
    """Mean softmax cross-entropy and its gradient w.r.t. the logits."""
    p = softmax(s)
    B = s.shape[0]
    logp = s - s.max(axis=1, keepdims=True)
    logp = logp - np.log(np.exp(logp).sum(axis=1, keepdims=True))
    loss = float(-(y * logp).sum() / B)
    return loss, (p * y.sum(axis=1, keepdims=True) - y) / B


def backward(params, cache, ds, bf16=False):
    g = {}
    dsr = _r(ds, bf16)
    g["W3"] = dsr.T @ cache["h2r"]
    g["b3"] = ds.sum(axis=0)
    dh2 = dsr @ cache["W3"]
    da2 = dh2 * gelu_grad(cache["a2"])
    da2r = _r(da2, bf16)
    g["W2"] = da2r.T @ cache["h1r"]
    g["b2"] = da2.sum(axis=0)
    dh1 = da2r @ cache["W2"]
    da1 = dh1 * gelu_grad(cache["a1"])
    da1r = _r(da1, bf16)
    g["W1"] = da1r.T @ cache["xh"]
    g["b1"] = da1.sum(axis=0)
    return g


def adam_step(params, grads, state, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1).  state holds m and v per tensor."""
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = b1 * m + (1 - b1) * grads[k]
        v[...] = b2 * v + (1 - b2) * grads[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params


def grain_targets(gt_ids: np.ndarray, labels_of_row: np.ndarray, G: int) -> np.ndarray:
    """Target distribution: fraction of each query's exact neighbours in each grain."""
    nq, k = gt_ids.shape
    y = np.zeros((nq, G))
    for i in range(nq):
        for j in gt_ids[i]:
            y[i, labels_of_row[j]] += 1.0 / k
    return y


def route_learned(params, x, mean, std, P, bf16=True):
    s, _ = forward(params, x, mean, std, bf16)
    G = s.shape[1]
    order = np.lexsort((np.broadcast_to(np.arange(G), s.shape), -s), axis=1)[:, :P]
    return order, np.take_along_axis(s, order, 1)


def mass_cut(scores, probes, mass):
    """Probability-mass probe budget: probes (rows x P, descending score) are
    kept up to and including the first slot at which the cumulative softmax
    probability (over all G scores of the row) reaches `mass`; later slots
    become -1.  mass <= 0 or >= 1 keeps every slot."""
    probes = np.array(probes, copy=True)
    if mass <= 0.0 or mass >= 1.0:
        return probes
    s = np.asarray(scores, dtype=np.float64)
    for i in range(len(s)):
        m = s[i].max()
        z = np.exp(s[i] - m).sum()
        c = 0.0
        for j in range(probes.shape[1]):
            c += np.exp(s[i, probes[i, j]] - m) / z
            if c >= mass:
                probes[i, j + 1:] = -1
                break
    return probes


def route_learned_mass(params, x, mean, std, P, mass, bf16=True):
    """Learned routing under a probability-mass budget (mass_cut of the top-P)."""
    s, _ = forward(params, x, mean, std, bf16)
    probes, _ = route_learned(params, x, mean, std, P, bf16)
    return mass_cut(s, probes, mass), s


def route_with_fallback(params, x, mean, std, centroids, P, tau, bf16=True):
    """Learned routing with the centroid fallback: a query whose largest softmax
    probability over the grains is below tau takes the P nearest centroids
    (ties to the lower grain) instead of the router's top-P."""
    from .search import route
    s, _ = forward(params, x, mean, std, bf16)
    pmax = 1.0 / np.exp(s - s.max(axis=1, keepdims=True)).sum(axis=1)
    probes, _ = route_learned(params, x, mean, std, P, bf16)
    low = pmax < tau
    if low.any():
        cp, _ = route(np.asarray(x)[low], centroids, P)
        probes = probes.copy()
        probes[low] = cp
    return probes, pmax
