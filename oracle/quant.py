"""Rounding emulation for the reduced-precision forms (oracle).

* BF16: IEEE binary32 with the low 16 mantissa bits removed, rounded to
  nearest with ties to even (RNE), computed on the float32 bit pattern.
* FP8 E4M3 "fn" (OCP 8-bit floating point specification): 1 sign bit,
  4 exponent bits (bias 7), 3 mantissa bits, no infinities; largest finite
  value 448, smallest normal 2^-6, subnormal quantum 2^-9.  Conversion rounds
  to nearest even and saturates to +-448.
* Per-grain FP8 scale: ``s_g = amax_{i in g, j} |z_ij| / 448`` and the stored
  code is ``fp8(z / s_g)``; the decoded value is ``code * s_g``.

These are written from the format definitions, not from any library.
Pins: exhaustive round-trip of every representable value, midpoint ties,
saturation, and the float32 -> bf16 -> float32 identity on bf16 values.
"""
from __future__ import annotations

import numpy as np

FP8_MAX = 448.0


def bf16_round(x) -> np.ndarray:
    """float32 -> nearest bf16 (RNE), returned as float32 values."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).reshape(a.shape)


def bf16_bits(x) -> np.ndarray:
    return (bf16_round(x).view(np.uint32) >> 16).astype(np.uint16)


def fp8_e4m3_round(x) -> np.ndarray:
    """Nearest E4M3fn value (RNE, saturating), as float64."""
    v = np.asarray(x, dtype=np.float64)
    s = np.sign(v)
    a = np.abs(v)
    out = np.zeros_like(a)
    nz = a > 0
    e = np.floor(np.log2(np.where(nz, a, 1.0)))
    e = np.maximum(e, -6.0)
    quantum = np.exp2(e - 3.0)
    q = np.rint(a / quantum) * quantum
    out = np.where(nz, q, 0.0)
    out = np.minimum(out, FP8_MAX)
    return np.copysign(out, v)  # the sign survives rounding to zero


def fp8_e4m3_values() -> np.ndarray:
    """All finite non-negative E4M3fn values, from the bit-field definition."""
    vals = []
    for e in range(16):
        for m in range(8):
            if e == 15 and m == 7:
                continue  # NaN encoding
            if e == 0:
                vals.append(m * 2.0 ** -9)
            else:
                vals.append((1 + m / 8.0) * 2.0 ** (e - 7))
    return np.array(vals)


def fp8_encode_byte(x) -> np.ndarray:
    """E4M3fn bit pattern (uint8) of already-rounded values."""
    v = np.asarray(x, dtype=np.float64)
    # rounding keeps the sign: a negative value that rounds to zero is -0 (0x80)
    sign = np.signbit(v).astype(np.uint8) << 7
    a = np.abs(v)
    out = np.zeros(a.shape, dtype=np.uint8)
    sub = a < 2.0 ** -6
    m_sub = np.rint(a / 2.0 ** -9).astype(np.int64)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0))).astype(np.int64)
    m_norm = np.rint((a / np.exp2(e) - 1.0) * 8).astype(np.int64)
    norm_bits = ((e + 7) << 3) | m_norm
    out = np.where(sub, m_sub, norm_bits).astype(np.uint8)
    return out | sign


def fp8_decode_byte(b) -> np.ndarray:
    b = np.asarray(b, dtype=np.uint8).astype(np.int64)
    s = np.where(b & 0x80, -1.0, 1.0)
    e = (b >> 3) & 0xF
    m = b & 7
    v = np.where(e == 0, m * 2.0 ** -9, (1 + m / 8.0) * np.exp2(e - 7))
    return s * v


def grain_fp8_scales(codes: np.ndarray, offsets: np.ndarray) -> np.ndarray:
    """Per-grain FP32 scale amax/448 computed as a float32 division (1.0 for an
    empty or all-zero grain)."""
    G = len(offsets) - 1
    sc = np.ones(G, dtype=np.float32)
    for g in range(G):
        a, b = int(offsets[g]), int(offsets[g + 1])
        if b > a:
            amax = np.abs(np.asarray(codes[a:b], dtype=np.float32)).max()
            if amax > 0:
                sc[g] = np.float32(amax) / np.float32(FP8_MAX)
    return sc


def fp8_grain_codes(codes: np.ndarray, offsets: np.ndarray):
    """FP8 code values (float64, exact E4M3fn values) of z / s_g with the
    quotient formed in float32, and the scales."""
    z = np.asarray(codes, dtype=np.float32)
    sc = grain_fp8_scales(z, offsets)
    out = np.zeros(z.shape, dtype=np.float64)
    for g in range(len(offsets) - 1):
        a, b = int(offsets[g]), int(offsets[g + 1])
        if b > a:
            out[a:b] = fp8_e4m3_round(z[a:b] / sc[g])
    return out, sc


def decoded_codes(codes: np.ndarray, offsets: np.ndarray, form: str) -> np.ndarray:
    """The code values a scan of the given form reads, as float64:
    fp32 - the stored values; bf16 - their BF16 rounding; fp8 - the float32
    product fl32(e4m3(z / s_g) * s_g)."""
    z = np.asarray(codes, dtype=np.float32)
    if form == "fp32":
        return z.astype(np.float64)
    if form == "bf16":
        return bf16_round(z).astype(np.float64)
    if form == "fp8":
        c, sc = fp8_grain_codes(z, offsets)
        out = np.zeros(z.shape, dtype=np.float32)
        for g in range(len(offsets) - 1):
            a, b = int(offsets[g]), int(offsets[g + 1])
            if b > a:
                out[a:b] = c[a:b].astype(np.float32) * sc[g]
        return out.astype(np.float64)
    raise ValueError(form)


# ------------------------------------------------------------ int16 (eq. 5)
# The paper's own reduced form: z_hat = round(z / Delta) as signed 16-bit and
# r_hat = round(r / Delta_res) as unsigned 16-bit (eq. 5), with the score
# ||z_q - z_i||^2 + r_q + r_i evaluated on the integers.  The paper gives no
# rule for the steps; here they are per grain and make the largest member
# value the largest code:  inv_g = fl32(32767 / amax_g) over |z_ij| (j < r),
# rinv_g = fl32(65535 / max_i eps_i) (1 when the maximum is 0); Delta = 1 / inv,
# Delta_res = 1 / rinv.  A value is quantised as rint(fl32(x) * inv) with the
# product formed in float32 (ties to even), then clamped to the 16-bit range;
# a query coordinate that needs clamping is saturated.  The query's residual
# r_q is one number per (query, grain) and enters unquantised (with the
# members' step it would clamp for every query far from the grain).  The score
# is Delta^2 * S + Delta_res * r_hat_i + r_q, S = sum_j (z_hat_q,j - z_hat_i,j)^2
# exactly (it needs more than 32 bits: up to r * 65534^2).
I16_MAX = 32767
U16_MAX = 65535
ENVELOPE_FRACTION = 0.25  # a grain is pruned for a query when more than this share of its coordinates saturate


def int16_grain_steps(codes: np.ndarray, eps: np.ndarray, offsets: np.ndarray, r: int):
    """Per-grain float32 reciprocal steps (inv_g, rinv_g)."""
    z = np.asarray(codes, dtype=np.float32)
    e = np.asarray(eps, dtype=np.float32)
    G = len(offsets) - 1
    inv = np.ones(G, dtype=np.float32)
    rinv = np.ones(G, dtype=np.float32)
    for g in range(G):
        a, b = int(offsets[g]), int(offsets[g + 1])
        if b > a:
            amax = float(np.abs(z[a:b, :r]).max())
            emax = float(e[a:b].max())
            if amax > 0:
                inv[g] = np.float32(I16_MAX / np.float64(np.float32(amax)))
            if emax > 0:
                rinv[g] = np.float32(U16_MAX / np.float64(np.float32(emax)))
    return inv, rinv


def int16_quantize(x, inv, lim: int, signed: bool = True):
    """rint(fl32(x) * fl32(inv)) (float32 product, ties to even) clamped to
    [-lim, lim] (signed) or [0, lim]; returns (int64 values, saturated mask)."""
    p = np.asarray(x, dtype=np.float32) * np.float32(inv)
    q = np.rint(p.astype(np.float64))
    lo = -lim if signed else 0
    sat = (q > lim) | (q < lo)
    return np.clip(q, lo, lim).astype(np.int64), sat


def int16_grain_codes(codes: np.ndarray, eps: np.ndarray, offsets: np.ndarray, r: int):
    """Integer codes (N x r) and residuals (N) in grain order, and the steps."""
    inv, rinv = int16_grain_steps(codes, eps, offsets, r)
    z = np.asarray(codes, dtype=np.float32)[:, :r]
    e = np.asarray(eps, dtype=np.float32)
    zh = np.zeros(z.shape, dtype=np.int64)
    rh = np.zeros(len(e), dtype=np.int64)
    for g in range(len(offsets) - 1):
        a, b = int(offsets[g]), int(offsets[g + 1])
        if b > a:
            zh[a:b], _ = int16_quantize(z[a:b], inv[g], I16_MAX)
            rh[a:b], _ = int16_quantize(e[a:b], rinv[g], U16_MAX, signed=False)
    return zh, rh, inv, rinv


def int16_scores(zq, epsq, zh, rh, inv, rinv):
    """The integer-form score of members (zh, rh) of one grain for one query:
    (scores float64, envelope-pruned flag)."""
    r = zh.shape[1]
    zq_h, sat = int16_quantize(np.asarray(zq)[:r], inv, I16_MAX)
    if sat.sum() > ENVELOPE_FRACTION * r:
        return None, True
    S = ((zq_h[None, :] - zh) ** 2).sum(axis=1)  # exact int64
    step = 1.0 / np.float64(inv)
    rstep = 1.0 / np.float64(rinv)
    eq = np.float64(np.float32(epsq))
    return S.astype(np.float64) * step * step + rh.astype(np.float64) * rstep + eq, False
