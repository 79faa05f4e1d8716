// Projection of queries onto the local PCA bases of their probed grains
// (paper Section 2.2, eq. 1-4), one wave per 16 (query, grain) pairs:
//
//   q'    = q - mu_g                    (eq. 1, centred first, in FP32)
//   z_q   = W_g^T q'                    (eq. 2, MFMA)
//   eps_q = max(0, ||q'||^2 - ||z_q||^2) (eq. 3-4: since W_g has orthonormal
//                                         columns, ||q' - W_g z_q||^2 equals
//                                         ||q'||^2 - ||z_q||^2)
//
// ||q'||^2 is accumulated by direct squares of the centred values fed to the
// MFMA.  Outputs are pair-major: T[pair][r], epsq[pair], pair = q * P + slot.
// Used by the grain-major projection kernel and by the fused persistent kernel.
#pragma once

#include "hntl_device.h"
#include "hntl_internal.h"

namespace hntl {
namespace proj_detail {

constexpr int PT = 16;    // pairs per wave (rows of one 16x16 MFMA tile)
constexpr int KS = 8;       // consecutive depth values per lane and chunk
constexpr int KC = 4 * KS;  // depth chunk: KS MFMA steps of K = 4

// Loads KS consecutive floats src[0..KS) (zero from `lim` on) into v.
template <bool VEC>
__device__ __forceinline__ void load_ks(float (&v)[KS], const float* __restrict__ src, int lim) {
  if (VEC) {
#pragma unroll
    for (int e = 0; e < KS; e += 4) {
      floatx4 t = {0.f, 0.f, 0.f, 0.f};
      if (e < lim) t = ldg(reinterpret_cast<const floatx4*>(src + e));
      v[e] = t[0];
      v[e + 1] = t[1];
      v[e + 2] = t[2];
      v[e + 3] = t[3];
    }
  } else {
#pragma unroll
    for (int e = 0; e < KS; ++e) v[e] = e < lim ? ldg(src + e) : 0.f;
  }
}

// Epilogue of every projection form.  In: the wave's NCT accumulator tiles
// (MFMA layout: lane l holds rows 4 (l / 16) + t, t < 4, of column c 16 + l % 16)
// and each lane's partial ||q'||^2 of row l % 16 (one of its four K slots).
// Writes z_q (T[pair][0..r)) and eps_q = max(0, ||q'||^2 - ||z_q||^2) of the
// first cnt rows.
template <int NCT>
__device__ __forceinline__ void project_store(const floatx4 (&acc)[NCT], float sq, int r,
                                              const int32_t* __restrict__ pairs, int cnt, float* __restrict__ T,
                                              float* __restrict__ epsq) {
  const int lane = lane_id();
  // ||q'||^2 of row i: the four K slots of the row
  sq += __uint_as_float(lane_xor<16>(__float_as_uint(sq)));
  sq += __uint_as_float(lane_xor<32>(__float_as_uint(sq)));
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int row = 4 * (lane >> 4) + t;
    float zz = 0.f;
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      const int col = c * 16 + (lane & 15);
      if (col < r) zz = fmaf(acc[c][t], acc[c][t], zz);
    }
    zz += __uint_as_float(lane_xor<1>(__float_as_uint(zz)));
    zz += __uint_as_float(lane_xor<2>(__float_as_uint(zz)));
    zz += __uint_as_float(lane_xor<4>(__float_as_uint(zz)));
    zz += __uint_as_float(lane_xor<8>(__float_as_uint(zz)));
    const float q2 = __shfl(sq, row, 64);  // lane `row` holds row `row`'s ||q'||^2
    if (row < cnt) {
      const int p = ldg(pairs + row);
#pragma unroll
      for (int c = 0; c < NCT; ++c) {
        const int col = c * 16 + (lane & 15);
        if (col < r) stg(T + (size_t)p * r + col, acc[c][t]);
      }
      if ((lane & 15) == 0) stg(epsq + p, fmaxf(q2 - zz, 0.f));
    }
  }
}

// The MFMA sums over the four K slots of each
// instruction; lane (i = lane % 16, kq = lane / 16) feeds slot kq with depth
// k0 + KS kq + e in step e, for the A operand (centred query row i) and the B
// operand (basis row c * 16 + i) alike, so each lane reads KS contiguous floats
// per operand and chunk straight from global memory.  NCT = ceil(r / 16)
// column tiles.
// Projects the cnt (<= 16) pairs pairs[0..cnt) of grain g with one wave.
template <bool VEC, int NCT>
__device__ __forceinline__ void project_wave(const float* __restrict__ Q, int d, int P,
                                             const float* __restrict__ centroids, const float* __restrict__ basis,
                                             int r, int g, const int32_t* __restrict__ pairs, int cnt,
                                             float* __restrict__ T, float* __restrict__ epsq) {
  const int lane = lane_id();
  const int i = lane & 15, kq = lane >> 4;
  const int qrow = i < cnt ? ldg(pairs + i) / P : -1;
  const float* mu = centroids + (size_t)g * d;
  const float* Wg = basis + (size_t)g * r * d;
  const float* qp = Q + (size_t)(qrow < 0 ? 0 : qrow) * d;

  floatx4 acc[NCT];
#pragma unroll
  for (int c = 0; c < NCT; ++c) acc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
  float sq = 0.f;

  // two register sets: the next depth chunk loads while this one multiplies
  auto load = [&](float (&a)[KS], float (&m)[KS], float (&b)[NCT][KS], int k0) {
    const int kb = k0 + KS * kq;
    const int lim = d - kb;  // valid floats from kb (may be <= 0: zeros)
    load_ks<VEC>(m, mu + kb, lim);
    load_ks<VEC>(a, qp + kb, qrow >= 0 ? lim : 0);
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      const int j = c * 16 + i;
      load_ks<VEC>(b[c], Wg + (size_t)(j < r ? j : 0) * d + kb, j < r ? lim : 0);
    }
  };
  auto mult = [&](float (&a)[KS], const float (&m)[KS], const float (&b)[NCT][KS]) {
#pragma unroll
    for (int e = 0; e < KS; ++e) {
      a[e] = qrow >= 0 ? a[e] - m[e] : 0.f;
      sq = fmaf(a[e], a[e], sq);
    }
#pragma unroll
    for (int e = 0; e < KS; ++e)
#pragma unroll
      for (int c = 0; c < NCT; ++c) acc[c] = mfma16x16x4(a[e], b[c][e], acc[c]);
  };
  float a0[KS], m0[KS], b0[NCT][KS], a1[KS], m1[KS], b1[NCT][KS];
  load(a0, m0, b0, 0);
  for (int k0 = 0; k0 < d; k0 += 2 * KC) {
    const bool second = k0 + KC < d;
    if (second) load(a1, m1, b1, k0 + KC);
    mult(a0, m0, b0);
    if (second) {
      if (k0 + 2 * KC < d) load(a0, m0, b0, k0 + 2 * KC);
      mult(a1, m1, b1);
    }
  }

  project_store<NCT>(acc, sq, r, pairs, cnt, T, epsq);
}

// BF16 projection (the precision form): q' = q - mu_g is formed in FP32 and
// rounded to BF16 (nearest even), the basis is the BF16 copy, and
// v_mfma_f32_16x16x32_bf16 accumulates the exact BF16 products in FP32.
// ||q'||^2 comes from the unrounded FP32 q', as in the FP32 kernel.  Lane
// (i, kq) feeds depths k0 + 8 kq .. + 7 of row / column i in every MFMA.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t bf16_rne_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

// BF16 form of project_wave (d % 8 == 0, 16-byte aligned query rows).
template <int NCT>
__device__ __forceinline__ void project_wave_bf16(const float* __restrict__ Q, int d, int P,
                                                  const float* __restrict__ centroids,
                                                  const uint16_t* __restrict__ basis16, int r, int g,
                                                  const int32_t* __restrict__ pairs, int cnt, float* __restrict__ T,
                                                  float* __restrict__ epsq) {
  const int lane = lane_id();
  const int i = lane & 15, kq = lane >> 4;
  const int qrow = i < cnt ? ldg(pairs + i) / P : -1;
  const float* mu = centroids + (size_t)g * d;
  const uint16_t* Wg = basis16 + (size_t)g * r * d;
  const float* qp = Q + (size_t)(qrow < 0 ? 0 : qrow) * d;

  floatx4 acc[NCT];
#pragma unroll
  for (int c = 0; c < NCT; ++c) acc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
  float sq = 0.f;
  for (int k0 = 0; k0 < d; k0 += 32) {
    const int kb = k0 + 8 * kq;
    const bool in = kb < d;  // d is a multiple of 8 on this path: whole 8-runs are in or out
    float a[8], m[8];
    load_ks<true>(m, mu + kb, in ? 8 : 0);
    load_ks<true>(a, qp + kb, (in && qrow >= 0) ? 8 : 0);
    u32x4 av;
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      const float v0 = qrow >= 0 ? a[e] - m[e] : 0.f;
      const float v1 = qrow >= 0 ? a[e + 1] - m[e + 1] : 0.f;
      sq = fmaf(v0, v0, fmaf(v1, v1, sq));
      av[e / 2] = bf16_rne_bits(v0) | (bf16_rne_bits(v1) << 16);
    }
#pragma unroll
    for (int c = 0; c < NCT; ++c) {
      const int j = c * 16 + i;
      u32x4 bv = {0u, 0u, 0u, 0u};
      if (j < r && in) bv = ldg(reinterpret_cast<const u32x4*>(Wg + (size_t)j * d + kb));
      acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv),
                                                        acc[c], 0, 0, 0);
    }
  }
  project_store<NCT>(acc, sq, r, pairs, cnt, T, epsq);
}

}  // namespace proj_detail
}  // namespace hntl
