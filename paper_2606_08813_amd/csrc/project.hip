// Projection of queries onto the local PCA bases of their probed grains
// (paper Section 2.2, eq. 1-4), grain-major:
//
//   q'    = q - mu_g                    (eq. 1, centred first, in FP32)
//   z_q   = W_g^T q'                    (eq. 2, FP32 MFMA 16x16x4)
//   eps_q = max(0, ||q'||^2 - ||z_q||^2) (eq. 3-4: since W_g has orthonormal
//                                         columns, ||q' - W_g z_q||^2 equals
//                                         ||q'||^2 - ||z_q||^2)
//
// One wave handles one work item: up to 16 pairs of one grain.  The centred
// query rows (16 x 64 chunk) and the basis rows (r x 64 chunk) are staged in
// LDS and fed to the MFMA; ||q'||^2 is accumulated by direct squares while
// staging.  Outputs are pair-major: T[pair][r], epsq[pair], pair = q * P + slot.
#include "hntl_device.h"
#include "hntl_internal.h"

namespace hntl {

namespace {

constexpr int PT = 16;     // pairs per work item
constexpr int KC = 64;     // depth chunk
constexpr int LDK = KC + 1;

__global__ __launch_bounds__(128) void project_kernel(const float* __restrict__ Q, int d, int P,
                                                      const float* __restrict__ centroids,
                                                      const float* __restrict__ basis, int r,
                                                      const int32_t* __restrict__ items,
                                                      const int32_t* __restrict__ nitems,
                                                      const int32_t* __restrict__ gcount,
                                                      const int32_t* __restrict__ gstart,
                                                      const int32_t* __restrict__ order, float* __restrict__ T,
                                                      float* __restrict__ epsq) {
  extern __shared__ float smem[];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int item = blockIdx.x * 2 + wave;
  if (item >= *nitems) return;
  const int g = items[2 * item], start = items[2 * item + 1];
  const int cnt = min(PT, gcount[g] - start);
  const int nct = (r + 15) >> 4;  // column tiles of 16
  float* As = smem + wave * ((PT + 64) * LDK);
  float* Bs = As + PT * LDK;

  int qrow[PT];
#pragma unroll
  for (int i = 0; i < PT; ++i) {
    const int p = i < cnt ? order[gstart[g] + start + i] : 0;
    qrow[i] = p / P;
  }
  const float* mu = centroids + (size_t)g * d;
  const float* Wg = basis + (size_t)g * r * d;

  floatx4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
  float sq[PT];
#pragma unroll
  for (int i = 0; i < PT; ++i) sq[i] = 0.f;

  for (int k0 = 0; k0 < d; k0 += KC) {
    const int kk = k0 + lane;
    const bool in = kk < d;
    const float m = in ? mu[kk] : 0.f;
    float qv[PT];
#pragma unroll
    for (int i = 0; i < PT; ++i) qv[i] = (i < cnt && in) ? Q[(size_t)qrow[i] * d + kk] : 0.f;
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const float v = (i < cnt && in) ? qv[i] - m : 0.f;
      As[i * LDK + lane] = v;
      sq[i] = fmaf(v, v, sq[i]);
    }
    // basis rows: issue every load of the chunk before the LDS stores
    float wv[64];
#pragma unroll
    for (int j = 0; j < 64; ++j) wv[j] = (j < r && in) ? Wg[(size_t)j * d + kk] : 0.f;
#pragma unroll
    for (int j = 0; j < 64; ++j)
      if (j < nct * 16) Bs[j * LDK + lane] = wv[j];
    wave_sync();
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int kr = 4 * s + (lane >> 4);
      const float a = As[(lane & 15) * LDK + kr];
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (c < nct) acc[c] = mfma16x16x4(a, Bs[(c * 16 + (lane & 15)) * LDK + kr], acc[c]);
    }
    wave_sync();
  }

  // ||q'||^2 per row, ||z||^2 per row
  float qn[PT];
#pragma unroll
  for (int i = 0; i < PT; ++i) qn[i] = wave_sum(sq[i]);
  float zn[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float t = 0.f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int col = c * 16 + (lane & 15);
      if (c < nct && col < r) t = fmaf(acc[c][i], acc[c][i], t);
    }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) t += __shfl_xor(t, o, 64);
    zn[i] = t;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = 4 * (lane >> 4) + i;
    if (row < cnt) {
      const int p = order[gstart[g] + start + row];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int col = c * 16 + (lane & 15);
        if (c < nct && col < r) T[(size_t)p * r + col] = acc[c][i];
      }
      if ((lane & 15) == 0) {
        float q2 = 0.f;
#pragma unroll
        for (int j = 0; j < PT; ++j)
          if (j == row) q2 = qn[j];
        epsq[p] = fmaxf(q2 - zn[i], 0.f);
      }
    }
  }
}

}  // namespace

void launch_project(const Index& ix, const float* Q, int P, const Buckets& b, float* T, float* epsq,
                    hipStream_t s) {
  const size_t shmem = 2 * (PT + 64) * LDK * sizeof(float);
  const unsigned grid = (unsigned)((b.max_items + 1) / 2);
  if (grid == 0) return;
  hipLaunchKernelGGL(project_kernel, dim3(grid), dim3(128), shmem, s, Q, (int)ix.d, P, ix.centroids, ix.basis,
                     (int)ix.r, b.items, b.nitems, b.gcount, b.gstart, b.order, T, epsq);
  HIP_TRY(hipGetLastError());
}

}  // namespace hntl
