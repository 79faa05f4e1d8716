// Candidate pool and exact rerank (paper Section 2.1 steps 3-4, Mode B).
//
// One workgroup (4 waves) per query:
//   1. wave 0 merges the P per-grain top-C lists into the query's pool: the C
//      smallest (D, id) over the union of the probed grains.  This is exact
//      because the global top-C is contained in the union of per-grain top-Cs.
//   2. all waves gather the raw float32 rows of the pool (HBM-resident copy of
//      the corpus) and compute ||q - x||^2 by direct differences in FP32,
//      16-byte loads, one row per wave at a time.
//   3. wave 0 keeps the k smallest (distance, id).
#include "hntl_device.h"
#include "hntl_internal.h"

namespace hntl {

namespace {

template <int CAP>
__global__ __launch_bounds__(256) void merge_rerank_kernel(const float* __restrict__ Q, int d, int P, int C, int k,
                                                           int G, int64_t N, const int32_t* __restrict__ probes,
                                                           const uint64_t* __restrict__ part,
                                                           const int32_t* __restrict__ pool_in,
                                                           const float* __restrict__ X, int32_t* __restrict__ pool_out,
                                                           float* __restrict__ pool_D_out, int32_t* __restrict__ ids,
                                                           float* __restrict__ dist, bool vec4) {
  __shared__ uint64_t lst[2 * CAP];
  __shared__ int32_t pool[CAP];
  __shared__ float delta[CAP];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t q = blockIdx.x;

  if (pool_in == nullptr) {
    if (wave == 0) {
      WaveTopC<CAP> L;
      L.init(lst, C);
      const uint64_t* src = part + (size_t)q * P * C;
      for (int s = 0; s < P; ++s) {
        const int g = probes[q * P + s];
        if (g < 0 || g >= G) continue;  // invalid probe: its list was never written
        for (int c0 = 0; c0 < C; c0 += HNTL_WAVE) {
          const int c = c0 + lane;
          const uint64_t key = c < C ? src[(size_t)s * C + c] : KEY_NONE;
          L.offer(key, key != KEY_NONE);
        }
      }
      L.finish();
      for (int c = lane; c < C; c += HNTL_WAVE) {
        const uint64_t key = L.best[c];
        const int32_t id = key == KEY_NONE ? -1 : (int32_t)key_id(key);
        pool[c] = id;
        if (pool_out) pool_out[q * C + c] = id;
        if (pool_D_out) pool_D_out[q * C + c] = key == KEY_NONE ? __builtin_inff() : key_dist(key);
      }
    }
  } else {
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
      const int32_t id = pool_in[q * C + c];
      pool[c] = (id >= 0 && id < N) ? id : -1;  // out-of-range ids count as padding
    }
  }
  __syncthreads();

  const float* qv = Q + (size_t)q * d;
  for (int c = wave; c < C; c += 4) {
    const int32_t id = pool[c];
    if (id < 0) {
      if (lane == 0) delta[c] = __builtin_inff();
      continue;
    }
    const float* x = X + (size_t)id * d;
    float acc = 0.f;
    if (vec4) {
      for (int j = lane * 4; j < d; j += 4 * HNTL_WAVE) {
        const float4 a = *reinterpret_cast<const float4*>(x + j);
        const float4 b = *reinterpret_cast<const float4*>(qv + j);
        const float d0 = a.x - b.x, d1 = a.y - b.y, d2 = a.z - b.z, d3 = a.w - b.w;
        acc = fmaf(d0, d0, acc);
        acc = fmaf(d1, d1, acc);
        acc = fmaf(d2, d2, acc);
        acc = fmaf(d3, d3, acc);
      }
    } else {
      for (int j = lane; j < d; j += HNTL_WAVE) {
        const float df = x[j] - qv[j];
        acc = fmaf(df, df, acc);
      }
    }
    acc = wave_sum(acc);
    if (lane == 0) delta[c] = acc;
  }
  __syncthreads();

  if (wave == 0) {
    WaveTopC<CAP> L;
    L.init(lst, k);
    for (int c0 = 0; c0 < C; c0 += HNTL_WAVE) {
      const int c = c0 + lane;
      const bool ok = c < C && pool[c] >= 0;
      const uint64_t key = ok ? make_key(delta[c], (uint32_t)pool[c]) : KEY_NONE;
      L.offer(key, ok);
    }
    L.finish();
    for (int j = lane; j < k; j += HNTL_WAVE) {
      const uint64_t key = L.best[j];
      ids[q * k + j] = key == KEY_NONE ? -1 : (int32_t)key_id(key);
      dist[q * k + j] = key == KEY_NONE ? __builtin_inff() : key_dist(key);
    }
  }
}

}  // namespace

void launch_merge_rerank(const Index& ix, const float* Q, int64_t nq, int P, int C, int k, const int32_t* probes,
                         const uint64_t* part,
                         const int32_t* pool_in, int32_t* pool_out, float* pool_D_out, int32_t* ids, float* dist,
                         hipStream_t s) {
  if (nq <= 0) return;
  const bool vec4 = (ix.d % 4) == 0 && ((uintptr_t)Q % 16) == 0 && ((uintptr_t)ix.X % 16) == 0;
  const int cap = pow2_at_least(C < 64 ? 64 : C);
  dim3 grid((unsigned)nq);
#define HNTL_MR(CAPV)                                                                                             \
  hipLaunchKernelGGL(merge_rerank_kernel<CAPV>, grid, dim3(256), 0, s, Q, (int)ix.d, P, C, k, (int)ix.G,    \
                     (int64_t)ix.N, probes, part, pool_in, ix.X,                                                  \
                     pool_out, pool_D_out, ids, dist, vec4)
  if (cap == 64)
    HNTL_MR(64);
  else if (cap == 128)
    HNTL_MR(128);
  else
    HNTL_MR(256);
#undef HNTL_MR
  HIP_TRY(hipGetLastError());
}

}  // namespace hntl
