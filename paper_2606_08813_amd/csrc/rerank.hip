// Candidate pool and exact rerank (paper Section 2.1 steps 3-4, Mode B).
//
// One workgroup (4 waves) per query:
//   1. wave 0 merges the P per-grain top-C lists into the query's pool: the C
//      smallest (D, id) over the union of the probed grains.  This is exact
//      because the global top-C is contained in the union of per-grain top-Cs.
//   2. all waves gather the raw float32 rows of the pool (HBM-resident copy of
//      the corpus) and compute ||q - x||^2 by direct differences in FP32:
//      16-byte non-temporal loads (each row is used once), two rows per wave
//      at a time (measured faster than one or four on MI355X).
//   3. wave 0 keeps the k smallest (distance, id).
#include <mutex>

#include "hntl_device.h"
#include "hntl_internal.h"

namespace hntl {

namespace {

template <int CAP, int RR, int JU, bool NT>
__global__ __launch_bounds__(256) void merge_rerank_kernel(const float* __restrict__ Q, int d, int P, int C, int k,
                                                           int G, int64_t N, const int32_t* __restrict__ probes,
                                                           const uint64_t* __restrict__ part,
                                                           const int32_t* __restrict__ pool_in,
                                                           const float* __restrict__ X, int32_t* __restrict__ pool_out,
                                                           float* __restrict__ pool_D_out, int32_t* __restrict__ ids,
                                                           float* __restrict__ dist, bool vec4,
                                                           const int32_t* __restrict__ qoff,
                                                           const float* __restrict__ eps_id, int64_t nrows,
                                                           const int32_t* __restrict__ nlim) {
  __shared__ uint64_t lst[2 * CAP];
  __shared__ int32_t pool[CAP];
  __shared__ float delta[CAP];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  // one workgroup per row; rows from the batch size *nlim on (a plan's device
  // batch size) only get -1 / +inf results
  const int64_t q = blockIdx.x;
  if (q >= nrows) return;
  if (nlim && q >= (int64_t)*nlim) {
    if ((int)threadIdx.x < k) {
      ids[q * k + threadIdx.x] = -1;
      dist[q * k + threadIdx.x] = __builtin_inff();
    }
    return;  // uniform over the workgroup, before any barrier
  }

  if (pool_in == nullptr) {
    if constexpr (CAP == 64) {
      if (wave == 0) {
        WaveTop64 L;
        L.init(lst, C);
        // the query's lists: one per probe, or (grains split into block
        // ranges) the contiguous run qoff[q] .. qoff[q + 1]
        const int64_t l0 = qoff ? qoff[q] : q * P;
        const int nl = qoff ? qoff[q + 1] - qoff[q] : P;
        const uint64_t* src = part + (size_t)l0 * C;
        constexpr int U = 4;  // lists loaded together
        for (int s0 = 0; s0 < nl; s0 += U) {
          uint64_t key[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int s = s0 + u;
            bool ok = s < nl;
            if (ok && !qoff) {
              const int g = probes[q * P + s];
              ok = g >= 0 && g < G;  // invalid probe: its list was never written
            }
            key[u] = (ok && lane < C) ? src[(size_t)s * C + lane] : KEY_NONE;
          }
          // lists hold their keys in any order (a non-empty one with a key
          // first); a pruned list holds one KEY_NONE and nothing else written:
          // skip it whole
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (lane_u64(key[u], 0) != KEY_NONE) L.offer(key[u], key[u] != KEY_NONE);
        }
        L.finish();
        if (lane < C) {
          const int32_t id = L.best == KEY_NONE ? -1 : (int32_t)key_id(L.best);
          pool[lane] = id;
          // Mode A: eq. 6 minus eps_i is the reconstruction distance ||z_q - z_i||^2 + eps_q
          if (eps_id) delta[lane] = id < 0 ? __builtin_inff() : key_dist(L.best) - eps_id[id];
          if (pool_out) pool_out[q * C + lane] = id;
          if (pool_D_out) pool_D_out[q * C + lane] = L.best == KEY_NONE ? __builtin_inff() : key_dist(L.best);
        }
      }
    } else if (wave == 0) {
      WaveTopR<CAP / 64> L;
      L.init(lst, C);
      const int64_t l0 = qoff ? qoff[q] : q * P;
      const int nl = qoff ? qoff[q + 1] - qoff[q] : P;
      const uint64_t* src = part + (size_t)l0 * C;
      constexpr int NR = CAP / 64, U = 2;  // lists loaded together
      for (int s0 = 0; s0 < nl; s0 += U) {
        uint64_t key[U][NR];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int s = s0 + u;
          bool ok = s < nl;
          if (ok && !qoff) {
            const int g = probes[q * P + s];
            ok = g >= 0 && g < G;  // invalid probe: its list was never written
          }
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const int c = r * 64 + lane;
            key[u][r] = (ok && c < C) ? src[(size_t)s * C + c] : KEY_NONE;
          }
        }
        // lists hold their keys in any order, KEY_NONE-padded, a non-empty
        // one with a key first; a pruned list holds one KEY_NONE and nothing
        // else written: skip it whole
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (lane_u64(key[u][0], 0) != KEY_NONE)
#pragma unroll
            for (int r = 0; r < NR; ++r) L.offer(key[u][r], key[u][r] != KEY_NONE);
      }
      L.finish();
#pragma unroll
      for (int rr = 0; rr < CAP / 64; ++rr) {
        const int c = rr * 64 + lane;
        if (c >= C) continue;
        const uint64_t key = L.best[rr];
        const int32_t id = key == KEY_NONE ? -1 : (int32_t)key_id(key);
        pool[c] = id;
        if (eps_id) delta[c] = id < 0 ? __builtin_inff() : key_dist(key) - eps_id[id];
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

  // each wave gathers RR pool rows at a time (Mode B only); a lane issues the
  // loads of JU float4 column groups of all RR rows before using any of them,
  // so every wave keeps RR x JU x 1 KB of row data in flight
  const float* qv = Q + (size_t)q * d;
  for (int c0 = wave * RR; c0 < C && !eps_id; c0 += 4 * RR) {
    int32_t id[RR];
    const float* x[RR];
    float acc[RR];
#pragma unroll
    for (int u = 0; u < RR; ++u) {
      id[u] = c0 + u < C ? pool[c0 + u] : -1;
      x[u] = X + (size_t)(id[u] < 0 ? 0 : id[u]) * d;
      acc[u] = 0.f;
    }
    if (vec4) {
      for (int j0 = lane * 4; j0 < d; j0 += 4 * HNTL_WAVE * JU) {
        float4 b[JU];
        float4 a[RR][JU];
#pragma unroll
        for (int v = 0; v < JU; ++v) {
          const int j = j0 + v * 4 * HNTL_WAVE;
          b[v] = j < d ? *reinterpret_cast<const float4*>(qv + j) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < RR; ++u)
#pragma unroll
          for (int v = 0; v < JU; ++v) {
            const int j = j0 + v * 4 * HNTL_WAVE;
            if (id[u] < 0 || j >= d) {
              a[u][v] = make_float4(0.f, 0.f, 0.f, 0.f);  // masked below; no wait on the query loads
            } else if (NT) {
              const float4* src = reinterpret_cast<const float4*>(x[u] + j);
              a[u][v] = make_float4(__builtin_nontemporal_load(&src->x), __builtin_nontemporal_load(&src->y),
                                    __builtin_nontemporal_load(&src->z), __builtin_nontemporal_load(&src->w));
            } else {
              a[u][v] = *reinterpret_cast<const float4*>(x[u] + j);
            }
          }
#pragma unroll
        for (int u = 0; u < RR; ++u)
#pragma unroll
          for (int v = 0; v < JU; ++v) {
            const bool ok = id[u] >= 0 && j0 + v * 4 * HNTL_WAVE < d;
            const float d0 = ok ? a[u][v].x - b[v].x : 0.f, d1 = ok ? a[u][v].y - b[v].y : 0.f;
            const float d2 = ok ? a[u][v].z - b[v].z : 0.f, d3 = ok ? a[u][v].w - b[v].w : 0.f;
            acc[u] = fmaf(d0, d0, acc[u]);
            acc[u] = fmaf(d1, d1, acc[u]);
            acc[u] = fmaf(d2, d2, acc[u]);
            acc[u] = fmaf(d3, d3, acc[u]);
          }
      }
    } else {
      for (int j = lane; j < d; j += HNTL_WAVE) {
        const float b = qv[j];
#pragma unroll
        for (int u = 0; u < RR; ++u) {
          const float df = id[u] >= 0 ? x[u][j] - b : 0.f;
          acc[u] = fmaf(df, df, acc[u]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < RR; ++u) {
      const float t = wave_sum(acc[u]);
      if (lane == 0 && c0 + u < C) delta[c0 + u] = id[u] >= 0 ? t : __builtin_inff();
    }
  }
  __syncthreads();

  if constexpr (CAP == 64) {
    if (wave == 0) {
      // top k of at most 64 exact distances: one bitonic sort across the lanes
      const bool ok = lane < C && pool[lane] >= 0;
      uint64_t key = ok ? make_key(delta[lane], (uint32_t)pool[lane]) : KEY_NONE;
      key = wave_sort64(key);
      if (lane < k) {
        ids[q * k + lane] = key == KEY_NONE ? -1 : (int32_t)key_id(key);
        dist[q * k + lane] = key == KEY_NONE ? __builtin_inff() : key_dist(key);
      }
    }
  } else if (wave == 0) {
    WaveTopR<CAP / 64> L;
    L.init(lst, k);
    for (int c0 = 0; c0 < C; c0 += HNTL_WAVE) {
      const int c = c0 + lane;
      const bool ok = c < C && pool[c] >= 0;
      const uint64_t key = ok ? make_key(delta[c], (uint32_t)pool[c]) : KEY_NONE;
      L.offer(key, ok);
    }
    L.finish();
#pragma unroll
    for (int rr = 0; rr < CAP / 64; ++rr) {
      const int j = rr * 64 + lane;
      if (j >= k) continue;
      const uint64_t key = L.best[rr];
      ids[q * k + j] = key == KEY_NONE ? -1 : (int32_t)key_id(key);
      dist[q * k + j] = key == KEY_NONE ? __builtin_inff() : key_dist(key);
    }
  }
}

// eps_id[perm[p]] = eps of grain position p (one workgroup per grain).
__global__ __launch_bounds__(256) void eps_by_id_kernel(const float* __restrict__ eps, const int32_t* __restrict__ goff,
                                                        const int32_t* __restrict__ boff,
                                                        const int32_t* __restrict__ perm, float* __restrict__ out) {
  const int g = blockIdx.x;
  const int a = goff[g], n = goff[g + 1] - a, b0 = boff[g];
  for (int m = threadIdx.x; m < n; m += blockDim.x) out[perm[a + m]] = eps[((size_t)b0 + m / B) * B + m % B];
}
std::mutex g_eps_mu;
}  // namespace

void ensure_eps_by_id(Index& ix, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_eps_mu);
  if (ix.eps_id) return;
  float* p = dev_alloc<float>(&ix, ix.N);
  hipLaunchKernelGGL(eps_by_id_kernel, dim3(ix.G), dim3(256), 0, s, ix.eps, ix.goff, ix.boff, ix.perm, p);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  ix.eps_id = p;
}

void launch_merge_rerank(const Index& ix, const float* Q, int64_t nq, int P, int C, int k, const int32_t* probes,
                         const uint64_t* part,
                         const int32_t* pool_in, int32_t* pool_out, float* pool_D_out, int32_t* ids, float* dist,
                         hipStream_t s, const int32_t* qoff, const float* eps_id, const int32_t* nlim) {
  if (nq <= 0) return;
  if (eps_id && pool_in) throw ArgError{HNTL_EUNSUPPORTED, "Mode A answers need the merged pool, not an injected one"};
  if (!eps_id && !ix.X) throw ArgError{HNTL_ESTATE, "this index holds no raw vectors: only Mode A searches"};
  const bool vec4 = (ix.d % 4) == 0 && ((uintptr_t)Q % 16) == 0 && ((uintptr_t)ix.X % 16) == 0;
  const int cap = pow2_at_least(C < 64 ? 64 : C);
  dim3 grid((unsigned)nq);
  // rows of up to 256 floats: one column group per lane and 8 rows per wave (few
  // registers, many waves); longer rows: 3 column groups x 4 rows
#define HNTL_MR(CAPV, RRV, JUV)                                                                                  \
  hipLaunchKernelGGL((merge_rerank_kernel<CAPV, RRV, JUV, true>), grid, dim3(256), 0, s, Q, (int)ix.d, P, C, k,      \
                     (int)ix.G, (int64_t)ix.N, probes, part, pool_in, ix.X, pool_out, pool_D_out, ids, dist, vec4,   \
                     qoff, eps_id, nq, nlim)
  const bool narrow = ix.d <= 4 * HNTL_WAVE;
  if (cap == 64) {
    if (narrow)
      HNTL_MR(64, 8, 1);
    else
      HNTL_MR(64, 4, 3);
  } else if (cap == 128) {
    if (narrow)
      HNTL_MR(128, 8, 1);
    else
      HNTL_MR(128, 4, 3);
  } else {
    if (narrow)
      HNTL_MR(256, 8, 1);
    else
      HNTL_MR(256, 4, 3);
  }
#undef HNTL_MR
  HIP_TRY(hipGetLastError());
}

}  // namespace hntl
