// Grain-major projection kernels (paper Section 2.2, eq. 1-4).  Two item
// sizes over the grain-bucketed pairs:
//   * PT (16) pairs: a single-wave workgroup per item, the basis streamed from
//     L2 (small batches, where most grains hold a pair or two);
//   * PROJECT_TILE pairs: a workgroup of PROJECT_TILE / 16 waves per item; the
//     grain's basis and centroid pass through LDS once per workgroup in depth
//     chunks, and every wave projects its 16 rows from there.
// Both give bit-identical tangents: the MFMA operands and their order per 32
// depths are those of project_wave / project_wave_bf16.
#include <type_traits>

#include "project_impl.h"

namespace hntl {

namespace {

using namespace proj_detail;

template <bool VEC, int NCT>
__global__ __launch_bounds__(64) void project_kernel(
    const float* __restrict__ Q, int d, int P, const float* __restrict__ centroids, const float* __restrict__ basis,
    int r, const int32_t* __restrict__ ioff, const int32_t* __restrict__ lstart, const int32_t* __restrict__ lcount,
    int G, const int32_t* __restrict__ gorder, const int32_t* __restrict__ order, float* __restrict__ T,
    float* __restrict__ epsq) {
  int rank;
  if (!item_grain(ioff, G, blockIdx.x, rank)) return;
  const int g = gorder ? gorder[rank] : rank;
  const int first = (blockIdx.x - ioff[rank]) * PT;  // within the grain's pairs
  const int cnt = min(PT, lcount[g] - first);
  if (cnt <= 0) return;
  project_wave<VEC, NCT>(Q, d, P, centroids, basis, r, g, order + lstart[g] + first, cnt, T, epsq);
}

template <int NCT>
__global__ __launch_bounds__(64) void project_bf16_kernel(
    const float* __restrict__ Q, int d, int P, const float* __restrict__ centroids,
    const uint16_t* __restrict__ basis16, int r, const int32_t* __restrict__ ioff, const int32_t* __restrict__ lstart,
    const int32_t* __restrict__ lcount, int G, const int32_t* __restrict__ gorder, const int32_t* __restrict__ order,
    float* __restrict__ T, float* __restrict__ epsq) {
  int rank;
  if (!item_grain(ioff, G, blockIdx.x, rank)) return;
  const int g = gorder ? gorder[rank] : rank;
  const int first = (blockIdx.x - ioff[rank]) * PT;
  const int cnt = min(PT, lcount[g] - first);
  if (cnt <= 0) return;
  project_wave_bf16<NCT>(Q, d, P, centroids, basis16, r, g, order + lstart[g] + first, cnt, T, epsq);
}

// ---- shared-basis form
constexpr int GK = 64;   // depths per LDS chunk (two 32-depth MFMA groups)
constexpr int XRUN = 4;  // consecutive items kept on one XCD

// Item of workgroup `b`: workgroups are dealt to the 8 XCDs round-robin
// (b % 8), so XCD x's k-th workgroup (k = b / 8) takes item
// ((k / XRUN) 8 + x) XRUN + k % XRUN.  Runs of XRUN consecutive items (the
// items of one grain are consecutive) then share one L2, while whole runs
// still alternate over the XCDs.  The map is a bijection on [0, 8 XRUN m) for a
// grid of 8 XRUN m workgroups.
__device__ __forceinline__ int xcd_item(int b) {
  const int x = b & 7, k = b >> 3;
  return ((k / XRUN) * 8 + x) * XRUN + k % XRUN;
}

// A workgroup of NW waves projects up to 16 NW pairs of one grain.  Per depth
// chunk k0 .. k0 + GK - 1: every thread loads its share of the 16 NCT basis rows
// (zero rows from r on, zeros from d on) and of the centroid into registers,
// then LDS; each wave reads its 16 query rows' slices straight from memory into
// registers (the next chunk's while this chunk's MFMAs run) and forms
// q' = q - mu in FP32.  Two LDS buffers, one barrier per chunk.  Lane (i, kq)
// feeds depth 32 h + 8 kq + e of row / basis row i of chunk half h, as in
// project_wave (FP32: 8 steps of 16x16x4, e = step) and project_wave_bf16
// (one 16x16x32 BF16 step, e = 0..7).  Needs d % 4 == 0 (FP32) or d % 8 == 0
// (BF16) and 16-byte aligned rows.
template <bool BF16, int NCT, int NW>
__global__ __launch_bounds__(64 * NW) void project_lds_kernel(
    const float* __restrict__ Q, int d, int P, const float* __restrict__ centroids, const float* __restrict__ basis,
    const uint16_t* __restrict__ basis16, int r, const int32_t* __restrict__ ioff, const int32_t* __restrict__ lstart,
    const int32_t* __restrict__ lcount, int G, const int32_t* __restrict__ gorder, const int32_t* __restrict__ order,
    float* __restrict__ T, float* __restrict__ epsq) {
  using E = std::conditional_t<BF16, uint16_t, float>;
  constexpr int ROWS = 16 * NCT;
  constexpr int EPV = 16 / (int)sizeof(E);    // elements per 16-byte vector
  constexpr int VPR = GK / EPV;               // vectors per basis row and chunk
  constexpr int RS = GK + EPV;                // padded LDS row stride (elements): rows start 16 B apart in the banks
  constexpr int NB = ROWS * VPR;              // basis vectors per chunk
  constexpr int NV = NB + GK / 4;             // + centroid vectors (FP32)
  constexpr int NT = 64 * NW;
  constexpr int PER = (NV + NT - 1) / NT;     // vectors staged per thread and chunk
  __shared__ __align__(16) E wsh[2][ROWS * RS];
  __shared__ __align__(16) float msh[2][GK];

  const int item = xcd_item((int)blockIdx.x);
  int rank;
  if (!item_grain(ioff, G, item, rank)) return;  // uniform over the workgroup
  const int wave = (int)threadIdx.x >> 6, lane = lane_id();
  const int i = lane & 15, kq = lane >> 4;
  const int g = gorder ? gorder[rank] : rank;
  const int first = (item - ioff[rank]) * (16 * NW) + 16 * wave;  // within the grain's pairs
  const int cnt = __builtin_amdgcn_readfirstlane(min(16, lcount[g] - first));  // <= 0: this wave only stages
  const int32_t* pairs = order + lstart[g] + (first < 0 ? 0 : first);
  const int qrow = i < cnt ? ldg(pairs + i) / P : -1;
  const float* qp = Q + (size_t)(qrow < 0 ? 0 : qrow) * d;
  const float* mu = centroids + (size_t)g * d;
  const E* Wg = BF16 ? (const E*)(basis16 + (size_t)g * r * d) : (const E*)(basis + (size_t)g * r * d);

  using u32x4 = unsigned int __attribute__((ext_vector_type(4)));
  u32x4 st[PER];
  auto stage_load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int v = u * NT + (int)threadIdx.x;
      u32x4 x = {0u, 0u, 0u, 0u};
      if (v < NB) {
        const int row = v / VPR, k = k0 + (v % VPR) * EPV;
        if (row < r && k < d) x = ldg(reinterpret_cast<const u32x4*>(Wg + (size_t)row * d + k));
      } else if (v < NV) {
        const int k = k0 + (v - NB) * 4;
        if (k < d) x = ldg(reinterpret_cast<const u32x4*>(mu + k));
      }
      st[u] = x;
    }
  };
  auto stage_store = [&](int buf) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int v = u * NT + (int)threadIdx.x;
      if (v < NB)
        *reinterpret_cast<u32x4*>(&wsh[buf][(v / VPR) * RS + (v % VPR) * EPV]) = st[u];
      else if (v < NV)
        *reinterpret_cast<u32x4*>(&msh[buf][(v - NB) * 4]) = st[u];
    }
  };
  // the lane's query slices of one chunk: halves h = 0, 1, 8 floats each
  auto q_load = [&](float (&qv)[16], int k0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int kb = k0 + 32 * h + 8 * kq;
      load_ks<true>(*reinterpret_cast<float(*)[8]>(&qv[8 * h]), qp + kb, qrow >= 0 ? d - kb : 0);
    }
  };

  floatx4 acc[NCT];
#pragma unroll
  for (int c = 0; c < NCT; ++c) acc[c] = floatx4{0.f, 0.f, 0.f, 0.f};
  float sq = 0.f;

  auto compute = [&](int buf, const float (&qv)[16], int k0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (k0 + 32 * h >= d) break;  // uniform: no zero-only MFMA group past d
      const int kl = 32 * h + 8 * kq;
      float m[8];
      *reinterpret_cast<floatx4*>(&m[0]) = *reinterpret_cast<const floatx4*>(&msh[buf][kl]);
      *reinterpret_cast<floatx4*>(&m[4]) = *reinterpret_cast<const floatx4*>(&msh[buf][kl + 4]);
      if constexpr (BF16) {
        u32x4 av;
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          const float v0 = qrow >= 0 ? qv[8 * h + e] - m[e] : 0.f;
          const float v1 = qrow >= 0 ? qv[8 * h + e + 1] - m[e + 1] : 0.f;
          sq = fmaf(v0, v0, fmaf(v1, v1, sq));
          av[e / 2] = bf16_rne_bits(v0) | (bf16_rne_bits(v1) << 16);
        }
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
          const u32x4 bv = *reinterpret_cast<const u32x4*>(&wsh[buf][(c * 16 + i) * RS + kl]);
          acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av),
                                                            __builtin_bit_cast(bf16x8, bv), acc[c], 0, 0, 0);
        }
      } else {
        float a[8], bw[NCT][8];
#pragma unroll
        for (int c = 0; c < NCT; ++c) {
          const float* src = reinterpret_cast<const float*>(&wsh[buf][(c * 16 + i) * RS + kl]);
          *reinterpret_cast<floatx4*>(&bw[c][0]) = *reinterpret_cast<const floatx4*>(src);
          *reinterpret_cast<floatx4*>(&bw[c][4]) = *reinterpret_cast<const floatx4*>(src + 4);
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          a[e] = qrow >= 0 ? qv[8 * h + e] - m[e] : 0.f;
          sq = fmaf(a[e], a[e], sq);
        }
#pragma unroll
        for (int e = 0; e < 8; ++e)
#pragma unroll
          for (int c = 0; c < NCT; ++c) acc[c] = mfma16x16x4(a[e], bw[c][e], acc[c]);
      }
    }
  };

  const int nch = (d + GK - 1) / GK;
  float q0[16], q1[16];
  stage_load(0);
  q_load(q0, 0);
  stage_store(0);
  __syncthreads();
  // one chunk: prefetch chunk ch + 1 (LDS share into registers, query slices
  // into `nxt`), multiply chunk ch, publish chunk ch + 1 into the other buffer
  auto step = [&](int ch, const float (&cur)[16], float (&nxt)[16]) {
    const bool more = ch + 1 < nch;
    if (more) {
      stage_load((ch + 1) * GK);
      q_load(nxt, (ch + 1) * GK);
    }
    if (cnt > 0) compute(ch & 1, cur, ch * GK);
    if (more) stage_store((ch + 1) & 1);
    __syncthreads();
  };
  for (int ch = 0; ch < nch; ch += 2) {
    step(ch, q0, q1);
    if (ch + 1 < nch) step(ch + 1, q1, q0);
  }
  if (cnt > 0) project_store<NCT>(acc, sq, r, pairs, cnt, T, epsq);
}

}  // namespace

template <bool BF16, bool VEC, int NCT>
void launch_project_k(const Index& ix, const float* Q, int P, const Buckets& b, float* T, float* epsq,
                      const int32_t* gorder, hipStream_t s) {
  const ItemLists& L = b.lists;
  const int tile = L.tile[LIST_ALL];
  if (tile == PROJECT_TILE && VEC) {
    constexpr int NW = PROJECT_TILE / PT, M = 8 * XRUN;
    const dim3 grid((unsigned)((b.max_items[LIST_ALL] + M - 1) / M * M)), block(64 * NW);
    hipLaunchKernelGGL((project_lds_kernel<BF16, NCT, NW>), grid, block, 0, s, Q, (int)ix.d, P, ix.centroids,
                       ix.basis, ix.basis_bf16, (int)ix.r, L.ioff[LIST_ALL], L.lstart[LIST_ALL], L.lcount[LIST_ALL],
                       (int)ix.G, gorder, b.order, T, epsq);
    return;
  }
  if (tile != PT) throw ArgError{HNTL_EDEVICE, "projection item size must be 16 pairs (or PROJECT_TILE, vector form)"};
  const dim3 grid((unsigned)b.max_items[LIST_ALL]), block(64);
  if constexpr (BF16)
    hipLaunchKernelGGL((project_bf16_kernel<NCT>), grid, block, 0, s, Q, (int)ix.d, P, ix.centroids, ix.basis_bf16,
                       (int)ix.r, L.ioff[LIST_ALL], L.lstart[LIST_ALL], L.lcount[LIST_ALL], (int)ix.G, gorder, b.order,
                       T, epsq);
  else
    hipLaunchKernelGGL((project_kernel<VEC, NCT>), grid, block, 0, s, Q, (int)ix.d, P, ix.centroids, ix.basis,
                       (int)ix.r, L.ioff[LIST_ALL], L.lstart[LIST_ALL], L.lcount[LIST_ALL], (int)ix.G, gorder,
                       b.order, T, epsq);
}

template <bool BF16, bool VEC>
void launch_project_w(const Index& ix, const float* Q, int P, const Buckets& b, float* T, float* epsq,
                      const int32_t* gorder, hipStream_t s) {
  switch ((ix.r + 15) / 16) {
    case 1: launch_project_k<BF16, VEC, 1>(ix, Q, P, b, T, epsq, gorder, s); break;
    case 2: launch_project_k<BF16, VEC, 2>(ix, Q, P, b, T, epsq, gorder, s); break;
    case 3: launch_project_k<BF16, VEC, 3>(ix, Q, P, b, T, epsq, gorder, s); break;
    default: launch_project_k<BF16, VEC, 4>(ix, Q, P, b, T, epsq, gorder, s); break;
  }
}

int project_tile(const Index& ix, const float* Q, bool bf16) {
  const bool vec = (ix.d % (bf16 ? 8 : 4)) == 0 && ((uintptr_t)Q % 16) == 0;
  return vec ? PROJECT_TILE : PT;
}

void launch_project(const Index& ix, const float* Q, int P, const Buckets& b, float* T, float* epsq, bool bf16,
                    const int32_t* gorder, hipStream_t s) {
  if (b.max_items[LIST_ALL] <= 0) return;
  if (bf16) {
    if (!ix.basis_bf16) throw ArgError{HNTL_ESTATE, "BF16 projection needs the BF16 basis (build a reduced-precision code form)"};
    if ((ix.d % 8) != 0 || ((uintptr_t)Q % 16) != 0)
      throw ArgError{HNTL_EUNSUPPORTED, "BF16 projection needs d % 8 == 0 and 16-byte aligned queries"};
    launch_project_w<true, true>(ix, Q, P, b, T, epsq, gorder, s);
  } else if ((ix.d % 4) == 0 && ((uintptr_t)Q % 16) == 0) {
    launch_project_w<false, true>(ix, Q, P, b, T, epsq, gorder, s);
  } else {
    launch_project_w<false, false>(ix, Q, P, b, T, epsq, gorder, s);
  }
  HIP_TRY(hipGetLastError());
}

}  // namespace hntl
