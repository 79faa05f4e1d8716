// Block-SoA tangent scan with per-pair top-C selection (paper eq. 6, Section
// 2.1 step 3, layout of Section 2.4).
//
// For a work item (grain g, up to 16 query pairs probing g) one wave streams
// the grain's blocks: lane b of the wave owns vector b of the block and loads
// its rp coordinates as rp coalesced 256-byte rows plus its eps.  The query
// tangents of the tile sit in LDS and are read as broadcasts.  For every pair
// t of the tile and every member i:
//
//   D_i = sum_j (z_q[t][j] - z_i[j])^2 + eps_q[t] + eps_i
//
// in FP32 as direct differences (the expansion through ||z||^2 loses the
// relative accuracy the candidate ranking needs), then offered to pair t's
// wave top-C list.  Keys carry the grain-order position, whose order inside a
// grain equals original-id order, so (D, position) ranks like (D, id).  The C
// winners are written as (D, original id) keys: part[pair][0..C).
#include "hntl_device.h"
#include "hntl_internal.h"

namespace hntl {

namespace {

constexpr int ITEM = 16;  // pairs per scan work item (tile of LIST_SLOT0 and LIST_REST)
constexpr float PRUNE_SLACK = 1e-4f;  // relative margin on the FP32 lower bound

template <int CAP>
struct ListOf {
  using type = WaveTopC<CAP>;
  static constexpr int lds = 2 * CAP;  // keys of LDS per list
};
template <>
struct ListOf<64> {
  using type = WaveTop64;
  static constexpr int lds = 64;
};

// One workgroup per work item; its 16 / QT waves take QT pairs each and all
// stream the same grain (the repeated code reads hit in L1/L2).
template <int RP, int CAP, int QT>
__global__ __launch_bounds__(64 * (ITEM / QT)) void scan_f32_kernel(
    const float* __restrict__ codes, const float* __restrict__ eps, const int32_t* __restrict__ goff,
    const int32_t* __restrict__ boff, const int32_t* __restrict__ perm, int r, const float* __restrict__ T,
    const float* __restrict__ epsq, int P, int C, const int32_t* __restrict__ ioff,
    const int32_t* __restrict__ lstart, const int32_t* __restrict__ lcount, int G,
    const int32_t* __restrict__ order, uint64_t* __restrict__ part, const uint64_t* __restrict__ bound_lists,
    int prune, const float* __restrict__ blo, const float* __restrict__ bhi, const float* __restrict__ emin,
    unsigned long long* __restrict__ scored) {
  using List = typename ListOf<CAP>::type;
  constexpr int NW = ITEM / QT;
  __shared__ float zq_all[NW][QT][RP];
  __shared__ float eq_all[NW][QT];
  __shared__ uint64_t lists_all[NW][QT][ListOf<CAP>::lds];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  float (*zq)[RP] = zq_all[wave];
  float* eq = eq_all[wave];
  int g;
  if (!item_grain(ioff, G, blockIdx.x, g)) return;
  const int first = (blockIdx.x - ioff[g]) * ITEM;
  const int total = min(ITEM, lcount[g] - first);
  const int sub = wave * QT;
  if (sub >= total) return;  // no workgroup barrier below: idle waves may leave
  const int32_t* pairs = order + lstart[g] + first + sub;
  const int cnt = min(QT, total - sub);
  const int pos0 = goff[g];
  const int ng = goff[g + 1] - pos0;
  const int b0 = boff[g];
  const int nb = boff[g + 1] - b0;

  // stage the query tangents of this wave's pairs (zero beyond r and cnt)
  for (int idx = lane; idx < QT * RP; idx += HNTL_WAVE) {
    const int t = idx / RP, j = idx % RP;
    float v = 0.f;
    if (t < cnt && j < r) v = T[(size_t)pairs[t] * r + j];
    zq[t][j] = v;
  }
  if (lane < QT) eq[lane] = lane < cnt ? epsq[pairs[lane]] : 0.f;
  wave_sync();

  List L[QT];
  bool live[QT];
  int nlive = 0;
  // this lane's coordinate of the grain's code bounding box (lanes >= r idle)
  const float lo = (bound_lists && prune && lane < r) ? blo[(size_t)g * RP + lane] : 0.f;
  const float hi = (bound_lists && prune && lane < r) ? bhi[(size_t)g * RP + lane] : 0.f;
#pragma unroll
  for (int t = 0; t < QT; ++t) {
    uint64_t bnd = KEY_NONE;
    live[t] = t < cnt;
    if (live[t] && bound_lists) {
      const int p = pairs[t];
      bnd = bound_lists[((size_t)(p / P) * P) * C + C - 1];  // C-th key of the query's probe-0 list
      if (prune && bnd != KEY_NONE) {
        // eq. 6 lower bound over the grain: squared distance from z_q to the
        // code bounding box, plus eps_q, plus the grain's smallest eps_i
        const float v = lane < r ? zq[t][lane] : 0.f;
        const float dd = fmaxf(fmaxf(lo - v, v - hi), 0.f);
        const float lb = wave_sum(dd * dd) + eq[t] + emin[g];
        if (lb * (1.f - PRUNE_SLACK) > key_dist(bnd)) {
          live[t] = false;
          if (lane == 0) part[(size_t)p * C] = KEY_NONE;  // empty list
        }
      }
    }
    L[t].init(lists_all[wave][t], C, bnd);
    nlive += live[t] ? 1 : 0;
  }
  wave_sync();
  if (scored && lane == 0 && nlive > 0) atomicAdd(scored, (unsigned long long)nlive * (unsigned long long)ng);

  if (nlive > 0) {
    for (int b = 0; b < nb; ++b) {
      const float* cb = codes + (size_t)(b0 + b) * RP * B;
      float c[RP];
#pragma unroll
      for (int j = 0; j < RP; ++j) c[j] = cb[j * B + lane];
      const float ei = eps[(size_t)(b0 + b) * B + lane];
      const bool valid = b * B + lane < ng;
      const uint32_t pos = (uint32_t)(pos0 + b * B + lane);
#pragma unroll
      for (int t = 0; t < QT; ++t) {
        if (live[t]) {
          float acc = 0.f;
#pragma unroll
          for (int j = 0; j < RP; ++j) {
            const float df = zq[t][j] - c[j];
            acc = fmaf(df, df, acc);
          }
          L[t].offer(make_key(acc + eq[t] + ei, pos), valid);
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < QT; ++t) {
    if (live[t]) {
      L[t].finish();
      uint64_t* out = part + (size_t)pairs[t] * C;
      if constexpr (CAP == 64) {
        const uint64_t k = L[t].best;
        if (lane < C) out[lane] = (k == KEY_NONE) ? KEY_NONE : make_key(key_dist(k), (uint32_t)perm[key_id(k)]);
      } else {
        for (int i = lane; i < C; i += HNTL_WAVE) {
          const uint64_t k = L[t].best[i];
          out[i] = (k == KEY_NONE) ? KEY_NONE : make_key(key_dist(k), (uint32_t)perm[key_id(k)]);
        }
      }
    }
  }
}

// Per grain: minimum and maximum of every code coordinate and the smallest
// eps over its members (one workgroup per grain).
__global__ __launch_bounds__(256) void grain_bounds_kernel(const float* __restrict__ codes,
                                                           const float* __restrict__ eps, int rp, int r,
                                                           const int32_t* __restrict__ goff,
                                                           const int32_t* __restrict__ boff, float* __restrict__ blo,
                                                           float* __restrict__ bhi, float* __restrict__ emin) {
  __shared__ float red[256];
  const int g = blockIdx.x;
  const int b0 = boff[g], nb = boff[g + 1] - b0, ng = goff[g + 1] - goff[g];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // coordinates j = w, w + 4, ...: lanes run over members
  for (int j = w; j < rp; j += 4) {
    float mn = __builtin_inff(), mx = -__builtin_inff();
    for (int b = 0; b < nb; ++b)
      if (b * B + lane < ng) {
        const float v = codes[((size_t)(b0 + b) * rp + j) * B + lane];
        mn = fminf(mn, v);
        mx = fmaxf(mx, v);
      }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      mn = fminf(mn, __shfl_xor(mn, o, 64));
      mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    }
    if (lane == 0) {
      // an empty grain gets an empty box (+inf / -inf); rank padding is exact zero
      blo[(size_t)g * rp + j] = j < r ? mn : 0.f;
      bhi[(size_t)g * rp + j] = j < r ? mx : 0.f;
    }
  }
  float e = __builtin_inff();
  for (int i = threadIdx.x; i < nb * B; i += 256)
    if (i < ng) e = fminf(e, eps[(size_t)b0 * B + i]);
  red[threadIdx.x] = e;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fminf(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) emin[g] = red[0];
}

template <int RP, int CAP>
void launch_rp_cap(const Index& ix, const float* T, const float* epsq, int P, int C, const Buckets& b, int list,
                   uint64_t* part, const uint64_t* bound_lists, bool prune, unsigned long long* scored, hipStream_t s) {
  // unbounded lists (nearest grain) insert often: 4 pairs per wave for more
  // waves in flight; bounded lists insert rarely: 16 pairs share every code load
  constexpr int QT_WIDE = CAP <= 128 ? 16 : 8;
  const dim3 grid((unsigned)b.max_items[list]);
  const ItemLists& Ls = b.lists;
  if (bound_lists == nullptr)
    hipLaunchKernelGGL((scan_f32_kernel<RP, CAP, 4>), grid, dim3(64 * (ITEM / 4)), 0, s, ix.codes, ix.eps, ix.goff,
                       ix.boff, ix.perm, (int)ix.r, T, epsq, P, C, Ls.ioff[list], Ls.lstart[list], Ls.lcount[list],
                       (int)ix.G, b.order, part, bound_lists, prune ? 1 : 0, ix.blo, ix.bhi, ix.emin, scored);
  else
    hipLaunchKernelGGL((scan_f32_kernel<RP, CAP, QT_WIDE>), grid, dim3(64 * (ITEM / QT_WIDE)), 0, s, ix.codes,
                       ix.eps, ix.goff, ix.boff, ix.perm, (int)ix.r, T, epsq, P, C, Ls.ioff[list], Ls.lstart[list],
                       Ls.lcount[list], (int)ix.G, b.order, part, bound_lists, prune ? 1 : 0, ix.blo, ix.bhi, ix.emin, scored);
}

template <int RP>
void launch_rp(const Index& ix, const float* T, const float* epsq, int P, int C, const Buckets& b, int list,
               uint64_t* part,
               const uint64_t* bound_lists, bool prune, unsigned long long* scored, hipStream_t s) {
  const int cap = pow2_at_least(C < 64 ? 64 : C);
  if (cap == 64)
    launch_rp_cap<RP, 64>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s);
  else if (cap == 128)
    launch_rp_cap<RP, 128>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s);
  else
    launch_rp_cap<RP, 256>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s);
}

}  // namespace

void launch_scan(const Index& ix, int codes, const float* T, const float* epsq, int P, int C, const Buckets& b,
                 int list, uint64_t* part, const uint64_t* bound_lists, bool prune, unsigned long long* scored,
                 hipStream_t s) {
  (void)codes;
  if (b.max_items[list] <= 0) return;
  switch (ix.rp) {
    case 8: launch_rp<8>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s); break;
    case 16: launch_rp<16>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s); break;
    case 24: launch_rp<24>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s); break;
    case 32: launch_rp<32>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s); break;
    case 40: launch_rp<40>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s); break;
    case 48: launch_rp<48>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s); break;
    case 56: launch_rp<56>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s); break;
    case 64: launch_rp<64>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s); break;
    default: throw ArgError{HNTL_EUNSUPPORTED, "padded rank must be a multiple of 8 up to 64"};
  }
  HIP_TRY(hipGetLastError());
}

void launch_grain_bounds(Index& ix, hipStream_t s) {
  if (!ix.blo) ix.blo = dev_alloc<float>(&ix, (size_t)ix.G * ix.rp);
  if (!ix.bhi) ix.bhi = dev_alloc<float>(&ix, (size_t)ix.G * ix.rp);
  if (!ix.emin) ix.emin = dev_alloc<float>(&ix, ix.G);
  hipLaunchKernelGGL(grain_bounds_kernel, dim3(ix.G), dim3(256), 0, s, ix.codes, ix.eps, (int)ix.rp, (int)ix.r,
                     ix.goff, ix.boff, ix.blo, ix.bhi, ix.emin);
  HIP_TRY(hipGetLastError());
}

}  // namespace hntl
