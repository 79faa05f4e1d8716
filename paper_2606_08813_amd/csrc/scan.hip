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

constexpr int ITEM = 16;  // pairs per work item (shared with the projection)

template <int RP, int CAP, int QT>
__global__ __launch_bounds__(64) void scan_f32_kernel(const float* __restrict__ codes, const float* __restrict__ eps,
                                                      const int32_t* __restrict__ goff,
                                                      const int32_t* __restrict__ boff,
                                                      const int32_t* __restrict__ perm, int r,
                                                      const float* __restrict__ T, const float* __restrict__ epsq,
                                                      int C, const int32_t* __restrict__ items,
                                                      const int32_t* __restrict__ nitems,
                                                      const int32_t* __restrict__ gcount,
                                                      const int32_t* __restrict__ gstart,
                                                      const int32_t* __restrict__ order,
                                                      uint64_t* __restrict__ part) {
  __shared__ float zq[QT][RP];
  __shared__ float eq[QT];
  __shared__ uint64_t lists[QT][2 * CAP];
  const int lane = lane_id();
  const int item = blockIdx.x;
  if (item >= *nitems) return;
  const int g = items[2 * item], start = items[2 * item + 1];
  const int total = min(ITEM, gcount[g] - start);
  const int pos0 = goff[g];
  const int ng = goff[g + 1] - pos0;
  const int b0 = boff[g];
  const int nb = boff[g + 1] - b0;

  for (int sub = 0; sub < total; sub += QT) {
    const int cnt = min(QT, total - sub);
    // stage the tile's query tangents (zero beyond r and beyond cnt)
    for (int idx = lane; idx < QT * RP; idx += HNTL_WAVE) {
      const int t = idx / RP, j = idx % RP;
      float v = 0.f;
      if (t < cnt && j < r) {
        const int p = order[gstart[g] + start + sub + t];
        v = T[(size_t)p * r + j];
      }
      zq[t][j] = v;
    }
    if (lane < QT) {
      float v = 0.f;
      if (lane < cnt) v = epsq[order[gstart[g] + start + sub + lane]];
      eq[lane] = v;
    }
    WaveTopC<CAP> L[QT];
#pragma unroll
    for (int t = 0; t < QT; ++t) L[t].init(lists[t], C);  // init ends with wave_sync

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
        if (t < cnt) {
          float acc = 0.f;
#pragma unroll
          for (int j = 0; j < RP; ++j) {
            const float df = zq[t][j] - c[j];
            acc = fmaf(df, df, acc);
          }
          const float D = acc + eq[t] + ei;
          L[t].offer(make_key(D, pos), valid);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < QT; ++t) {
      if (t < cnt) {
        L[t].finish();
        const int p = order[gstart[g] + start + sub + t];
        uint64_t* out = part + (size_t)p * C;
        for (int i = lane; i < C; i += HNTL_WAVE) {
          const uint64_t k = L[t].best[i];
          out[i] = (k == KEY_NONE) ? KEY_NONE : make_key(key_dist(k), (uint32_t)perm[key_id(k)]);
        }
      }
    }
    wave_sync();
  }
}

template <int RP, int CAP>
void launch_rp_cap(const Index& ix, const float* T, const float* epsq, int C, const Buckets& b, uint64_t* part,
                   hipStream_t s) {
  constexpr int QT = CAP <= 128 ? 16 : 8;
  hipLaunchKernelGGL((scan_f32_kernel<RP, CAP, QT>), dim3((unsigned)b.max_items), dim3(64), 0, s, ix.codes, ix.eps,
                     ix.goff, ix.boff, ix.perm, (int)ix.r, T, epsq, C, b.items, b.nitems, b.gcount, b.gstart,
                     b.order, part);
}

template <int RP>
void launch_rp(const Index& ix, const float* T, const float* epsq, int C, const Buckets& b, uint64_t* part,
               hipStream_t s) {
  const int cap = pow2_at_least(C < 64 ? 64 : C);
  if (cap == 64)
    launch_rp_cap<RP, 64>(ix, T, epsq, C, b, part, s);
  else if (cap == 128)
    launch_rp_cap<RP, 128>(ix, T, epsq, C, b, part, s);
  else
    launch_rp_cap<RP, 256>(ix, T, epsq, C, b, part, s);
}

}  // namespace

void launch_scan(const Index& ix, int codes, const float* T, const float* epsq, int P, int C, const Buckets& b,
                 uint64_t* part, hipStream_t s) {
  (void)P;
  (void)codes;
  if (b.max_items <= 0) return;
  switch (ix.rp) {
    case 8: launch_rp<8>(ix, T, epsq, C, b, part, s); break;
    case 16: launch_rp<16>(ix, T, epsq, C, b, part, s); break;
    case 24: launch_rp<24>(ix, T, epsq, C, b, part, s); break;
    case 32: launch_rp<32>(ix, T, epsq, C, b, part, s); break;
    case 40: launch_rp<40>(ix, T, epsq, C, b, part, s); break;
    case 48: launch_rp<48>(ix, T, epsq, C, b, part, s); break;
    case 56: launch_rp<56>(ix, T, epsq, C, b, part, s); break;
    case 64: launch_rp<64>(ix, T, epsq, C, b, part, s); break;
    default: throw ArgError{HNTL_EUNSUPPORTED, "padded rank must be a multiple of 8 up to 64"};
  }
  HIP_TRY(hipGetLastError());
}

}  // namespace hntl
