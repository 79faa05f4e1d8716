// Block-SoA tangent scan kernels (included by one translation unit per code
// form).  Block-SoA tangent scan with per-pair top-C selection (paper eq. 6, Section
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
#pragma once

#include "hntl_device.h"
#include "hntl_internal.h"

namespace hntl {
namespace scan_detail {

constexpr int ITEM = 16;  // pairs per scan work item (tile of LIST_SLOT0 and LIST_REST)
constexpr float PRUNE_SLACK = 1e-4f;  // relative margin on the FP32 lower bound

template <int CAP>
struct ListOf {
  using type = WaveTopR<CAP / 64>;  // the sorted list in registers, NR = CAP / 64 keys per lane
  static constexpr int lds = 64;    // keys of LDS per list (the arrival stage)
};

// One workgroup per work item; its 16 / QT waves take QT pairs each and all
// stream the same grain (the repeated code reads hit in L1/L2).
// CT: code form (0 FP32, 1 BF16 packed in pairs, 2 FP8 E4M3 packed in fours
// with a per-grain scale; the decoded value of an FP8 code is fl32(code * s_g)).
// 32-bit words per lane and block of a code form: one FP32 code, two BF16 or
// int16 codes, four FP8 codes per word.
template <int RP, int CT>
struct RawWords {
  static constexpr int n = CT == 0 ? RP : (CT == 2 ? RP / 4 : RP / 2);
};

// The lane's words of block `blk` (word j of the block is row j of B words).
template <int RP, int CT, int RW = RawWords<RP, CT>::n>
__device__ __forceinline__ void load_raw(uint32_t (&w)[RW], const void* __restrict__ codes, size_t blk, int lane) {
  const uint32_t* wb = reinterpret_cast<const uint32_t*>(codes) + blk * RW * B;
#pragma unroll
  for (int j = 0; j < RW; ++j) w[j] = ldg(wb + j * B + lane);
}

// The decoded code values of a lane's words.
template <int RP, int CT, int RW = RawWords<RP, CT>::n>
__device__ __forceinline__ void decode_raw(float (&c)[RP], const uint32_t (&w)[RW], float s) {
  if constexpr (CT == 0) {
#pragma unroll
    for (int j = 0; j < RP; ++j) c[j] = __uint_as_float(w[j]);
  } else if constexpr (CT == 1) {
#pragma unroll
    for (int j = 0; j < RP / 2; ++j) {
      c[2 * j] = __uint_as_float(w[j] << 16);
      c[2 * j + 1] = __uint_as_float(w[j] & 0xFFFF0000u);
    }
  } else if constexpr (CT == 3) {
    // int16 codes as exact float integers
#pragma unroll
    for (int j = 0; j < RP / 2; ++j) {
      c[2 * j] = (float)(int16_t)(w[j] & 0xFFFFu);
      c[2 * j + 1] = (float)(int16_t)(w[j] >> 16);
    }
  } else {
#pragma unroll
    for (int j = 0; j < RP / 4; ++j) {
      const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[j], false);  // bytes 0, 1
      const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[j], true);   // bytes 2, 3
      c[4 * j] = lo[0] * s;
      c[4 * j + 1] = lo[1] * s;
      c[4 * j + 2] = hi[0] * s;
      c[4 * j + 3] = hi[1] * s;
    }
  }
}

template <int RP, int CT>
__device__ __forceinline__ void load_block(float (&c)[RP], const void* __restrict__ codes, size_t blk, int lane,
                                           float s) {
  uint32_t w[RawWords<RP, CT>::n];
  load_raw<RP, CT>(w, codes, blk, lane);
  decode_raw<RP, CT>(c, w, s);
}

// int16 form: S = sum_j (q_j - c_j)^2 over integers, evaluated exactly as
// |q|^2 + |c|^2 - 2 q.c with packed 16-bit dot products (two products and a
// 32-bit accumulation per instruction, no decoding of the code words).  Query
// coordinates and codes lie in [-32767, 32767] and there are at most 64 of
// them.  |c|^2: the dot of one word with itself is at most 2 * 32767^2 < 2^31;
// widened to float64 and summed (integers below 2^37) it is exact.  q.c: each pair's
// query is split once as q = 256 qh + ql (qh = q >> 8 in [-128, 127],
// ql = q & 255), so the partial dots qh.c (|.| < 64 * 128 * 32767 < 2^29) and
// ql.c (< 64 * 255 * 32767 < 2^30) accumulate exactly in 32 bits, and
// q.c = 256 qh.c + ql.c.  Every float64 step holds integers below 2^53, so S
// is the same integer as the sum of squared differences.
typedef short short2v __attribute__((ext_vector_type(2)));
typedef uint32_t uint32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int sdot2w(uint32_t a, uint32_t b, int acc) {
  return __builtin_amdgcn_sdot2(__builtin_bit_cast(short2v, a), __builtin_bit_cast(short2v, b), acc, false);
}

// |c|^2 of a lane's code words (RW even).  Two words' self-dots start from
// -2^31: -2^31 + s0 + s1 stays inside int32 for s0, s1 <= 2 * 32767^2, so one
// float64 widening and add serve two words; the offsets are added back at the
// end (all exact).
template <int RW>
__device__ __forceinline__ double i16_sq_norm(const uint32_t (&w)[RW]) {
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < RW; j += 2) s += (double)sdot2w(w[j + 1], w[j + 1], sdot2w(w[j], w[j], INT32_MIN));
  return s + (double)(RW / 2) * 2147483648.0;
}

// q.c from a pair's split query words (qh in words [0, RW), ql in [RW, 2 RW),
// 16-byte aligned, RW a multiple of 4) and a lane's code words
template <int RW>
__device__ __forceinline__ double i16_cross(const uint32_t* __restrict__ qw, const uint32_t (&w)[RW]) {
  const uint32x4* h4 = reinterpret_cast<const uint32x4*>(qw);
  const uint32x4* l4 = reinterpret_cast<const uint32x4*>(qw + RW);
  int a = 0, b = 0;
#pragma unroll
  for (int k = 0; k < RW / 4; ++k) {
    const uint32x4 h = h4[k], l = l4[k];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      a = sdot2w(h[e], w[4 * k + e], a);
      b = sdot2w(l[e], w[4 * k + e], b);
    }
  }
  return fma((double)a, 256.0, (double)b);
}

// Rewrites a pair's quantised query (RP exact float integers, zero beyond r)
// in place as its split words and returns |q|^2 (one wave, all lanes).
template <int RP>
__device__ __forceinline__ double i16_split_query(float* __restrict__ zrow, int lane) {
  constexpr int RW = RP / 2;
  const float v = lane < RP ? zrow[lane] : 0.f;
  const double qn = wave_sum_d((double)v * (double)v);
  uint32_t hw = 0, lw = 0;
  if (lane < RW) {
    const int i0 = (int)zrow[2 * lane], i1 = (int)zrow[2 * lane + 1];
    hw = ((uint32_t)(i0 >> 8) & 0xFFFFu) | ((uint32_t)(i1 >> 8) << 16);
    lw = (uint32_t)(i0 & 255) | ((uint32_t)(i1 & 255) << 16);
  }
  wave_sync();  // every lane's reads of the row precede the writes
  uint32_t* qw = reinterpret_cast<uint32_t*>(zrow);
  if (lane < RW) {
    qw[lane] = hw;
    qw[RW + lane] = lw;
  }
  // the sum is the same in every lane: keep it in scalar registers
  const uint64_t u = (uint64_t)__double_as_longlong(qn);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// int16 code of a float code value (float32 product, ties to even, clamped),
// as the index's packing computes it.
__device__ __forceinline__ float q16f(float x, float inv, float lo, float hi) {
  return fminf(fmaxf(rintf(x * inv), lo), hi);
}

template <int RP, int CAP, int QT, int CT>
__global__ __launch_bounds__(64 * (ITEM / QT)) void scan_f32_kernel(
    const void* __restrict__ codes, const float* __restrict__ scales, const float* __restrict__ eps, const int32_t* __restrict__ goff,
    const int32_t* __restrict__ boff, const int32_t* __restrict__ perm, int r, const float* __restrict__ T,
    const float* __restrict__ epsq, int P, int C, const int32_t* __restrict__ ioff,
    const int32_t* __restrict__ lstart, const int32_t* __restrict__ lcount, int G,
    const int32_t* __restrict__ order, uint64_t* __restrict__ part, const uint64_t* __restrict__ bound_lists,
    int prune, const float* __restrict__ blo, const float* __restrict__ bhi, const float* __restrict__ emin,
    unsigned long long* __restrict__ scored) {
  using List = typename ListOf<CAP>::type;
  constexpr int NW = ITEM / QT;
  __shared__ __align__(16) float zq_all[NW][QT][RP];
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
  // int16 form: the query coordinates quantised with the grain's step (float32
  // product, ties to even, clamped to +-32767), counting saturated ones
  int nsat[QT];
  float d2 = 1.f;
  if constexpr (CT == 3) {
    const float inv = scales[(size_t)g * 4];
    d2 = scales[(size_t)g * 4 + 2];
#pragma unroll
    for (int t = 0; t < QT; ++t) {
      const float q = rintf((lane < r ? zq[t][lane] : 0.f) * inv);
      const bool sat = lane < r && fabsf(q) > 32767.f;
      nsat[t] = __popcll(__ballot(sat));
      if (lane < r) zq[t][lane] = fminf(fmaxf(q, -32767.f), 32767.f);
    }
    wave_sync();
  }

  List L[QT];
  bool live[QT];
  int nlive = 0;
  const float sg = CT == 2 ? scales[g] : 1.f;
  // this lane's coordinate of the grain's code bounding box (lanes >= r idle),
  // widened by the largest rounding error of the code form so that it holds
  // the decoded values the scan uses: BF16 half-ulp 2^-9 relative; FP8 E4M3
  // half-ulp 2^-4 relative plus the subnormal quantum 2^-10 s_g
  float lo = (bound_lists && prune && lane < r) ? blo[(size_t)g * RP + lane] : 0.f;
  float hi = (bound_lists && prune && lane < r) ? bhi[(size_t)g * RP + lane] : 0.f;
  if (CT == 1 || CT == 2) {
    const float amax = fmaxf(fabsf(lo), fabsf(hi));
    const float w = CT == 1 ? amax * 0.001953125f : amax * 0.0625f + sg * 0.0009765625f;
    lo -= 1.0001f * w;
    hi += 1.0001f * w;
  }
  // int16 form: the box in code space (the code rounding is monotone, so the
  // codes of the box ends bound every member's codes), and the smallest
  // decoded residual (the decoded residual is monotone in eps_i)
  float emin_g = 0.f;
  if (CT == 3 && bound_lists && prune) {
    const float inv = scales[(size_t)g * 4];
    lo = lane < r ? q16f(lo, inv, -32767.f, 32767.f) : 0.f;
    hi = lane < r ? q16f(hi, inv, -32767.f, 32767.f) : 0.f;
    emin_g = q16f(emin[g], scales[(size_t)g * 4 + 1], 0.f, 65535.f) * scales[(size_t)g * 4 + 3];
  } else if (bound_lists && prune) {
    emin_g = emin[g];
  }
#pragma unroll
  for (int t = 0; t < QT; ++t) {
    uint64_t bnd = KEY_NONE;
    live[t] = t < cnt;
    if constexpr (CT == 3) {
      // quantisation envelope filter (Section 2.3): more than a quarter of the
      // coordinates saturated -> the grain is pruned for this query
      if (live[t] && 4 * nsat[t] > r) {
        live[t] = false;
        // empty list: every entry, so that a bound read from entry C - 1 of a
        // slot-0 list never sees a key left by an earlier search
        for (int i = lane; i < C; i += HNTL_WAVE) part[(size_t)pairs[t] * C + i] = KEY_NONE;
      }
    }
    if (live[t] && bound_lists) {
      const int p = pairs[t];
      // C-th key of the query's probe-0 list: KEY_NONE when that list holds
      // fewer than C candidates, was pruned, or was never written (an invalid
      // probe; the caller resets that entry before the slot-0 pass)
      bnd = bound_lists[((size_t)(p / P) * P) * C + C - 1];
      // that key holds an original id while this scan keys by grain position:
      // keep every candidate whose distance does not exceed the bound's, so an
      // exact distance tie is settled by the merge, in (distance, id) order
      if (bnd != KEY_NONE) bnd |= 0xFFFFFFFFull;
      if (prune && bnd != KEY_NONE) {
        // eq. 6 lower bound over the grain: squared distance from z_q to the
        // code bounding box, plus eps_q, plus the grain's smallest eps_i
        float lb;
        if constexpr (CT == 3) {
          // integer distance from the query's codes to the code box, exact in
          // float64, then the score's own arithmetic: a lower bound of every
          // member's score
          const float v = lane < r ? zq[t][lane] : 0.f;
          const double dd = (double)fmaxf(fmaxf(lo - v, v - hi), 0.f);
          const double S = wave_sum_d(dd * dd);
          lb = fmaf((float)S, d2, emin_g + eq[t]);
        } else {
          const float v = lane < r ? zq[t][lane] : 0.f;
          const float dd = fmaxf(fmaxf(lo - v, v - hi), 0.f);
          lb = wave_sum(dd * dd) + eq[t] + emin_g;
        }
        if (lb * (1.f - PRUNE_SLACK) > key_dist(bnd)) {
          live[t] = false;
          for (int i = lane; i < C; i += HNTL_WAVE) part[(size_t)p * C + i] = KEY_NONE;  // empty list
        }
      }
    }
    L[t].init(lists_all[wave][t], C, bnd);
    nlive += live[t] ? 1 : 0;
  }
  wave_sync();
  if (scored && lane == 0 && nlive > 0) atomicAdd(scored, (unsigned long long)nlive * (unsigned long long)ng);
  // int16 form: each pair's query as split words, and |q|^2
  double qn[QT];
  if constexpr (CT == 3) {
#pragma unroll
    for (int t = 0; t < QT; ++t) qn[t] = i16_split_query<RP>(zq[t], lane);
    wave_sync();
  }

  if (nlive > 0) {
    for (int b = 0; b < nb; ++b) {
      const float ei = eps[(size_t)(b0 + b) * B + lane];
      const bool valid = b * B + lane < ng;
      const uint32_t pos = (uint32_t)(pos0 + b * B + lane);
      if constexpr (CT == 3) {
        uint32_t w[RP / 2];
        load_raw<RP, CT>(w, codes, (size_t)(b0 + b), lane);
        const double cn = i16_sq_norm<RP / 2>(w);
#pragma unroll
        for (int t = 0; t < QT; ++t) {
          if (live[t]) {
            // the integer distance, exact; then (1 / inv_g)^2 S + r_hat_i / rinv_g + eps_q
            const double S = fma(-2.0, i16_cross<RP / 2>(reinterpret_cast<const uint32_t*>(zq[t]), w), qn[t] + cn);
            L[t].offer_f(fmaf((float)S, d2, ei + eq[t]), pos, valid);
          }
        }
        continue;
      }
      float c[RP];
      load_block<RP, CT>(c, codes, (size_t)(b0 + b), lane, sg);
#pragma unroll
      for (int t = 0; t < QT; ++t) {
        if (live[t]) {
          {
            const floatx4* z4 = reinterpret_cast<const floatx4*>(zq[t]);
            float acc = 0.f;
#pragma unroll
            for (int j4 = 0; j4 < RP / 4; ++j4) {
              const floatx4 z = z4[j4];
#pragma unroll
              for (int e4 = 0; e4 < 4; ++e4) {
                const float df = z[e4] - c[4 * j4 + e4];
                acc = fmaf(df, df, acc);
              }
            }
            L[t].offer_f(acc + eq[t] + ei, pos, valid);
          }
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < QT; ++t) {
    if (live[t]) {
      L[t].finish();
      uint64_t* out = part + (size_t)pairs[t] * C;
#pragma unroll
      for (int rr = 0; rr < CAP / 64; ++rr) {
        const int i = rr * 64 + lane;
        const uint64_t k = L[t].best[rr];
        if (i < C) out[i] = (k == KEY_NONE) ? KEY_NONE : make_key(key_dist(k), (uint32_t)perm[key_id(k)]);
      }
    }
  }
}

template <int RP, int CAP, int CT>
void launch_rp_cap(const Index& ix, const float* T, const float* epsq, int P, int C, const Buckets& b, int list,
                   uint64_t* part, const uint64_t* bound_lists, bool prune, unsigned long long* scored, hipStream_t s) {
  // unbounded lists (nearest grain) insert often: 4 pairs per wave for more
  // waves in flight; bounded lists insert rarely: 16 pairs share every code load
  constexpr int QT_WIDE = CAP <= 128 ? 16 : 8;
  const dim3 grid((unsigned)b.max_items[list]);
  const void* codes = CT == 0 ? (const void*)ix.codes
                    : CT == 1 ? (const void*)ix.codes_bf16
                    : CT == 2 ? (const void*)ix.codes_fp8
                              : (const void*)ix.codes_i16;
  const float* scales = CT == 3 ? ix.i16_steps : ix.scales;
  const float* eps = CT == 3 ? ix.eps_i16 : ix.eps;
  const ItemLists& Ls = b.lists;
  if (bound_lists == nullptr)
    hipLaunchKernelGGL((scan_f32_kernel<RP, CAP, 4, CT>), grid, dim3(64 * (ITEM / 4)), 0, s, codes, scales, eps,
                       ix.goff,
                       ix.boff, ix.perm, (int)ix.r, T, epsq, P, C, Ls.ioff[list], Ls.lstart[list], Ls.lcount[list],
                       (int)ix.G, b.order, part, bound_lists, prune ? 1 : 0, ix.blo, ix.bhi, ix.emin, scored);
  else
    hipLaunchKernelGGL((scan_f32_kernel<RP, CAP, QT_WIDE, CT>), grid, dim3(64 * (ITEM / QT_WIDE)), 0, s, codes,
                       scales, eps, ix.goff, ix.boff, ix.perm, (int)ix.r, T, epsq, P, C, Ls.ioff[list], Ls.lstart[list],
                       Ls.lcount[list], (int)ix.G, b.order, part, bound_lists, prune ? 1 : 0, ix.blo, ix.bhi, ix.emin, scored);
}

template <int RP, int CT>
void launch_rp(const Index& ix, const float* T, const float* epsq, int P, int C, const Buckets& b, int list,
               uint64_t* part,
               const uint64_t* bound_lists, bool prune, unsigned long long* scored, hipStream_t s) {
  const int cap = pow2_at_least(C < 64 ? 64 : C);
  if (cap == 64)
    launch_rp_cap<RP, 64, CT>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s);
  else if (cap == 128)
    launch_rp_cap<RP, 128, CT>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s);
  else
    launch_rp_cap<RP, 256, CT>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s);
}

template <int CT>
void launch_ct(const Index& ix, const float* T, const float* epsq, int P, int C, const Buckets& b, int list,
               uint64_t* part, const uint64_t* bound_lists, bool prune, unsigned long long* scored, hipStream_t s) {
  switch (ix.rp) {
    case 8: launch_rp<8, CT>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s); break;
    case 16: launch_rp<16, CT>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s); break;
    case 24: launch_rp<24, CT>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s); break;
    case 32: launch_rp<32, CT>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s); break;
    case 40: launch_rp<40, CT>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s); break;
    case 48: launch_rp<48, CT>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s); break;
    case 56: launch_rp<56, CT>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s); break;
    case 64: launch_rp<64, CT>(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s); break;
    default: throw ArgError{HNTL_EUNSUPPORTED, "padded rank must be a multiple of 8 up to 64"};
  }
}

}  // namespace scan_detail
}  // namespace hntl
