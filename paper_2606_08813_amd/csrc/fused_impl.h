// Persistent fused project-scan-select kernel: the batching form of the
// search (paper Section 2.1 steps 2-3 and eq. 1-6) for batches of uneven size
// over grains of very uneven size.
//
// One launch runs a fixed number of workgroups (as many as fit the device);
// every wave of them is an independent worker that takes work items from
// device ticket counters until the items run out (no workgroup barriers).
// The items come in three runs, each ordered largest grain first so that the
// long items start early:
//
//   1. projection items: 16 (query, grain) pairs of one grain, whose tangents
//      z_q and eps_q the wave computes on the MFMA units (the same wave
//      routine as the grain-major projection kernel), then flags the item
//      as done (release);
//   2. scan items of probe slot 0 (each query's nearest grain);
//   3. scan items of the other probe slots.
//
// With the schedule option proj = 1 the projection runs as its own launch
// before this kernel, which then has no projection items and no waits.
//
// A scan item holds QT pairs of one grain and one block range of it (R
// blocks, or the whole grain for R = 0).  Consecutive items are the tiles of
// one range; a class of workgroups takes runs of them, so the waves that run
// them read the same blocks through one L2.  Every item was decoded before
// the launch into a descriptor (grain, range, pairs, and the projection items
// that hold those pairs).  Before it reads tangents, a scan item waits until
// those projection items are done (acquire).  The wait cannot deadlock:
// tickets are handed out in item order, so every projection item was taken
// earlier by a running wave that never waits itself; a spin limit still
// bounds it and flags an error.
//
// Two passes (a schedule option): the launch with phase 1 runs only the
// projection and slot-0 items, a second launch with phase 2 the other slots,
// which then start from the bound of each query's nearest grain, as in the
// staged search; phase 0 runs all items in one launch.
//
// Exact shared pruning.  Every query keeps one bound in device memory, the
// smallest C-th distance of any of its lists that already holds C
// candidates.  The query's final pool (the C smallest (D, id) over all its
// probed grains) cannot contain a candidate whose distance exceeds that
// bound, so a list may drop such candidates, and a whole pair is skipped when
// a lower bound of eq. 6 over its grain exceeds it: first eps_q + the grain's
// smallest eps_i (no tangent needed), then the box distance of z_q to the
// grain's code bounding box added to that.  Lists publish their C-th distance
// (atomic min) and re-read the bound every REFRESH blocks.  Which candidates
// a list drops depends on timing; the merged pool does not, since it is the
// exact top C in every case.
#pragma once

#include <algorithm>

#include "project_impl.h"
#include "scan_impl.h"

namespace hntl {
namespace fused_detail {

using proj_detail::project_wave;
using proj_detail::project_wave_bf16;
using scan_detail::i16_cross;
using scan_detail::i16_sq_norm;
using scan_detail::i16_split_query;
using scan_detail::ListOf;
using scan_detail::load_block;
using scan_detail::PRUNE_SLACK;
using scan_detail::q16f;

constexpr int REFRESH = 16;                 // blocks between bound exchanges
constexpr long long SPIN_LIMIT = 1ll << 26;  // wait polls before giving up

constexpr uint32_t NO_BOUND = 0xFFFFFFFFu;
constexpr int NCTR = 8;          // scan-item ticket counters (classes of workgroups)
constexpr int CTR_STRIDE = 64;   // ints between counters (256 bytes)
constexpr int RUN = 16;          // consecutive scan items per class and turn

// A bound on the distance part only: the list keys carry grain positions,
// which do not order like the original ids across grains, so every candidate
// at the bound's distance is kept and the merge settles exact ties.
__device__ __forceinline__ uint64_t bound_key(uint32_t ord) {
  return ord == NO_BOUND ? KEY_NONE : (((uint64_t)ord << 32) | 0xFFFFFFFFull);
}

// A wave's LDS: the tile's query tangents zq[QT][RP] first (16-byte rows, so
// the scoring loop reads them as 16-byte vectors at small constant offsets
// from one base), then eps_q[QT] (padded to 16 bytes), then the QT lists'
// staging areas.
template <int RP, int QT>
constexpr size_t zq_lds_bytes() {
  return (size_t)QT * RP * 4 + ((size_t)QT * 4 + 15) / 16 * 16;
}
template <int RP, int QT, int LK>
constexpr size_t wave_lds_bytes() {
  return zq_lds_bytes<RP, QT>() + (size_t)QT * LK * 8;
}

// One wave's part of a scan item: its cnt (<= QT) pairs of grain g against
// block range `range` of the grain (no workgroup barrier inside).
template <int RP, int CAP, int QT, int CT>
__device__ __forceinline__ void scan_tile(const FusedArgs& a, uint64_t* my, int g, int range,
                                          const int32_t* __restrict__ pairs, int cnt) {
  using List = typename ListOf<CAP>::type;
  constexpr int LK = ListOf<CAP>::lds;
  const int lane = lane_id();
  const int P = a.P, C = a.C, r = a.r;
  float(*zq)[RP] = reinterpret_cast<float(*)[RP]>(my);
  float* eq = reinterpret_cast<float*>(my) + QT * RP;
  uint64_t* lists_lds = my + zq_lds_bytes<RP, QT>() / 8;
  const int pos0 = ldg(a.goff + g);
  const int ng = ldg(a.goff + g + 1) - pos0;
  const int b0 = ldg(a.boff + g);
  const int nb = ldg(a.boff + g + 1) - b0;
  const int rb0 = a.R ? range * a.R : 0;
  const int rb1 = a.R ? min(nb, rb0 + a.R) : nb;

  // lane t < cnt holds pair t, its query's current bound, its eps_q and its
  // list base: one round of loads for all pairs of the tile
  int pv = 0;
  if (lane < cnt) pv = ldg(pairs + lane);
  uint32_t obv = NO_BOUND;
  float eqv = 0.f;
  int lbv = pv;
  if (lane < cnt) {
    obv = __hip_atomic_load(gptr(a.qbound + pv / P), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    eqv = ldg(a.epsq + pv);
    if (a.lbase) lbv = ldg(a.lbase + pv);
  }
  // the grain's smallest eps_i; for the int16 form the smallest decoded
  // residual (monotone in eps_i, so the decoded value of the grain's smallest
  // eps_i), with the index's own arithmetic
  float emin_g = 0.f;
  if (a.prune) {
    emin_g = ldg(a.emin + g);
    if constexpr (CT == 3)
      emin_g = q16f(emin_g, ldg(a.scales + (size_t)g * 4 + 1), 0.f, 65535.f) * ldg(a.scales + (size_t)g * 4 + 3);
  }
  // eps_q + the grain's smallest eps_i bounds eq. 6 from below without the
  // tangent (the squared tangent distance is >= 0 and the float sums are
  // monotone): when it already exceeds every pair's query bound, the tile is
  // done without loading its tangents
  if (a.prune) {
    const bool cut = lane < cnt && obv != NO_BOUND && (eqv + emin_g) * (1.f - PRUNE_SLACK) > ord2f(obv);
    const uint64_t all = cnt >= 64 ? ~0ull : ((1ull << cnt) - 1ull);
    if (__ballot(cut) == all) {
      if (lane < cnt) stg(a.part + (size_t)((int64_t)lbv + range) * C, KEY_NONE);  // empty lists
      return;
    }
  }
  for (int idx = lane; idx < QT * RP; idx += HNTL_WAVE) {
    const int t = idx / RP, j = idx % RP;
    const int pt = __shfl(pv, t, 64);
    zq[t][j] = (t < cnt && j < r) ? ldg(a.T + (size_t)pt * r + j) : 0.f;
  }
  if (lane < QT) eq[lane] = eqv;
  wave_sync();
  // int16 form: the pairs' tangents quantised with the grain's step (float32
  // product, ties to even, clamped to +-32767, kept as exact float integers),
  // counting saturated coordinates for the envelope filter
  int nsat[QT];
  float d2 = 1.f;
  if constexpr (CT == 3) {
    const float inv = ldg(a.scales + (size_t)g * 4);
    d2 = ldg(a.scales + (size_t)g * 4 + 2);
#pragma unroll
    for (int t = 0; t < QT; ++t) {
      const float qv = rintf((lane < r ? zq[t][lane] : 0.f) * inv);
      nsat[t] = __popcll(__ballot(lane < r && fabsf(qv) > 32767.f));
      if (lane < r) zq[t][lane] = fminf(fmaxf(qv, -32767.f), 32767.f);
    }
    wave_sync();
  }

  const float sg = CT == 2 ? ldg(a.scales + g) : 1.f;
  float lo = (a.prune && lane < r) ? ldg(a.blo + (size_t)g * RP + lane) : 0.f;
  float hi = (a.prune && lane < r) ? ldg(a.bhi + (size_t)g * RP + lane) : 0.f;
  if (CT == 1 || CT == 2) {  // the box must hold the decoded values the scan uses
    const float amax = fmaxf(fabsf(lo), fabsf(hi));
    const float w = CT == 1 ? amax * 0.001953125f : amax * 0.0625f + sg * 0.0009765625f;
    lo -= 1.0001f * w;
    hi += 1.0001f * w;
  } else if (CT == 3) {  // the box in code space (the code rounding is monotone)
    const float inv = ldg(a.scales + (size_t)g * 4);
    lo = lane < r ? q16f(lo, inv, -32767.f, 32767.f) : 0.f;
    hi = lane < r ? q16f(hi, inv, -32767.f, 32767.f) : 0.f;
  }
  List Ls[QT];
  bool live[QT];
  int nlive = 0;
#pragma unroll
  for (int t = 0; t < QT; ++t) {
    live[t] = t < cnt;
    uint64_t bnd = KEY_NONE;
    if constexpr (CT == 3) {
      // quantisation envelope filter (Section 2.3): more than a quarter of the
      // coordinates saturated -> the grain is pruned for this query
      if (live[t] && 4 * nsat[t] > r) {
        live[t] = false;
        const int64_t slot = (int64_t)__builtin_amdgcn_readlane(lbv, t) + range;
        if (lane == 0) stg(a.part + (size_t)slot * C, KEY_NONE);  // empty list
      }
    }
    if (live[t]) {
      const uint32_t ob = (uint32_t)__builtin_amdgcn_readlane((int)obv, t);
      bnd = bound_key(ob);
      if (a.prune && ob != NO_BOUND) {
        float lb;
        if constexpr (CT == 3) {
          // exact integer distance to the code box, then the score's arithmetic
          const float v = lane < r ? zq[t][lane] : 0.f;
          const double dd = (double)fmaxf(fmaxf(lo - v, v - hi), 0.f);
          lb = fmaf((float)wave_sum_d(dd * dd), d2, emin_g + eq[t]);
        } else {
          const float v = lane < r ? zq[t][lane] : 0.f;
          const float dd = fmaxf(fmaxf(lo - v, v - hi), 0.f);
          lb = wave_sum(dd * dd) + eq[t] + emin_g;
        }
        if (__builtin_amdgcn_readfirstlane(lb * (1.f - PRUNE_SLACK) > ord2f(ob) ? 1 : 0)) {
          live[t] = false;
          const int64_t slot = (int64_t)__builtin_amdgcn_readlane(lbv, t) + range;
          if (lane == 0) stg(a.part + (size_t)slot * C, KEY_NONE);  // empty list
        }
      }
    }
    Ls[t].init(lists_lds + t * LK, C, bnd);
    nlive += live[t] ? 1 : 0;
  }
  wave_sync();
  if (nlive == 0) return;
  // int16 form: each pair's query as split words, and |q|^2
  double qn[QT];
  if constexpr (CT == 3) {
#pragma unroll
    for (int t = 0; t < QT; ++t) qn[t] = i16_split_query<RP>(zq[t], lane);
    wave_sync();
  }
  if (a.scored && lane == 0) {
    const int nvec = min(ng, rb1 * B) - rb0 * B;
    if (nvec > 0)
      __hip_atomic_fetch_add(gptr(a.scored), (unsigned long long)nlive * (unsigned long long)nvec, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }

  const void* codes = a.codes;
  auto exchange = [&]() {
    // publish each list's C-th distance, adopt the query's bound
#pragma unroll
    for (int t = 0; t < QT; ++t) {
      if (live[t]) {
        const int q = __builtin_amdgcn_readlane(pv, t) / P;
        const uint64_t own = Ls[t].cth();
        if (own != KEY_NONE && lane == 0)
          __hip_atomic_fetch_min(gptr(a.qbound + q), (uint32_t)(own >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t ob = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(gptr(a.qbound + q), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        Ls[t].tighten(bound_key(ob));
      }
    }
  };
  auto score = [&](const float(&c)[RP], float e, int b) {
    const bool valid = b * B + lane < ng;
    const uint32_t pos = (uint32_t)(pos0 + b * B + lane);
#pragma unroll
    for (int t = 0; t < QT; ++t) {
      if (live[t]) {
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
        Ls[t].offer_f(acc + eq[t] + e, pos, valid);
      }
    }
  };
  // int16 form: scored from the raw code words; the integer distance is exact,
  // then (1 / inv_g)^2 S + r_hat_i / rinv_g + eps_q
  constexpr int RW = scan_detail::RawWords<RP, CT>::n;
  auto score16 = [&](const uint32_t(&w)[RW], float e, int b) {
    const bool valid = b * B + lane < ng;
    const uint32_t pos = (uint32_t)(pos0 + b * B + lane);
    const double cn = i16_sq_norm<RW>(w);
#pragma unroll
    for (int t = 0; t < QT; ++t) {
      if (live[t]) {
        const double S = fma(-2.0, i16_cross<RW>(reinterpret_cast<const uint32_t*>(zq[t]), w), qn[t] + cn);
        Ls[t].offer_f(fmaf((float)S, d2, e + eq[t]), pos, valid);
      }
    }
  };
  if constexpr (QT == 1) {
    // one pair per wave (small batches, few waves, latency-bound): a ring of
    // NBUF register buffers of raw code words, NBUF - 1 blocks requested ahead
    // of the one being scored (decoded only when scored, so no wait is forced
    // at the request)
    constexpr int NBUF = RW * 4 <= 160 ? 4 : (RW * 3 <= 160 ? 3 : 2);
    uint32_t wr[NBUF][RW];
    float er[NBUF];
#pragma unroll
    for (int u = 0; u < NBUF - 1; ++u)
      if (rb0 + u < rb1) {
        scan_detail::load_raw<RP, CT>(wr[u], codes, (size_t)(b0 + rb0 + u), lane);
        er[u] = ldg(a.eps + (size_t)(b0 + rb0 + u) * B + lane);
      }
    for (int b = rb0; b < rb1; b += NBUF) {
#pragma unroll
      for (int u = 0; u < NBUF; ++u) {
        const int bb = b + u;
        if (bb < rb1) {
          if (bb > rb0 && ((bb - rb0) % REFRESH) == 0) exchange();
          const int nx = bb + NBUF - 1;
          if (nx < rb1) {
            scan_detail::load_raw<RP, CT>(wr[(u + NBUF - 1) % NBUF], codes, (size_t)(b0 + nx), lane);
            er[(u + NBUF - 1) % NBUF] = ldg(a.eps + (size_t)(b0 + nx) * B + lane);
          }
          if constexpr (CT == 3) {
            score16(wr[u], er[u], bb);
          } else {
            float c[RP];
            scan_detail::decode_raw<RP, CT>(c, wr[u], sg);
            score(c, er[u], bb);
          }
        }
      }
    }
  } else {
    // one block of codes in registers per wave; the loads of the other waves
    // on the CU cover the HBM latency
    for (int b = rb0; b < rb1; ++b) {
      if (b > rb0 && ((b - rb0) % REFRESH) == 0) exchange();
      if constexpr (CT == 3) {
        uint32_t w[RW];
        scan_detail::load_raw<RP, CT>(w, codes, (size_t)(b0 + b), lane);
        score16(w, ldg(a.eps + (size_t)(b0 + b) * B + lane), b);
      } else {
        float c[RP];
        load_block<RP, CT>(c, codes, (size_t)(b0 + b), lane, sg);
        score(c, ldg(a.eps + (size_t)(b0 + b) * B + lane), b);
      }
    }
  }

  // The merge takes each list's keys in any order, so a list whose staged
  // arrivals fit after its sorted keys is written without the final flush
  // (about half of the lists on the 10M Zipf workload: those that start
  // from a tight query bound see few arrivals).  Its C-th key is published
  // only when it is full and sorted.
  wave_sync();
#pragma unroll
  for (int t = 0; t < QT; ++t) {
    if (live[t]) {
      const int nm = Ls[t].merged();
      const bool as_is = nm + Ls[t].nstage <= C;
      if (!as_is) Ls[t].finish();
      const int p = __builtin_amdgcn_readlane(pv, t);
      const uint64_t own = Ls[t].cth();
      if (own != KEY_NONE && lane == 0)
        __hip_atomic_fetch_min(gptr(a.qbound + p / P), (uint32_t)(own >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int64_t slot = (int64_t)__builtin_amdgcn_readlane(lbv, t) + range;
      uint64_t* out = a.part + (size_t)slot * C;
#pragma unroll
      for (int rr = 0; rr < CAP / 64; ++rr) {
        const int i = rr * 64 + lane;
        const uint64_t kk = as_is ? Ls[t].unsorted_at(i, rr, nm) : Ls[t].best[rr];
        if (i < C) stg(out + i, (kk == KEY_NONE) ? KEY_NONE : make_key(key_dist(kk), (uint32_t)ldg(a.perm + key_id(kk))));
      }
    }
  }
}

template <int RP, int CAP, int QT, int CT>
__global__ __launch_bounds__(512) void fused_kernel(const FusedArgs* __restrict__ ap) {
  const FusedArgs& a = *ap;
  constexpr int LK = ListOf<CAP>::lds;
  constexpr int NCT = (RP + 15) / 16;
  extern __shared__ uint64_t smem[];
  const int lane = lane_id();
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint64_t* my = smem + (size_t)wave * (wave_lds_bytes<RP, QT, LK>() / 8);
  const int G = a.G;
  const int nP = __builtin_amdgcn_readfirstlane(ldg(a.ioff[LIST_ALL] + G));
  const int n0 = __builtin_amdgcn_readfirstlane(ldg(a.ioff[LIST_SLOT0] + G));
  const int n1 = __builtin_amdgcn_readfirstlane(ldg(a.ioff[LIST_REST] + G));
  const int total = nP + n0 + n1;
  using ivec4 = int __attribute__((ext_vector_type(4)));
  const ivec4* desc = reinterpret_cast<const ivec4*>(a.items);  // two per item

  // Each wave is its own worker: it takes tickets until they run out, and
  // nothing in the loop synchronises waves.  All 64 lanes add 1 to a counter,
  // so it moves by 64 per fetch (the compiler folds the wave's adds into one
  // atomic) and lane 0's old value / 64 is the ticket.  Projection items come
  // from one counter (checked with a plain load before any atomic, so waves
  // that find it exhausted cost no atomic); scan items are interleaved over
  // NCTR counters, one per class of workgroups, so tickets are not all taken
  // from one address.  A wave reaches the scan items only after every
  // projection ticket has been handed out.  A class takes runs of RUN
  // consecutive scan items (the tiles of one grain and block range are
  // consecutive), and class kc = blockIdx.x % 8 is also the XCD the workgroup
  // runs on, so the tiles that re-read a grain's blocks share one L2.  Items
  // are decoded once per run into descriptors (one 32-byte record each).
  using gptr = int32_t __attribute__((address_space(1)))*;
  if (a.phase != 2 && !a.proj_ext) {
    const gptr pctr = (gptr)a.ticket;
    for (;;) {
      if (__builtin_amdgcn_readfirstlane(__hip_atomic_load(pctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >=
          nP * 64)
        break;
      const int it =
          __builtin_amdgcn_readfirstlane(__hip_atomic_fetch_add(pctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >>
          6;
      if (it >= nP) break;
      const ivec4 d = ldg(desc + 2 * (size_t)it);
      const int g = __builtin_amdgcn_readfirstlane(d[0]);
      const int cnt = __builtin_amdgcn_readfirstlane(d[3]);
      const int32_t* pairs = a.order + __builtin_amdgcn_readfirstlane(d[2]);
      if (a.proj_bf16)
        project_wave_bf16<NCT>(a.Q, a.d, a.P, a.centroids, a.basis16, a.r, g, pairs, cnt, a.T, a.epsq);
      else
        project_wave<true, NCT>(a.Q, a.d, a.P, a.centroids, a.basis, a.r, g, pairs, cnt, a.T, a.epsq);
      // release: the tangents of this item are visible before its flag is
      __hip_atomic_store((gptr)(a.proj_done + it), 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  const int kc = (int)(blockIdx.x % NCTR);
  const gptr sctr = (gptr)(a.ticket + CTR_STRIDE * (1 + kc));
  const int slo = a.phase == 2 ? nP + n0 : nP;     // scan items of this launch
  const int shi = a.phase == 1 ? nP + n0 : total;
  // the next ticket is taken while the current item runs, so its atomic
  // round trip is hidden
  int tv = __hip_atomic_fetch_add(sctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    const int tk = __builtin_amdgcn_readfirstlane(tv) >> 6;
    const int it = slo + (tk / RUN) * (NCTR * RUN) + kc * RUN + tk % RUN;
    if (it >= shi) break;
    const ivec4 d = ldg(desc + 2 * (size_t)it);
    tv = __hip_atomic_fetch_add(sctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int g = __builtin_amdgcn_readfirstlane(d[0]);
    const int range = __builtin_amdgcn_readfirstlane(d[1]);
    const int32_t* pairs = a.order + __builtin_amdgcn_readfirstlane(d[2]);
    const int cnt = __builtin_amdgcn_readfirstlane(d[3]);
    if (!a.proj_ext) {
      // wait (acquire) for the projection items that hold this tile's pairs
      const ivec4 e = ldg(desc + 2 * (size_t)it + 1);
      const int c0 = __builtin_amdgcn_readfirstlane(e[0]), c1 = __builtin_amdgcn_readfirstlane(e[1]);
      for (int c = c0; c <= c1; ++c) {
        for (long long spin = 0;; ++spin) {
          const int done = __builtin_amdgcn_readfirstlane(
              __hip_atomic_load(gptr(a.proj_done + c), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT));
          if (done != 0) break;
          if (spin > SPIN_LIMIT) {
            __hip_atomic_fetch_or(gptr(a.err), 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
    }
    scan_tile<RP, CAP, QT, CT>(a, my, g, range, pairs, cnt);
  }
}

template <int RP, int CAP, int QT, int CT>
struct Inst {
  static constexpr size_t lds_per_wave = wave_lds_bytes<RP, QT, ListOf<CAP>::lds>();
  static int resident(int nw) {
    static int cache[9] = {0};
    if (nw < 1 || nw > 8) return 0;
    if (cache[nw] == 0) {
      int per_cu = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fused_kernel<RP, CAP, QT, CT>, 64 * nw,
                                                       lds_per_wave * nw) != hipSuccess)
        per_cu = 1;
      int dev = 0, ncu = 0;
      (void)hipGetDevice(&dev);
      (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
      cache[nw] = std::max(1, per_cu) * std::max(1, ncu);
    }
    return cache[nw];
  }
  static void launch(const FusedArgs* a, int nw, int grid, hipStream_t s) {
    if (grid <= 0) grid = resident(nw);
    hipLaunchKernelGGL((fused_kernel<RP, CAP, QT, CT>), dim3((unsigned)grid), dim3(64 * nw), lds_per_wave * nw, s, a);
  }
};

// Dispatch over (rp, cap, qt) for one code form; F(Inst) is called with the
// matching instantiation.  Returns false for combinations not compiled.
template <int CT, class F>
bool dispatch(int rp, int C, int qt, F&& f) {
  const int cap = pow2_at_least(C < 64 ? 64 : C);
#define HNTL_FQ(RPV, CAPV)                               \
  if (rp == RPV && cap == CAPV) {                        \
    if (qt == 1) return f(Inst<RPV, CAPV, 1, CT>{}), true; \
    if (qt == 2) return f(Inst<RPV, CAPV, 2, CT>{}), true; \
    if (qt == 4) return f(Inst<RPV, CAPV, 4, CT>{}), true; \
    if (qt == 8) return f(Inst<RPV, CAPV, 8, CT>{}), true; \
    return false;                                        \
  }
#define HNTL_FR(RPV) HNTL_FQ(RPV, 64) HNTL_FQ(RPV, 128) HNTL_FQ(RPV, 256)
  HNTL_FR(16)
  HNTL_FR(32)
  HNTL_FR(48)
  HNTL_FR(64)
#undef HNTL_FR
#undef HNTL_FQ
  return false;
}

}  // namespace fused_detail
}  // namespace hntl

// Defines the per-code-form entry points of one translation unit.
#define HNTL_FUSED_TU(CT)                                                                                      \
  namespace hntl {                                                                                             \
  bool launch_fused_ct##CT(const FusedArgs* a, int rp, int C, int qt, int nw, int grid, hipStream_t s) {       \
    return fused_detail::dispatch<CT>(rp, C, qt, [&](auto inst) { decltype(inst)::launch(a, nw, grid, s); }); \
  }                                                                                                            \
  int fused_resident_ct##CT(int rp, int C, int qt, int nw) {                                                   \
    int n = 0;                                                                                                 \
    fused_detail::dispatch<CT>(rp, C, qt, [&](auto inst) { n = decltype(inst)::resident(nw); });              \
    return n;                                                                                                  \
  }                                                                                                            \
  }
