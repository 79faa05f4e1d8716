// Device helpers shared by the HNTL kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define HNTL_WAVE 64

typedef float floatx4 __attribute__((ext_vector_type(4)));

namespace hntl {

// ---------------------------------------------------------------- sort keys
// A candidate is one 64-bit key: the float's order-preserving bit image in the
// high half, the id in the low half.  Unsigned comparison of keys is then the
// lexicographic (distance, id) order, which is the tie rule everywhere.
__device__ __forceinline__ uint32_t f2ord(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t o) {
  uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
  return __uint_as_float(u);
}
__device__ __forceinline__ uint64_t make_key(float d, uint32_t id) {
  return ((uint64_t)f2ord(d) << 32) | (uint64_t)id;
}
__device__ __forceinline__ float key_dist(uint64_t k) { return ord2f((uint32_t)(k >> 32)); }
__device__ __forceinline__ uint32_t key_id(uint64_t k) { return (uint32_t)k; }
constexpr uint64_t KEY_NONE = ~0ull;

// ---------------------------------------------------------------- wave utils
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// Orders LDS accesses of the lanes of one wave (no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int mbcnt64(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------- register-resident top-64 list
// One wave keeps the C <= 64 smallest keys of a stream, the sorted list held
// in registers, one key per lane (lane i holds the i-th smallest).  A key is
// staged only if it beats the current threshold (the C-th best key); arrivals
// are compacted into a 64-entry LDS stage, and when the stage would overflow
// a flush loads it one key per lane, sorts it with a bitonic network across
// the lanes (shuffles, no LDS round trips) and merges it into the register
// list.  Threshold and stage count are wave-uniform (scalar registers).  This
// is the threshold + buffer + merging-network scheme of GPU k-selection
// (Johnson, Douze, Jegou, "Billion-scale similarity search with GPUs"), laid
// out for 64-wide waves.
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  const uint32_t lo = __shfl_xor((uint32_t)v, m, 64);
  const uint32_t hi = __shfl_xor((uint32_t)(v >> 32), m, 64);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  const uint32_t lo = __shfl((uint32_t)v, src, 64);
  const uint32_t hi = __shfl((uint32_t)(v >> 32), src, 64);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Ascending bitonic sort of one key per lane.
__device__ __forceinline__ uint64_t wave_sort64(uint64_t key) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint64_t other = shfl_xor_u64(key, j);
      const bool up = (lane & k) == 0;
      const bool lower = (lane & j) == 0;
      const uint64_t mn = key < other ? key : other;
      const uint64_t mx = key < other ? other : key;
      key = (up == lower) ? mn : mx;
    }
  return key;
}

struct WaveTop64 {
  uint64_t* stage;  // 64 keys of LDS
  uint64_t best;    // this lane's entry of the sorted list
  uint64_t thr;     // uniform
  uint64_t bound;   // uniform
  int nstage;       // uniform
  int C;

  __device__ __forceinline__ void init(uint64_t* lds, int C_, uint64_t bound_ = KEY_NONE) {
    stage = lds;
    C = C_;
    nstage = 0;
    bound = bound_;
    thr = bound_;
    best = KEY_NONE;
  }

  __device__ __forceinline__ void flush() {
    if (nstage == 0) return;
    const int lane = lane_id();
    wave_sync();
    uint64_t k = lane < nstage ? stage[lane] : KEY_NONE;
    wave_sync();
    k = wave_sort64(k);
    // half-cleaner of (best ascending, arrivals descending), then bitonic merge
    const uint64_t rev = shfl_u64(k, 63 - lane);
    uint64_t m = best < rev ? best : rev;
#pragma unroll
    for (int j = 32; j > 0; j >>= 1) {
      const uint64_t other = shfl_xor_u64(m, j);
      const bool lower = (lane & j) == 0;
      const uint64_t mn = m < other ? m : other;
      const uint64_t mx = m < other ? other : m;
      m = lower ? mn : mx;
    }
    best = m;
    const uint64_t t = uniform_u64(shfl_u64(best, C - 1));
    thr = t < bound ? t : bound;
    nstage = 0;
  }

  __device__ __forceinline__ void offer(uint64_t key, bool valid) {
    bool pass = valid && key < thr;
    uint64_t m = __ballot(pass);
    if (m == 0) return;
    int cnt = __popcll(m);
    if (nstage + cnt > 64) {
      flush();
      pass = valid && key < thr;
      m = __ballot(pass);
      if (m == 0) return;
      cnt = __popcll(m);
    }
    if (pass) stage[nstage + mbcnt64(m)] = key;
    nstage += cnt;
  }

  // After finish(), lane i holds the i-th smallest key (KEY_NONE padded).
  __device__ __forceinline__ void finish() { flush(); }

  __device__ __forceinline__ void tighten(uint64_t b) {
    if (b < bound) bound = b;
    if (b < thr) thr = b;
  }
  __device__ __forceinline__ uint64_t cth() const { return uniform_u64(shfl_u64(best, C - 1)); }
};

// ------------------------------------- register-resident top-(64 NR) list
// WaveTop64 widened to C <= 64 NR: the sorted list is NR keys per lane, list
// element r * 64 + lane in best[r].  A flush sorts the (at most 64) staged
// arrivals across the lanes, folds them into the last register block with a
// half-cleaner against the reversed arrivals (the elementwise minimum of the
// ascending list and the descending arrivals is bitonic and holds the 64 NR
// smallest of both), then sorts that bitonic sequence: compare-exchanges
// between register blocks for strides of 64 and more, lane shuffles below.
template <int NR>
struct WaveTopR {
  uint64_t* stage;   // 64 keys of LDS
  uint64_t best[NR];
  uint64_t thr;      // uniform
  uint64_t bound;    // uniform
  int nstage;        // uniform
  int C;

  __device__ __forceinline__ void init(uint64_t* lds, int C_, uint64_t bound_ = KEY_NONE) {
    stage = lds;
    C = C_;
    nstage = 0;
    bound = bound_;
    thr = bound_;
#pragma unroll
    for (int r = 0; r < NR; ++r) best[r] = KEY_NONE;
  }

  __device__ __forceinline__ void flush() {
    if (nstage == 0) return;
    const int lane = lane_id();
    wave_sync();
    uint64_t k = lane < nstage ? stage[lane] : KEY_NONE;
    wave_sync();
    k = wave_sort64(k);
    const uint64_t rev = shfl_u64(k, 63 - lane);
    best[NR - 1] = best[NR - 1] < rev ? best[NR - 1] : rev;
#pragma unroll
    for (int st = NR / 2; st >= 1; st >>= 1)
#pragma unroll
      for (int r = 0; r < NR; ++r)
        if ((r & st) == 0) {
          const uint64_t a = best[r], b = best[r + st];
          best[r] = a < b ? a : b;
          best[r + st] = a < b ? b : a;
        }
#pragma unroll
    for (int j = 32; j > 0; j >>= 1) {
      const bool lower = (lane & j) == 0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const uint64_t m = best[r];
        const uint64_t other = shfl_xor_u64(m, j);
        const uint64_t mn = m < other ? m : other;
        const uint64_t mx = m < other ? other : m;
        best[r] = lower ? mn : mx;
      }
    }
    const uint64_t t = cth();
    thr = t < bound ? t : bound;
    nstage = 0;
  }

  __device__ __forceinline__ void offer(uint64_t key, bool valid) {
    bool pass = valid && key < thr;
    uint64_t m = __ballot(pass);
    if (m == 0) return;
    int cnt = __popcll(m);
    if (nstage + cnt > 64) {
      flush();
      pass = valid && key < thr;
      m = __ballot(pass);
      if (m == 0) return;
      cnt = __popcll(m);
    }
    if (pass) stage[nstage + mbcnt64(m)] = key;
    nstage += cnt;
  }

  // After finish(), list element r * 64 + lane is best[r] (KEY_NONE padded).
  __device__ __forceinline__ void finish() { flush(); }

  __device__ __forceinline__ void tighten(uint64_t b) {
    if (b < bound) bound = b;
    if (b < thr) thr = b;
  }
  // The C-th smallest key merged so far (KEY_NONE while fewer than C).
  __device__ __forceinline__ uint64_t cth() const {
    const int e = C - 1;
    uint64_t v = best[0];
#pragma unroll
    for (int r = 1; r < NR; ++r)
      if ((e >> 6) == r) v = best[r];
    return uniform_u64(shfl_u64(v, e & 63));
  }
};

// ------------------------------------------------------------- work items
// Grain of work item `item` of a list whose items per grain have the exclusive
// prefix ioff[0..G] (the largest g with ioff[g] <= item); false past the end.
__device__ __forceinline__ bool item_grain(const int32_t* __restrict__ ioff, int G, int item, int& g) {
  if (item >= ioff[G]) return false;
  int lo = 0, hi = G;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ioff[mid] <= item)
      lo = mid;
    else
      hi = mid;
  }
  g = lo;
  return true;
}

// ------------------------------------------------------------------- MFMA
// v_mfma_f32_16x16x4_f32: lane l supplies A[l%16][l/16] and B[l/16][l%16] of a
// 16x4 by 4x16 product and holds D[4*(l/16)+i][l%16] for i = 0..3.
__device__ __forceinline__ floatx4 mfma16x16x4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

}  // namespace hntl
