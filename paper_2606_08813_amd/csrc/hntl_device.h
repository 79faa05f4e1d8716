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

// ------------------------------------------------------- global accesses
// Loads and stores through global (address space 1) pointers.  A pointer read
// from a struct in device memory is a generic pointer, and accesses through it
// compile to flat instructions, which count against the LDS wait counter as
// well: a wait for a shuffle or an LDS read would then also wait for every
// load in flight.  These helpers give global_load / global_store instead.
// T must be a scalar or a clang vector type (a class type would be copied
// through a generic reference).
#define HNTL_AS1 __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ T ldg(const T* p) {
  return *(const T HNTL_AS1*)p;
}
template <class T>
__device__ __forceinline__ void stg(T* p, T v) {
  *(T HNTL_AS1*)p = v;
}
template <class T>
__device__ __forceinline__ T HNTL_AS1* gptr(T* p) {
  return (T HNTL_AS1*)p;
}

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
// Lane `src` (wave-uniform) of v, read into scalar registers.
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int src) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}

// ------------------------------------------ lane exchanges without the LDS
// The value of lane (lane ^ J).  J <= 8 stays inside a row of 16 lanes and is
// one or two DPP moves (quad permutations for 1 and 2, a rotation by 8 for 8,
// shifts by 4 up and down for 4); J = 16 and 32 use the gfx950 permlane swaps
// of odd / even rows and of the two wave halves.  None of them goes through
// the LDS, so a sorting network built on them waits on no LDS round trip.
constexpr int DPP_QP_1032 = 0xB1;   // quad_perm [1, 0, 3, 2]
constexpr int DPP_QP_2301 = 0x4E;   // quad_perm [2, 3, 0, 1]
constexpr int DPP_FROM_UP4 = 0x104;  // row_shl:4, lane i reads lane i + 4 of its row
constexpr int DPP_FROM_DN4 = 0x114;  // row_shr:4, lane i reads lane i - 4 of its row
constexpr int DPP_ROR8 = 0x128;      // row_ror:8, lane i reads lane i ^ 8 of its row

// A DPP move with no old value to keep: every lane a caller uses reads a
// valid source lane (the two shifts by 4 leave four lanes of each row without
// one, and lane_xor<4> takes each lane's value from the shift that has it), so
// the result needs no copy of the source into the destination first.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}

template <int J>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
  const int lane = lane_id();
  if constexpr (J == 1) {
    return dpp_mov<DPP_QP_1032>(v);
  } else if constexpr (J == 2) {
    return dpp_mov<DPP_QP_2301>(v);
  } else if constexpr (J == 4) {
    const uint32_t up = dpp_mov<DPP_FROM_UP4>(v), dn = dpp_mov<DPP_FROM_DN4>(v);
    return (lane & 4) ? dn : up;
  } else if constexpr (J == 8) {
    return dpp_mov<DPP_ROR8>(v);
  } else if constexpr (J == 16) {
    // result 0: odd rows replaced by the even rows below them; result 1: even
    // rows replaced by the odd rows above them
    const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (lane & 16) ? p[0] : p[1];
  } else {
    static_assert(J == 32, "lane_xor: J must be a power of two below 64");
    const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (lane & 32) ? p[0] : p[1];
  }
}

// Compare-exchange of one key per lane with lane (lane ^ J): the smaller of
// the two where keep_min, the larger elsewhere.
template <int J>
__device__ __forceinline__ uint64_t cmpx_t(uint64_t key, bool keep_min) {
  const uint32_t lo = (uint32_t)key, hi = (uint32_t)(key >> 32);
  uint64_t a, b;
  if constexpr (J == 16 || J == 32) {
    // the swap leaves {own, partner} in its two results (their order depends
    // on the lane, which min / max do not care about)
    const auto pl = J == 16 ? __builtin_amdgcn_permlane16_swap(lo, lo, false, false)
                            : __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto ph = J == 16 ? __builtin_amdgcn_permlane16_swap(hi, hi, false, false)
                            : __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    a = ((uint64_t)ph[0] << 32) | pl[0];
    b = ((uint64_t)ph[1] << 32) | pl[1];
  } else {
    a = key;
    b = ((uint64_t)lane_xor<J>(hi) << 32) | lane_xor<J>(lo);
  }
  return (a < b) == keep_min ? a : b;
}
// j is a compile-time constant once the callers' loops are unrolled.
__device__ __forceinline__ uint64_t cmpx(uint64_t key, int j, bool keep_min) {
  switch (j) {
    case 1: return cmpx_t<1>(key, keep_min);
    case 2: return cmpx_t<2>(key, keep_min);
    case 4: return cmpx_t<4>(key, keep_min);
    case 8: return cmpx_t<8>(key, keep_min);
    case 16: return cmpx_t<16>(key, keep_min);
    default: return cmpx_t<32>(key, keep_min);
  }
}

// Sum over the wave (butterfly: every lane ends with the same total).
__device__ __forceinline__ float wave_sum(float v) {
  v += __uint_as_float(lane_xor<32>(__float_as_uint(v)));
  v += __uint_as_float(lane_xor<16>(__float_as_uint(v)));
  v += __uint_as_float(lane_xor<8>(__float_as_uint(v)));
  v += __uint_as_float(lane_xor<4>(__float_as_uint(v)));
  v += __uint_as_float(lane_xor<2>(__float_as_uint(v)));
  v += __uint_as_float(lane_xor<1>(__float_as_uint(v)));
  return v;
}

// Bitonic sort of one key per lane, ascending (DESC = false) or descending.
template <bool DESC = false>
__device__ __forceinline__ uint64_t wave_sort64(uint64_t key) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const bool up = (lane & k) == 0;
      const bool lower = (lane & j) == 0;
      key = cmpx(key, j, (up == lower) != DESC);
    }
  return key;
}

// The value part of a threshold key as a float ceiling: a key whose value
// exceeds it cannot enter (no threshold: +inf).  Comparing values against it
// admits a superset of the keys below the threshold key (equal values with
// larger ids too); a flush orders them by the whole key.
__device__ __forceinline__ float key_ceil(uint64_t k) { return k == KEY_NONE ? __builtin_inff() : key_dist(k); }

struct WaveTop64 {
  uint64_t* stage;  // 64 keys of LDS
  uint64_t best;    // this lane's entry of the sorted list
  uint64_t thr;     // uniform
  uint64_t bound;   // uniform
  float thr_f;      // uniform: key_ceil(thr)
  int nstage;       // uniform
  int C;

  __device__ __forceinline__ void init(uint64_t* lds, int C_, uint64_t bound_ = KEY_NONE) {
    stage = lds;
    C = C_;
    nstage = 0;
    bound = bound_;
    thr = bound_;
    thr_f = key_ceil(thr);
    best = KEY_NONE;
  }

  __device__ __forceinline__ void flush() {
    if (nstage == 0) return;
    const int lane = lane_id();
    wave_sync();
    uint64_t k = lane < nstage ? stage[lane] : KEY_NONE;
    wave_sync();
    k = wave_sort64<true>(k);
    // half-cleaner of (best ascending, arrivals descending), then bitonic merge
    uint64_t m = best < k ? best : k;
#pragma unroll
    for (int j = 32; j > 0; j >>= 1) m = cmpx(m, j, (lane & j) == 0);
    best = m;
    const uint64_t t = lane_u64(best, C - 1);
    thr = t < bound ? t : bound;
    thr_f = key_ceil(thr);
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

  // offer(make_key(v, id), valid) for v >= 0 or any non-NaN v: the threshold
  // test on the float value, the key formed only for staged candidates
  __device__ __forceinline__ void offer_f(float v, uint32_t id, bool valid) {
    bool pass = valid && v <= thr_f;
    uint64_t m = __ballot(pass);
    if (m == 0) return;
    int cnt = __popcll(m);
    if (nstage + cnt > 64) {
      flush();
      pass = valid && v <= thr_f;
      m = __ballot(pass);
      if (m == 0) return;
      cnt = __popcll(m);
    }
    if (pass) stage[nstage + mbcnt64(m)] = make_key(v, id);
    nstage += cnt;
  }

  // After finish(), lane i holds the i-th smallest key (KEY_NONE padded).
  __device__ __forceinline__ void finish() { flush(); }

  __device__ __forceinline__ void tighten(uint64_t b) {
    if (b < bound) bound = b;
    if (b < thr) thr = b;
    thr_f = key_ceil(thr);
  }
  __device__ __forceinline__ uint64_t cth() const { return lane_u64(best, C - 1); }
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
  float thr_f;       // uniform: key_ceil(thr)
  int nstage;        // uniform
  int C;

  __device__ __forceinline__ void init(uint64_t* lds, int C_, uint64_t bound_ = KEY_NONE) {
    stage = lds;
    C = C_;
    nstage = 0;
    bound = bound_;
    thr = bound_;
    thr_f = key_ceil(thr);
#pragma unroll
    for (int r = 0; r < NR; ++r) best[r] = KEY_NONE;
  }

  __device__ __forceinline__ void flush() {
    if (nstage == 0) return;
    const int lane = lane_id();
    wave_sync();
    uint64_t k = lane < nstage ? stage[lane] : KEY_NONE;
    wave_sync();
    k = wave_sort64<true>(k);  // descending: the half-cleaner pairs it with the ascending list
    best[NR - 1] = best[NR - 1] < k ? best[NR - 1] : k;
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
      for (int r = 0; r < NR; ++r) best[r] = cmpx(best[r], j, lower);
    }
    const uint64_t t = cth();
    thr = t < bound ? t : bound;
    thr_f = key_ceil(thr);
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

  // as WaveTop64::offer_f
  __device__ __forceinline__ void offer_f(float v, uint32_t id, bool valid) {
    bool pass = valid && v <= thr_f;
    uint64_t m = __ballot(pass);
    if (m == 0) return;
    int cnt = __popcll(m);
    if (nstage + cnt > 64) {
      flush();
      pass = valid && v <= thr_f;
      m = __ballot(pass);
      if (m == 0) return;
      cnt = __popcll(m);
    }
    if (pass) stage[nstage + mbcnt64(m)] = make_key(v, id);
    nstage += cnt;
  }

  // After finish(), list element r * 64 + lane is best[r] (KEY_NONE padded).
  __device__ __forceinline__ void finish() { flush(); }

  // Keys merged into the sorted list so far (its valid prefix; uniform).
  __device__ __forceinline__ int merged() const {
    int n = 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) n += __popcll(__ballot(best[r] != KEY_NONE));
    return n;
  }

  // Element i < merged() + nstage of the list's keys without a flush: the
  // sorted ones first, then the staged arrivals in arrival order (KEY_NONE
  // past the end).  Call wave_sync() first (stage entries of other lanes).
  __device__ __forceinline__ uint64_t unsorted_at(int i, int r, int nm) const {
    if (i < nm) return best[r];
    return i < nm + nstage ? stage[i - nm] : KEY_NONE;
  }

  __device__ __forceinline__ void tighten(uint64_t b) {
    if (b < bound) bound = b;
    if (b < thr) thr = b;
    thr_f = key_ceil(thr);
  }
  // The C-th smallest key merged so far (KEY_NONE while fewer than C).
  __device__ __forceinline__ uint64_t cth() const {
    const int e = C - 1;
    uint64_t v = best[0];
#pragma unroll
    for (int r = 1; r < NR; ++r)
      if ((e >> 6) == r) v = best[r];
    return lane_u64(v, e & 63);
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
