// Grain bucketing of (query, probe) pairs.  Routing gives every query P grains;
// projection and scan run grain-major so that a grain's basis and Block-SoA
// codes are read once per tile of queries instead of once per query.
//
// A counting sort groups the pair ids q * P + slot by grain.  Inside a grain's
// range the pairs of probe slot 0 (each query's nearest grain) come first, so
// the scan can take slot 0 in a pass of its own whose results bound the other
// slots.  Three work-item lists are cut from the ranges without materialising
// them: per list L and grain g, lstart[L][g] / lcount[L][g] give the pairs, and
// the exclusive prefix ioff[L][g] of ceil(lcount / tile_L) numbers its items;
// a kernel finds the grain of item i by binary search in ioff.
#include <algorithm>

#include <atomic>

#include "hntl_device.h"
#include "hntl_internal.h"

namespace hntl {

namespace {

constexpr int CHUNK = 4096;      // pairs per workgroup
constexpr int LDS_MAX_G = 8192;  // grain counters kept in LDS up to this G (scatter: 4 G ints = 128 KiB)

__device__ __forceinline__ int probe_of(const int32_t* __restrict__ probes, int64_t p, int G) {
  const int g = probes[p];
  return (g >= 0 && g < G) ? g : -1;
}

// Per-grain pair counts, all slots and slot 0; counters live in LDS per
// workgroup and are added to the global ones once per (workgroup, grain).
__global__ __launch_bounds__(256) void bucket_hist_kernel(const int32_t* __restrict__ probes, int64_t npairs, int P,
                                                          int G, int32_t* __restrict__ gcount,
                                                          int32_t* __restrict__ gcount0) {
  extern __shared__ int lds_mem[];
  int* lc = lds_mem;
  int* lc0 = lds_mem + G;
  const bool lds = G <= LDS_MAX_G;
  if (lds) {
    for (int g = threadIdx.x; g < G; g += 256) {
      lc[g] = 0;
      lc0[g] = 0;
    }
    __syncthreads();
  }
  const int64_t p0 = (int64_t)blockIdx.x * CHUNK;
  for (int u = threadIdx.x; u < CHUNK; u += 256) {
    const int64_t p = p0 + u;
    if (p >= npairs) break;
    const int g = probe_of(probes, p, G);
    if (g < 0) continue;
    const bool s0 = (p % P) == 0;
    if (lds) {
      atomicAdd(&lc[g], 1);
      if (s0) atomicAdd(&lc0[g], 1);
    } else {
      atomicAdd(&gcount[g], 1);
      if (s0) atomicAdd(&gcount0[g], 1);
    }
  }
  if (!lds) return;
  __syncthreads();
  for (int g = threadIdx.x; g < G; g += 256) {
    if (lc[g]) atomicAdd(&gcount[g], lc[g]);
    if (lc0[g]) atomicAdd(&gcount0[g], lc0[g]);
  }
}

// Exclusive scan of one value per thread of a 1024-thread workgroup.
__device__ int block_exclusive_scan(int v, int* tmp /* >= 16 ints */, int& total) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) tmp[wave] = x;
  __syncthreads();
  int wsum = 0, all = 0;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; ++w) {
    const int t = tmp[w];
    if (w < wave) wsum += t;
    all += t;
  }
  __syncthreads();
  total = all;
  return wsum + x - v;
}

// Exclusive scan of four values per thread of a 1024-thread workgroup.
__device__ void block_exclusive_scan4(const int (&v)[4], int (&ex)[4], int (&total)[4], int (*tmp)[4]) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  int x[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    x[c] = v[c];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x[c], o, 64);
      if (lane >= o) x[c] += y;
    }
  }
  if (lane == 63)
#pragma unroll
    for (int c = 0; c < 4; ++c) tmp[wave][c] = x[c];
  __syncthreads();
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    int wsum = 0, all = 0;
    for (int w = 0; w < nw; ++w) {
      const int t = tmp[w][c];
      if (w < wave) wsum += t;
      all += t;
    }
    ex[c] = wsum + x[c] - v[c];
    total[c] = all;
  }
  __syncthreads();
}

// Single workgroup: grain starts (gstart) and the three lists' item offsets.
// Grains are visited in the order `gorder` (rank -> grain; identity if null)
// and ioff is indexed by that rank, so items come out in that order; the
// per-grain list ranges (lstart, lcount, indexed by grain) follow from gstart
// in bucket_lists_kernel.  With `nsplit`, a grain's slot-0 and rest
// tiles each become nsplit[g] items (one per block range of the grain).
// Thread t owns the consecutive ranks t * per .. t * per + per - 1: a local
// pass sums its pairs and items, one workgroup scan turns the sums into
// offsets, a second local pass writes them.
__global__ __launch_bounds__(1024) void bucket_scan_kernel(const int32_t* __restrict__ gcount,
                                                           const int32_t* __restrict__ gcount0, int G,
                                                           const int32_t* __restrict__ gorder,
                                                           const int32_t* __restrict__ nsplit,
                                                           int32_t* __restrict__ gstart, ItemLists lists) {
  __shared__ int tmp[16][4];
  const int per = (G + (int)blockDim.x - 1) / (int)blockDim.x;
  const int r0 = (int)threadIdx.x * per;
  const int t0 = lists.tile[LIST_SLOT0], t1 = lists.tile[LIST_REST], t2 = lists.tile[LIST_ALL];
  // up to SCAN_REG ranks per thread (G <= 8,192): every load of a thread's ranks
  // is issued before any is used, and the values stay in registers for the
  // second pass (no chains of dependent loads)
  constexpr int SCAN_REG = 8;
  const bool reg = per <= SCAN_REG;
  int gg[SCAN_REG], cc[SCAN_REG], c0s[SCAN_REG], sp[SCAN_REG];
  if (reg) {
#pragma unroll
    for (int i = 0; i < SCAN_REG; ++i) {
      const int rank = r0 + i;
      gg[i] = (i < per && rank < G) ? (gorder ? gorder[rank] : rank) : -1;
    }
#pragma unroll
    for (int i = 0; i < SCAN_REG; ++i) {
      const int g = gg[i];
      cc[i] = g >= 0 ? gcount[g] : 0;
      c0s[i] = g >= 0 ? gcount0[g] : 0;
      sp[i] = g >= 0 ? (nsplit ? nsplit[g] : 1) : 0;
    }
  }
  auto fetch = [&](int i, int& g, int& c, int& c0, int& split) -> bool {
    const int rank = r0 + i;
    if (i >= per || rank >= G) return false;
    if (reg && i < SCAN_REG) {
      g = gg[i];
      c = cc[i];
      c0 = c0s[i];
      split = sp[i];
    } else {
      g = gorder ? gorder[rank] : rank;
      c = gcount[g];
      c0 = gcount0[g];
      split = nsplit ? nsplit[g] : 1;
    }
    return true;
  };
  int loc[4] = {0, 0, 0, 0};  // pairs, items of slot 0, of the rest, of all
  for (int i = 0; i < per; ++i) {
    int g, c, c0, split;
    if (!fetch(i, g, c, c0, split)) break;
    loc[0] += c;
    loc[1] += (c0 + t0 - 1) / t0 * split;
    loc[2] += (c - c0 + t1 - 1) / t1 * split;
    loc[3] += (c + t2 - 1) / t2;
  }
  int run[4], tot[4];
  block_exclusive_scan4(loc, run, tot, tmp);
  for (int i = 0; i < per; ++i) {
    int g, c, c0, split;
    if (!fetch(i, g, c, c0, split)) break;
    const int rank = r0 + i;
    gstart[g] = run[0];  // the other per-grain fields: bucket_lists_kernel, many workgroups
    lists.ioff[LIST_SLOT0][rank] = run[1];
    lists.ioff[LIST_REST][rank] = run[2];
    lists.ioff[LIST_ALL][rank] = run[3];
    run[0] += c;
    run[1] += (c0 + t0 - 1) / t0 * split;
    run[2] += (c - c0 + t1 - 1) / t1 * split;
    run[3] += (c + t2 - 1) / t2;
  }
  if (threadIdx.x == 0) {
    lists.ioff[LIST_SLOT0][G] = tot[1];
    lists.ioff[LIST_REST][G] = tot[2];
    lists.ioff[LIST_ALL][G] = tot[3];
  }
}

// Per-grain list ranges from the grain starts (one thread per grain): these
// scattered writes are spread over many workgroups instead of the scan's one.
__global__ __launch_bounds__(256) void bucket_lists_kernel(const int32_t* __restrict__ gcount,
                                                           const int32_t* __restrict__ gcount0, int G,
                                                           const int32_t* __restrict__ gstart,
                                                           int32_t* __restrict__ cur0, int32_t* __restrict__ cur1,
                                                           ItemLists lists) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= G) return;
  const int c = gcount[g], c0 = gcount0[g], st = gstart[g];
  cur0[g] = 0;
  cur1[g] = 0;
  lists.lstart[LIST_SLOT0][g] = st;
  lists.lcount[LIST_SLOT0][g] = c0;
  lists.lstart[LIST_REST][g] = st + c0;
  lists.lcount[LIST_REST][g] = c - c0;
  lists.lstart[LIST_ALL][g] = st;
  lists.lcount[LIST_ALL][g] = c;
}

// Scatter pair ids into their grain's range (slot 0 first): each workgroup
// reserves one run per grain and kind with a single global atomic, then ranks
// its pairs with LDS atomics.  The order inside a grain's run is not fixed;
// every consumer writes its results by pair id, so outputs do not depend on it.
__global__ __launch_bounds__(256) void bucket_scatter_kernel(const int32_t* __restrict__ probes, int64_t npairs,
                                                             int P, int G, const int32_t* __restrict__ gstart,
                                                             const int32_t* __restrict__ gcount0,
                                                             int32_t* __restrict__ cur0, int32_t* __restrict__ cur1,
                                                             int32_t* __restrict__ order) {
  extern __shared__ int lds_mem[];
  const bool lds = G <= LDS_MAX_G;
  const int64_t p0 = (int64_t)blockIdx.x * CHUNK;
  if (!lds) {
    for (int u = threadIdx.x; u < CHUNK; u += 256) {
      const int64_t p = p0 + u;
      if (p >= npairs) break;
      const int g = probe_of(probes, p, G);
      if (g < 0) continue;
      const int pos = (p % P) == 0 ? gstart[g] + atomicAdd(&cur0[g], 1)
                                   : gstart[g] + gcount0[g] + atomicAdd(&cur1[g], 1);
      order[pos] = (int32_t)p;
    }
    return;
  }
  int* n0 = lds_mem;
  int* n1 = lds_mem + G;
  int* b0 = lds_mem + 2 * G;
  int* b1 = lds_mem + 3 * G;
  for (int g = threadIdx.x; g < G; g += 256) {
    n0[g] = 0;
    n1[g] = 0;
  }
  __syncthreads();
  for (int u = threadIdx.x; u < CHUNK; u += 256) {
    const int64_t p = p0 + u;
    if (p >= npairs) break;
    const int g = probe_of(probes, p, G);
    if (g >= 0) atomicAdd((p % P) == 0 ? &n0[g] : &n1[g], 1);
  }
  __syncthreads();
  for (int g = threadIdx.x; g < G; g += 256) {
    b0[g] = n0[g] ? gstart[g] + atomicAdd(&cur0[g], n0[g]) : 0;
    b1[g] = n1[g] ? gstart[g] + gcount0[g] + atomicAdd(&cur1[g], n1[g]) : 0;
    n0[g] = 0;
    n1[g] = 0;
  }
  __syncthreads();
  for (int u = threadIdx.x; u < CHUNK; u += 256) {
    const int64_t p = p0 + u;
    if (p >= npairs) break;
    const int g = probe_of(probes, p, G);
    if (g < 0) continue;
    const int pos = (p % P) == 0 ? b0[g] + atomicAdd(&n0[g], 1) : b1[g] + atomicAdd(&n1[g], 1);
    order[pos] = (int32_t)p;
  }
}

// Per-pair list slots when grains are split into block ranges: pair
// (q, slot) of grain g owns the nsplit[g] consecutive lists from lbase[pair];
// a query's lists are contiguous, qoff[q] .. qoff[q + 1].  Three passes: the
// lists of each query (one thread per query), an exclusive scan over the
// queries (one workgroup, each thread a contiguous run), the per-slot bases
// (one thread per query).
__global__ __launch_bounds__(256) void query_lists_kernel(const int32_t* __restrict__ probes, int64_t nq, int P,
                                                          int G, const int32_t* __restrict__ nsplit,
                                                          int32_t* __restrict__ qoff) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  int tot = 0;
  for (int sl = 0; sl < P; ++sl) {
    const int g = probes[q * P + sl];
    tot += (g >= 0 && g < G) ? nsplit[g] : 0;
  }
  qoff[q] = tot;
}

__global__ __launch_bounds__(1024) void query_scan_kernel(int64_t nq, int32_t* __restrict__ qoff) {
  __shared__ int tmp[32];
  const int64_t per = (nq + (int64_t)blockDim.x - 1) / (int64_t)blockDim.x;
  const int64_t q0 = (int64_t)threadIdx.x * per;
  const int64_t q1 = q0 + per < nq ? q0 + per : nq;
  // up to QREG queries per thread (nq <= 16,384): all loads issued at once and
  // kept in registers for the second pass
  constexpr int QREG = 16;
  int sum = 0;
  if (per <= QREG) {
    int v[QREG];
#pragma unroll
    for (int i = 0; i < QREG; ++i) v[i] = q0 + i < q1 ? qoff[q0 + i] : 0;
#pragma unroll
    for (int i = 0; i < QREG; ++i) sum += v[i];
    int all;
    int run = block_exclusive_scan(sum, tmp, all);
#pragma unroll
    for (int i = 0; i < QREG; ++i)
      if (q0 + i < q1) {
        qoff[q0 + i] = run;
        run += v[i];
      }
    if (threadIdx.x == 0) qoff[nq] = all;
    return;
  }
  for (int64_t q = q0; q < q1; ++q) sum += qoff[q];
  int all;
  int run = block_exclusive_scan(sum, tmp, all);
  for (int64_t q = q0; q < q1; ++q) {
    const int v = qoff[q];
    qoff[q] = run;
    run += v;
  }
  if (threadIdx.x == 0) qoff[nq] = all;
}

__global__ __launch_bounds__(256) void pair_lists_kernel(const int32_t* __restrict__ probes, int64_t nq, int P,
                                                         int G, const int32_t* __restrict__ nsplit,
                                                         const int32_t* __restrict__ qoff,
                                                         int32_t* __restrict__ lbase) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  int run = qoff[q];
  for (int sl = 0; sl < P; ++sl) {
    const int g = probes[q * P + sl];
    lbase[q * P + sl] = run;
    run += (g >= 0 && g < G) ? nsplit[g] : 0;
  }
}

__global__ void fill_i32_kernel(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void fill_multi_kernel(FillList L) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int k = 0; k < L.n; ++k)
    if (i < L.seg[k].n) L.seg[k].p[i] = L.seg[k].v;
}

}  // namespace

// Fill with a kernel rather than hipMemsetAsync, so that captured graphs hold
// only kernel nodes.
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  HIP_TRY(hipGetLastError());
}

void launch_fill_multi(const FillList& L, hipStream_t s) {
  int64_t n = 0;
  for (int k = 0; k < L.n; ++k) n = std::max<int64_t>(n, L.seg[k].n);
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_multi_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, L);
  HIP_TRY(hipGetLastError());
}

namespace {
// Largest rank with ioff[rank] <= item (ioff[G] > item).
__device__ __forceinline__ int item_rank(const int32_t* __restrict__ ioff, int G, int item) {
  int lo = 0, hi = G;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ioff[mid] <= item)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void item_table_kernel(ItemLists lists, const int32_t* __restrict__ gorder, int G,
                                                         int qt, int64_t max_items, ItemDesc* __restrict__ out) {
  const int64_t it64 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (it64 >= max_items) return;
  const int it = (int)it64;
  const int nP = lists.ioff[LIST_ALL][G], n0 = lists.ioff[LIST_SLOT0][G], n1 = lists.ioff[LIST_REST][G];
  if (it >= nP + n0 + n1) return;
  ItemDesc d{};
  if (it < nP) {
    const int rank = item_rank(lists.ioff[LIST_ALL], G, it);
    const int g = gorder ? gorder[rank] : rank;
    const int tp = lists.tile[LIST_ALL];
    const int first = (it - lists.ioff[LIST_ALL][rank]) * tp;
    d.g = g;
    d.off = lists.lstart[LIST_ALL][g] + first;
    d.cnt = min(tp, lists.lcount[LIST_ALL][g] - first);
    d.c0 = d.c1 = it;
  } else {
    const int L = it < nP + n0 ? LIST_SLOT0 : LIST_REST;
    const int li = it - (L == LIST_SLOT0 ? nP : nP + n0);
    const int rank = item_rank(lists.ioff[L], G, li);
    const int g = gorder ? gorder[rank] : rank;
    const int lc = lists.lcount[L][g];
    const int ntiles = (lc + qt - 1) / qt;
    const int k = li - lists.ioff[L][rank];
    const int tile = k % ntiles;  // range-major: a range's tiles run together
    const int first = tile * qt;
    d.g = g;
    d.range = k / ntiles;
    d.off = lists.lstart[L][g] + first;
    d.cnt = min(qt, lc - first);
    // a grain's projection list is its slot-0 pairs followed by the others, in
    // 16-pair items when the fused kernel projects (the only reader of c0 / c1):
    // this tile's pairs lie in items c0 .. c1 (at most two)
    const int base = (L == LIST_SLOT0 ? 0 : lists.lcount[LIST_SLOT0][g]) + first;
    const int pi0 = lists.ioff[LIST_ALL][rank];
    d.c0 = pi0 + base / 16;
    d.c1 = pi0 + (base + d.cnt - 1) / 16;
  }
  out[it] = d;
}
}  // namespace

void launch_item_table(const ItemLists& lists, const int32_t* gorder, int G, int qt, int64_t max_items,
                       ItemDesc* out, hipStream_t s) {
  if (max_items <= 0) return;
  hipLaunchKernelGGL(item_table_kernel, dim3((unsigned)((max_items + 255) / 256)), dim3(256), 0, s, lists, gorder, G,
                     qt, max_items, out);
  HIP_TRY(hipGetLastError());
}

void launch_pair_lists(const int32_t* probes, int64_t nq, int P, int G, const int32_t* nsplit, int32_t* lbase,
                       int32_t* qoff, hipStream_t s) {
  if (nq <= 0) return;
  const dim3 grid((unsigned)((nq + 255) / 256));
  hipLaunchKernelGGL(query_lists_kernel, grid, dim3(256), 0, s, probes, nq, P, G, nsplit, qoff);
  hipLaunchKernelGGL(query_scan_kernel, dim3(1), dim3(1024), 0, s, nq, qoff);
  hipLaunchKernelGGL(pair_lists_kernel, grid, dim3(256), 0, s, probes, nq, P, G, nsplit, qoff, lbase);
  HIP_TRY(hipGetLastError());
}

void launch_bucket(const int32_t* probes, int64_t nq, int P, int G, Buckets& b, hipStream_t s,
                   const int32_t* gorder, const int32_t* nsplit, bool counts_zeroed) {
  const int64_t npairs = nq * P;
  if (!counts_zeroed) {
    FillList f{};
    f.seg[0] = FillSeg{b.gcount, G, 0};
    f.seg[1] = FillSeg{b.gcount0, G, 0};
    f.n = 2;
    launch_fill_multi(f, s);
  }
  const unsigned nb = (unsigned)((npairs + CHUNK - 1) / CHUNK);
  if (npairs > 0) {
    hipLaunchKernelGGL(bucket_hist_kernel, dim3(nb), dim3(256), G <= LDS_MAX_G ? 2 * G * sizeof(int) : 0, s,
                       probes, npairs, P, G, b.gcount, b.gcount0);
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(bucket_scan_kernel, dim3(1), dim3(1024), 0, s, b.gcount, b.gcount0, G, gorder, nsplit, b.gstart,
                     b.lists);
  hipLaunchKernelGGL(bucket_lists_kernel, dim3((unsigned)((G + 255) / 256)), dim3(256), 0, s, b.gcount, b.gcount0, G,
                     b.gstart, b.cur0, b.cur1, b.lists);
  HIP_TRY(hipGetLastError());
  if (npairs > 0) {
    const size_t lds = G <= LDS_MAX_G ? 4 * (size_t)G * sizeof(int) : 0;
    // up to 128 KiB of dynamic LDS (gfx950 has 160 KiB per CU), allowed once per device
    static std::atomic<bool> lds_set[64];
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64 || !lds_set[dev].load()) {
      HIP_TRY(hipFuncSetAttribute((const void*)bucket_scatter_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(4 * LDS_MAX_G * sizeof(int))));
      if (dev >= 0 && dev < 64) lds_set[dev].store(true);
    }
    hipLaunchKernelGGL(bucket_scatter_kernel, dim3(nb), dim3(256), lds, s, probes, npairs, P, G, b.gstart, b.gcount0,
                       b.cur0, b.cur1, b.order);
    HIP_TRY(hipGetLastError());
  }
}

}  // namespace hntl
