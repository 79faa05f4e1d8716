// Grain bucketing of (query, probe) pairs.  Routing gives every query P grains;
// projection and scan run grain-major so that a grain's basis and Block-SoA
// codes are read once per tile of queries instead of once per query.  This
// groups the pair ids by grain (counting sort) and cuts each grain's pairs
// into tiles (work items) of at most `tile` pairs.
#include "hntl_device.h"
#include "hntl_internal.h"

namespace hntl {

namespace {

__global__ void bucket_hist_kernel(const int32_t* __restrict__ probes, int64_t npairs, int G,
                                   int32_t* __restrict__ gcount) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const int g = probes[p];
  if (g >= 0 && g < G) atomicAdd(&gcount[g], 1);
}

// Exclusive scan of 1024 values held one per thread; returns the total.
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

// Single workgroup: grain start offsets, per-grain tiles, work-item list.
__global__ __launch_bounds__(1024) void bucket_scan_kernel(const int32_t* __restrict__ gcount, int G, int tile,
                                                           int max_items, int32_t* __restrict__ gstart,
                                                           int32_t* __restrict__ cursor, int32_t* __restrict__ items,
                                                           int32_t* __restrict__ nitems) {
  __shared__ int tmp[32];
  int carry_p = 0, carry_t = 0;
  for (int base = 0; base < G; base += 1024) {
    const int g = base + (int)threadIdx.x;
    const int c = g < G ? gcount[g] : 0;
    const int nt = (c + tile - 1) / tile;
    int tot_p, tot_t;
    const int sp = block_exclusive_scan(c, tmp, tot_p);
    const int st = block_exclusive_scan(nt, tmp, tot_t);
    if (g < G) {
      gstart[g] = carry_p + sp;
      cursor[g] = 0;
      for (int t = 0; t < nt; ++t) {
        const int it = carry_t + st + t;
        if (it < max_items) {
          items[2 * it] = g;
          items[2 * it + 1] = t * tile;
        }
      }
    }
    carry_p += tot_p;
    carry_t += tot_t;
  }
  if (threadIdx.x == 0) *nitems = carry_t < max_items ? carry_t : max_items;
}

__global__ void bucket_scatter_kernel(const int32_t* __restrict__ probes, int64_t npairs, int G,
                                      const int32_t* __restrict__ gstart, int32_t* __restrict__ cursor,
                                      int32_t* __restrict__ order) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npairs) return;
  const int g = probes[p];
  if (g < 0 || g >= G) return;
  const int pos = gstart[g] + atomicAdd(&cursor[g], 1);
  order[pos] = (int32_t)p;
}

}  // namespace

void launch_bucket(const int32_t* probes, int64_t npairs, int G, Buckets& b, hipStream_t s) {
  HIP_TRY(hipMemsetAsync(b.gcount, 0, sizeof(int32_t) * G, s));
  if (npairs > 0) {
    const unsigned nb = (unsigned)((npairs + 255) / 256);
    hipLaunchKernelGGL(bucket_hist_kernel, dim3(nb), dim3(256), 0, s, probes, npairs, G, b.gcount);
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(bucket_scan_kernel, dim3(1), dim3(1024), 0, s, b.gcount, G, b.tile, b.max_items, b.gstart,
                     b.cursor, b.items, b.nitems);
  HIP_TRY(hipGetLastError());
  if (npairs > 0) {
    const unsigned nb = (unsigned)((npairs + 255) / 256);
    hipLaunchKernelGGL(bucket_scatter_kernel, dim3(nb), dim3(256), 0, s, probes, npairs, G, b.gstart, b.cursor,
                       b.order);
    HIP_TRY(hipGetLastError());
  }
}

}  // namespace hntl
