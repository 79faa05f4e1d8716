// Scan dispatch by code form, and the per-grain code bounding boxes used by
// the exact pruning of the scan.
#include "hntl_device.h"
#include "hntl_internal.h"

namespace hntl {

void launch_scan_ct0(const Index&, const float*, const float*, int, int, const Buckets&, int, uint64_t*,
                     const uint64_t*, bool, unsigned long long*, hipStream_t);
void launch_scan_ct1(const Index&, const float*, const float*, int, int, const Buckets&, int, uint64_t*,
                     const uint64_t*, bool, unsigned long long*, hipStream_t);
void launch_scan_ct2(const Index&, const float*, const float*, int, int, const Buckets&, int, uint64_t*,
                     const uint64_t*, bool, unsigned long long*, hipStream_t);
void launch_scan_ct3(const Index&, const float*, const float*, int, int, const Buckets&, int, uint64_t*,
                     const uint64_t*, bool, unsigned long long*, hipStream_t);

namespace {

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

// Entry C - 1 of every query's probe-slot-0 list set to KEY_NONE: a list that
// no scan item writes (its probe is outside 0 .. G-1) then bounds nothing.
__global__ void reset_slot0_tail_kernel(uint64_t* __restrict__ part, int64_t nq, int P, int C) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nq) part[(size_t)q * P * C + C - 1] = KEY_NONE;
}

}  // namespace

void launch_reset_slot0_tail(uint64_t* part, int64_t nq, int P, int C, hipStream_t s) {
  if (nq <= 0) return;
  hipLaunchKernelGGL(reset_slot0_tail_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, part, nq, P, C);
  HIP_TRY(hipGetLastError());
}

void launch_scan(const Index& ix, int codes, const float* T, const float* epsq, int P, int C, const Buckets& b,
                 int list, uint64_t* part, const uint64_t* bound_lists, bool prune, unsigned long long* scored,
                 hipStream_t s) {
  if (b.max_items[list] <= 0) return;
  if (codes == HNTL_CODES_FP32)
    launch_scan_ct0(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s);
  else if (codes == HNTL_CODES_BF16)
    launch_scan_ct1(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s);
  else if (codes == HNTL_CODES_FP8_E4M3)
    launch_scan_ct2(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s);
  else
    launch_scan_ct3(ix, T, epsq, P, C, b, list, part, bound_lists, prune, scored, s);
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
