// Grain-major projection kernels (paper Section 2.2, eq. 1-4): a work item
// holds up to 16 NW pairs of one grain; wave w projects rows 16 w .. 16 w + 15,
// and the waves share the grain's basis through L2.
#include "project_impl.h"

namespace hntl {

namespace {

using namespace proj_detail;

// Items of PROJECT_TILE pairs run as workgroups of 8 waves; items of PT pairs
// (16) as single-wave workgroups, so the launch holds no idle wave slots when
// most grains have few pairs.
template <bool VEC, int NCT, int NW>
__global__ __launch_bounds__(64 * NW) void project_kernel(
    const float* __restrict__ Q, int d, int P, const float* __restrict__ centroids, const float* __restrict__ basis,
    int r, const int32_t* __restrict__ ioff, const int32_t* __restrict__ lstart, const int32_t* __restrict__ lcount,
    int G, const int32_t* __restrict__ gorder, const int32_t* __restrict__ order, float* __restrict__ T,
    float* __restrict__ epsq) {
  const int wave = threadIdx.x >> 6;
  int rank;
  if (!item_grain(ioff, G, blockIdx.x, rank)) return;
  const int g = gorder ? gorder[rank] : rank;
  const int first = (blockIdx.x - ioff[rank]) * (PT * NW) + PT * wave;  // within the grain's pairs
  const int cnt = min(PT, lcount[g] - first);
  if (cnt <= 0) return;  // no workgroup barrier in this kernel
  project_wave<VEC, NCT>(Q, d, P, centroids, basis, r, g, order + lstart[g] + first, cnt, T, epsq);
}

template <int NCT, int NW>
__global__ __launch_bounds__(64 * NW) void project_bf16_kernel(
    const float* __restrict__ Q, int d, int P, const float* __restrict__ centroids,
    const uint16_t* __restrict__ basis16, int r, const int32_t* __restrict__ ioff, const int32_t* __restrict__ lstart,
    const int32_t* __restrict__ lcount, int G, const int32_t* __restrict__ gorder, const int32_t* __restrict__ order,
    float* __restrict__ T, float* __restrict__ epsq) {
  const int wave = threadIdx.x >> 6;
  int rank;
  if (!item_grain(ioff, G, blockIdx.x, rank)) return;
  const int g = gorder ? gorder[rank] : rank;
  const int first = (blockIdx.x - ioff[rank]) * (PT * NW) + PT * wave;
  const int cnt = min(PT, lcount[g] - first);
  if (cnt <= 0) return;  // no workgroup barrier in this kernel
  project_wave_bf16<NCT>(Q, d, P, centroids, basis16, r, g, order + lstart[g] + first, cnt, T, epsq);
}

}  // namespace

template <bool BF16, bool VEC, int NCT, int NW>
void launch_project_k(const Index& ix, const float* Q, int P, const Buckets& b, float* T, float* epsq,
                      const int32_t* gorder, hipStream_t s) {
  const ItemLists& L = b.lists;
  const dim3 grid((unsigned)b.max_items[LIST_ALL]), block(64 * NW);
  if constexpr (BF16)
    hipLaunchKernelGGL((project_bf16_kernel<NCT, NW>), grid, block, 0, s, Q, (int)ix.d, P, ix.centroids,
                       ix.basis_bf16, (int)ix.r, L.ioff[LIST_ALL], L.lstart[LIST_ALL], L.lcount[LIST_ALL], (int)ix.G,
                       gorder, b.order, T, epsq);
  else
    hipLaunchKernelGGL((project_kernel<VEC, NCT, NW>), grid, block, 0, s, Q, (int)ix.d, P, ix.centroids, ix.basis,
                       (int)ix.r, L.ioff[LIST_ALL], L.lstart[LIST_ALL], L.lcount[LIST_ALL], (int)ix.G, gorder,
                       b.order, T, epsq);
}

template <bool BF16, bool VEC, int NW>
void launch_project_r(const Index& ix, const float* Q, int P, const Buckets& b, float* T, float* epsq,
                      const int32_t* gorder, hipStream_t s) {
  switch ((ix.r + 15) / 16) {
    case 1: launch_project_k<BF16, VEC, 1, NW>(ix, Q, P, b, T, epsq, gorder, s); break;
    case 2: launch_project_k<BF16, VEC, 2, NW>(ix, Q, P, b, T, epsq, gorder, s); break;
    case 3: launch_project_k<BF16, VEC, 3, NW>(ix, Q, P, b, T, epsq, gorder, s); break;
    default: launch_project_k<BF16, VEC, 4, NW>(ix, Q, P, b, T, epsq, gorder, s); break;
  }
}

template <bool BF16, bool VEC>
void launch_project_w(const Index& ix, const float* Q, int P, const Buckets& b, float* T, float* epsq,
                      const int32_t* gorder, hipStream_t s) {
  if (b.lists.tile[LIST_ALL] == PROJECT_TILE)
    launch_project_r<BF16, VEC, PROJECT_TILE / PT>(ix, Q, P, b, T, epsq, gorder, s);
  else if (b.lists.tile[LIST_ALL] == PT)
    launch_project_r<BF16, VEC, 1>(ix, Q, P, b, T, epsq, gorder, s);
  else
    throw ArgError{HNTL_EDEVICE, "projection item size must be 16 or PROJECT_TILE pairs"};
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
