// Incremental segments: a new index = an existing one plus appended rows
// (Section 1 and the segment layer of Section 2, Fig. 1).  Grains are
// self-contained, so a new row changes only the grain it joins: it is routed
// to the nearest stored centroid and encoded with that grain's stored mu_g and
// W_g (eq. 1-4); every other grain, and every existing code, is copied as is.
// The base index is never written (segments are immutable); the result owns
// all of its memory.
//
// Oversized grains (more than split_max members after the append) are cut
// into m = ceil(n / split_max) children along their leading local principal
// axis: members ordered by the stored FP32 first code coordinate (ties by id),
// cut into m runs of sizes differing by at most one.  Child 0 keeps the
// grain's number, the others are numbered G, G + 1, ... in ascending order of
// the grains split.  Children get exact FP64 member means, their own local
// PCA bases and codes from the build's kernels.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "hntl_device.h"
#include "hntl_internal.h"

namespace hntl {
namespace {

constexpr int64_t SRC_PAD = -1;   // padding lane: zero codes, eps = +inf
constexpr int64_t SRC_SKIP = -2;  // written by the split grains' encode
// src <= -3: new row -3 - src;  src >= 0: slot (block * B + lane) of the base

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Codes of the new rows with their grain's stored centroid and basis, FP64
// arithmetic from the FP32 values: x' = x - mu_g (eq. 1), z = W_g^T x' (eq. 2),
// e = x' - W_g z (eq. 3), eps = ||e||^2 (eq. 4).  One workgroup per row; wave
// w computes the coordinates j = w, w + 4, ... and every thread the residual
// of its own columns k.
__global__ __launch_bounds__(256) void append_encode_kernel(const float* __restrict__ X, int d, int r,
                                                            const int32_t* __restrict__ lab,
                                                            const float* __restrict__ mu,
                                                            const float* __restrict__ basis, float* __restrict__ zout,
                                                            float* __restrict__ eout) {
  __shared__ double zs[HNTL_MAX_R];
  __shared__ double part[4];
  const int64_t i = blockIdx.x;
  const int g = lab[i];
  const float* x = X + (size_t)i * d;
  const float* m = mu + (size_t)g * d;
  const float* W = basis + (size_t)g * r * d;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int j = w; j < r; j += 4) {
    double acc = 0.0;
    for (int k = lane; k < d; k += 64) acc = fma((double)W[(size_t)j * d + k], (double)x[k] - (double)m[k], acc);
    acc = wave_sum_f64(acc);
    if (lane == 0) {
      zs[j] = acc;
      zout[(size_t)i * r + j] = (float)acc;
    }
  }
  __syncthreads();
  double e2 = 0.0;
  for (int k = threadIdx.x; k < d; k += 256) {
    double e = (double)x[k] - (double)m[k];
    for (int j = 0; j < r; ++j) e -= (double)W[(size_t)j * d + k] * zs[j];
    e2 = fma(e, e, e2);
  }
  e2 = wave_sum_f64(e2);
  if (lane == 0) part[w] = e2;
  __syncthreads();
  if (threadIdx.x == 0) eout[i] = (float)(part[0] + part[1] + part[2] + part[3]);
}

// Block-SoA codes and eps of the new layout, one thread per slot (block * B +
// lane), from the base's blocks or the new rows' codes (see SRC_*).
__global__ __launch_bounds__(256) void relayout_kernel(const int64_t* __restrict__ src, int64_t nslots, int r, int rp,
                                                       const float* __restrict__ codes0,
                                                       const float* __restrict__ eps0, const float* __restrict__ zn,
                                                       const float* __restrict__ en, float* __restrict__ codes,
                                                       float* __restrict__ eps) {
  const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (slot >= nslots) return;
  const int64_t sv = src[slot];
  if (sv == SRC_SKIP) return;
  const int64_t blk = slot / B, lane = slot % B;
  float* c = codes + (size_t)blk * rp * B + lane;
  if (sv >= 0) {
    const int64_t bb = sv / B, bl = sv % B;
    const float* c0 = codes0 + (size_t)bb * rp * B + bl;
    for (int j = 0; j < rp; ++j) c[(size_t)j * B] = c0[(size_t)j * B];
    eps[slot] = eps0[sv];
  } else if (sv == SRC_PAD) {
    for (int j = 0; j < rp; ++j) c[(size_t)j * B] = 0.f;
    eps[slot] = __builtin_inff();
  } else {
    const int64_t row = -3 - sv;
    for (int j = 0; j < rp; ++j) c[(size_t)j * B] = j < r ? zn[(size_t)row * r + j] : 0.f;
    eps[slot] = en[row];
  }
}

__global__ void gather_f32_kernel(const float* __restrict__ v, const int64_t* __restrict__ idx, int64_t n,
                                  float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = v[idx[i]];
}

struct Frees {
  std::vector<void*> p;
  template <class T>
  T* get(size_t n) {
    T* q = dev_alloc<T>(nullptr, n);
    p.push_back(q);
    return q;
  }
  ~Frees() {
    for (void* q : p) (void)hipFree(q);
  }
};

template <class T>
T* upload_to(Index* ix, const std::vector<T>& v, hipStream_t s) {
  T* d = dev_alloc<T>(ix, v.size());
  if (!v.empty()) HIP_TRY(hipMemcpyAsync(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
  return d;
}

}  // namespace
}  // namespace hntl

using namespace hntl;

extern "C" hntl_status hntl_index_append(const hntl_index* base, const float* X, uint64_t n,
                                         const hntl_append_params* params, void* stream, hntl_index** out) {
  set_error("");
  if (!out) return fail(HNTL_EINVAL, "out is NULL");
  *out = nullptr;
  if (!base) return fail(HNTL_EINVAL, "base is NULL");
  if (n > 0 && !X) return fail(HNTL_EINVAL, "X is NULL");
  const Index& b = base->ix;
  const uint64_t N = b.N, N2 = b.N + n;
  const uint32_t d = b.d, G = b.G, r = b.r, rp = b.rp;
  if (N2 >= (1ull << 31)) return fail(HNTL_EUNSUPPORTED, "N + n must be below 2^31");
  const uint32_t split_max = params ? params->split_max : 0;
  const uint32_t eig_iters = params && params->eig_iters ? params->eig_iters : 40;
  const uint64_t seed = params ? params->seed : 0;
  if (split_max > 0 && !b.X)
    return fail(HNTL_EUNSUPPORTED, "splitting grains needs the raw vectors of the base index");
  hipStream_t s = (hipStream_t)stream;
  hntl_index* h = nullptr;
  try {
    h = new hntl_index();
    Index* ix = &h->ix;
    Frees tmp;
    ix->device = b.device;
    ix->N = N2;
    ix->d = d;
    ix->r = r;
    ix->rp = rp;
    ix->kmeans_iters_run = b.kmeans_iters_run;

    // ---------------- the new rows: raw vectors, grains, codes
    const float* Xn = nullptr;
    if (b.X) {
      ix->X = dev_alloc<float>(ix, (size_t)N2 * d);
      HIP_TRY(hipMemcpyAsync(ix->X, b.X, sizeof(float) * N * d, hipMemcpyDeviceToDevice, s));
      if (n) HIP_TRY(hipMemcpyAsync(ix->X + (size_t)N * d, X, sizeof(float) * n * d, hipMemcpyDefault, s));
      Xn = ix->X + (size_t)N * d;
    } else if (n) {
      float* t = tmp.get<float>((size_t)n * d);
      HIP_TRY(hipMemcpyAsync(t, X, sizeof(float) * n * d, hipMemcpyDefault, s));
      Xn = t;
    }
    std::vector<int32_t> lab(n);
    float* zn = tmp.get<float>((size_t)std::max<uint64_t>(n, 1) * r);
    float* en = tmp.get<float>(std::max<uint64_t>(n, 1));
    if (n) {
      float* xn = tmp.get<float>(n);
      int32_t* dl = tmp.get<int32_t>(n);
      launch_row_norms(Xn, (int64_t)n, (int)d, xn, s);
      launch_argmin_rows(Xn, xn, (int64_t)n, b.centroids, b.cnorm, (int)G, (int)d, dl, nullptr, s);
      hipLaunchKernelGGL(append_encode_kernel, dim3((unsigned)n), dim3(256), 0, s, Xn, (int)d, (int)r, dl,
                         b.centroids, b.basis, zn, en);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpyAsync(lab.data(), dl, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    }
    std::vector<int32_t> perm0(N);
    HIP_TRY(hipMemcpyAsync(perm0.data(), b.perm, sizeof(int32_t) * N, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<std::vector<int32_t>> newrows(G);  // new row numbers (0 .. n-1) per grain, ascending
    for (uint64_t i = 0; i < n; ++i) {
      if (lab[i] < 0 || (uint32_t)lab[i] >= G) throw HipError(hipErrorUnknown, "grain assignment out of range");
      newrows[lab[i]].push_back((int32_t)i);
    }
    auto old_n = [&](uint32_t g) { return b.offsets_h[g + 1] - b.offsets_h[g]; };

    // ---------------- splits
    std::vector<uint32_t> split;
    if (split_max > 0)
      for (uint32_t g = 0; g < G; ++g)
        if ((uint64_t)(old_n(g) + (int64_t)newrows[g].size()) > split_max) split.push_back(g);
    std::vector<std::vector<int32_t>> kids;  // children 1 .. m-1 of every split grain, in order
    std::vector<std::vector<int32_t>> child0(G);
    std::vector<int32_t> children;           // grain numbers to re-encode
    if (!split.empty()) {
      // first code coordinate of every member of the split grains
      std::vector<int64_t> idx_old, idx_new;
      for (uint32_t g : split) {
        for (int64_t i = 0; i < old_n(g); ++i) idx_old.push_back(((int64_t)b.boff_h[g] + i / B) * rp * B + i % B);
        for (int32_t row : newrows[g]) idx_new.push_back((int64_t)row * r);
      }
      std::vector<float> t_old(idx_old.size()), t_new(idx_new.size());
      auto gather = [&](const float* v, const std::vector<int64_t>& idx, std::vector<float>& dst) {
        if (idx.empty()) return;
        int64_t* di = tmp.get<int64_t>(idx.size());
        float* dv = tmp.get<float>(idx.size());
        HIP_TRY(hipMemcpyAsync(di, idx.data(), sizeof(int64_t) * idx.size(), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(gather_f32_kernel, dim3((unsigned)((idx.size() + 255) / 256)), dim3(256), 0, s, v, di,
                           (int64_t)idx.size(), dv);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(dst.data(), dv, sizeof(float) * idx.size(), hipMemcpyDeviceToHost, s));
      };
      gather(b.codes, idx_old, t_old);
      gather(zn, idx_new, t_new);
      HIP_TRY(hipStreamSynchronize(s));
      size_t po = 0, pn = 0;
      uint32_t next = G;
      for (uint32_t g : split) {
        std::vector<std::pair<float, int32_t>> tv;
        for (int64_t i = 0; i < old_n(g); ++i) tv.emplace_back(t_old[po++], perm0[b.offsets_h[g] + i]);
        for (int32_t row : newrows[g]) tv.emplace_back(t_new[pn++], (int32_t)(N + row));
        std::sort(tv.begin(), tv.end());
        const int64_t ng = (int64_t)tv.size(), m = (ng + split_max - 1) / split_max;
        int64_t at = 0;
        for (int64_t k = 0; k < m; ++k) {
          const int64_t sz = ng / m + (k < ng % m ? 1 : 0);
          std::vector<int32_t> c;
          c.reserve(sz);
          for (int64_t q = at; q < at + sz; ++q) c.push_back(tv[q].second);
          at += sz;
          std::sort(c.begin(), c.end());
          if (k == 0) {
            child0[g] = std::move(c);
            children.push_back((int32_t)g);
          } else {
            kids.push_back(std::move(c));
          }
        }
      }
      for (size_t k = 0; k < kids.size(); ++k) children.push_back((int32_t)(next + k));
    }
    const uint32_t G2 = G + (uint32_t)kids.size();
    ix->G = G2;
    std::vector<char> is_split(G2, 0);
    for (int32_t g : children) is_split[g] = 1;

    // ---------------- grain order, block layout, slot sources
    std::vector<int64_t> off2(G2 + 1, 0);
    for (uint32_t g = 0; g < G2; ++g) {
      int64_t sz;
      if (g >= G) sz = (int64_t)kids[g - G].size();
      else if (is_split[g]) sz = (int64_t)child0[g].size();
      else sz = old_n(g) + (int64_t)newrows[g].size();
      off2[g + 1] = off2[g] + sz;
    }
    ix->offsets_h = off2;
    ix->boff_h.assign(G2 + 1, 0);
    uint32_t maxg = 0;
    for (uint32_t g = 0; g < G2; ++g) {
      const int64_t sz = off2[g + 1] - off2[g];
      maxg = std::max<uint32_t>(maxg, (uint32_t)sz);
      ix->boff_h[g + 1] = ix->boff_h[g] + (int32_t)((sz + B - 1) / B);
    }
    ix->max_grain = maxg;
    ix->nblocks = (uint64_t)ix->boff_h[G2];
    std::vector<int32_t> perm2(N2);
    std::vector<int64_t> src((size_t)ix->nblocks * B, SRC_PAD);
    for (uint32_t g = 0; g < G2; ++g) {
      const int64_t a = off2[g];
      const int64_t s0 = (int64_t)ix->boff_h[g] * B, s1 = (int64_t)ix->boff_h[g + 1] * B;
      if (is_split[g]) {
        const std::vector<int32_t>& c = g >= G ? kids[g - G] : child0[g];
        std::copy(c.begin(), c.end(), perm2.begin() + a);
        for (int64_t q = s0; q < s1; ++q) src[q] = SRC_SKIP;
        continue;
      }
      const int64_t no = old_n(g);
      for (int64_t i = 0; i < no; ++i) {
        perm2[a + i] = perm0[b.offsets_h[g] + i];
        src[s0 + i] = ((int64_t)b.boff_h[g] + i / B) * B + i % B;
      }
      for (size_t q = 0; q < newrows[g].size(); ++q) {
        perm2[a + no + (int64_t)q] = (int32_t)(N + newrows[g][q]);
        src[s0 + no + (int64_t)q] = -3 - (int64_t)newrows[g][q];
      }
    }
    std::vector<int32_t> goff32(G2 + 1);
    for (uint32_t g = 0; g <= G2; ++g) goff32[g] = (int32_t)off2[g];
    ix->goff = upload_to(ix, goff32, s);
    ix->boff = upload_to(ix, ix->boff_h, s);
    ix->perm = upload_to(ix, perm2, s);
    ix->codes = dev_alloc<float>(ix, (size_t)ix->nblocks * rp * B);
    ix->eps = dev_alloc<float>(ix, (size_t)ix->nblocks * B);
    ix->centroids = dev_alloc<float>(ix, (size_t)G2 * d);
    ix->basis = dev_alloc<float>(ix, (size_t)G2 * r * d);
    HIP_TRY(hipMemcpyAsync(ix->centroids, b.centroids, sizeof(float) * G * d, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(ix->basis, b.basis, sizeof(float) * G * r * d, hipMemcpyDeviceToDevice, s));
    {
      int64_t* dsrc = tmp.get<int64_t>(src.size());
      HIP_TRY(hipMemcpyAsync(dsrc, src.data(), sizeof(int64_t) * src.size(), hipMemcpyHostToDevice, s));
      const int64_t ns = (int64_t)src.size();
      if (ns > 0) {
        hipLaunchKernelGGL(relayout_kernel, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, s, dsrc, ns, (int)r,
                           (int)rp, b.codes, b.eps, zn, en, ix->codes, ix->eps);
        HIP_TRY(hipGetLastError());
      }
      HIP_TRY(hipStreamSynchronize(s));  // src and the host vectors above go out of scope
    }
    ix->captured.assign(G2, -1.0);
    if (b.captured.size() == G) std::copy(b.captured.begin(), b.captured.end(), ix->captured.begin());

    // ---------------- split grains: member means, local PCA, codes
    if (!children.empty()) {
      int64_t* d_off = tmp.get<int64_t>(G2 + 1);
      int* d_kids = tmp.get<int>(children.size());
      HIP_TRY(hipMemcpyAsync(d_off, off2.data(), sizeof(int64_t) * (G2 + 1), hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(d_kids, children.data(), sizeof(int) * children.size(), hipMemcpyHostToDevice, s));
      launch_segmented_mean(ix->X, (int)d, ix->perm, d_off, d_kids, (int)children.size(), ix->centroids, s);
      pca_encode_grains(ix, d_off, children, eig_iters, seed, (uint64_t)1 << 32, s);
    }
    ix->cnorm = dev_alloc<float>(ix, G2);
    launch_row_norms(ix->centroids, G2, (int)d, ix->cnorm, s);
    launch_grain_bounds(*ix, s);
    ix->codes_mask = b.codes_mask;
    if (ix->codes_mask & ~1u) launch_derive_lowp(*ix, s);
    HIP_TRY(hipStreamSynchronize(s));
  } catch (const ArgError& e) {
    delete h;
    return fail(e.code, e.msg);
  } catch (const HipError& e) {
    delete h;
    return fail(e.code == hipErrorOutOfMemory ? HNTL_ENOMEM : HNTL_EDEVICE, e.msg);
  } catch (const std::bad_alloc&) {
    delete h;
    return fail(HNTL_ENOMEM, "host allocation failed");
  }
  *out = h;
  return HNTL_OK;
}
