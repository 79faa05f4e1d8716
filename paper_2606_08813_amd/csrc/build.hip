// Index build (paper Section 2.2): k-means grains, per-grain local PCA basis,
// codes and residual energies (eq. 1-4), packed into Block-SoA (Section 2.4).
//
// k-means (the paper leaves the partitioning method open; k-means is the
// reading used here):
//   * training rows: a counter-based random subset of at most
//     train_per_grain * G rows; seeding rows: the first 262,144 of them
//     (seeding on a few rows per grain often merges clusters)
//   * seeding: greedy k-means++ on the device: per centroid, 16 candidates
//     drawn by D^2 sampling, the one lowering the potential most is
//     kept (candidate distances on the MFMA distance kernel; sample /
//     potential / choose / apply kernels; uniforms come from a counter-based
//     SplitMix64 hash, so no host round trip is needed)
//   * Lloyd: nearest-centroid assignment on FP32 MFMA (ties to the lower
//     grain), centroid = FP64 mean of its members summed in a fixed order, an
//     empty grain re-seeded with the training row farthest from its centroid
//   * final: assignment of every row; centroid = exact FP64 member mean.
//
// Local PCA in FP64: covariance S_g = (1/n_g) sum (x - mu_g)(x - mu_g)^T by
// a grouped FP64 kernel, then block subspace iteration on S_g + delta_g I
// (delta_g = 1e-6 trace(S_g) keeps every iterate full rank without moving
// eigenvectors) with Cholesky-QR2 re-orthonormalisation, and a final
// Rayleigh-Ritz step (Jacobi eigensolver on the small projected matrix).  The
// batched FP64 GEMM/TRSM are library calls (rocBLAS), as are the batched
// Cholesky and the small Jacobi eigensolver (rocSOLVER).
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <numeric>

#include "hntl_device.h"
#include "hntl_internal.h"

namespace hntl {

void finish_index(Index* ix, const std::vector<int64_t>& off, const float* codes_go_host, const float* eps_go_host);

namespace {

// ------------------------------------------------------------ random numbers
// SplitMix64 finaliser (Steele, Lea & Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014) used as a counter-based hash.
__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ inline double u01(uint64_t seed, uint64_t stream, uint64_t i) {
  const uint64_t h = mix64(seed ^ mix64(stream * 0xD1B54A32D192ED03ull + i));
  return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

struct Blas {
  rocblas_handle h = nullptr;
  explicit Blas(hipStream_t s) {
    if (rocblas_create_handle(&h) != rocblas_status_success) throw HipError(hipErrorUnknown, "rocblas_create_handle");
    rocblas_set_stream(h, s);
  }
  ~Blas() {
    if (h) rocblas_destroy_handle(h);
  }
};

void rb(rocblas_status st, const char* what) {
  if (st != rocblas_status_success)
    throw HipError(hipErrorUnknown, std::string(what) + " failed: " + rocblas_status_to_string(st));
}

// ----------------------------------------------------------------- kernels
__global__ void gather_rows_kernel(const float* __restrict__ X, int d, const int32_t* __restrict__ rows, int64_t n,
                                   float* __restrict__ out) {
  const int64_t i = blockIdx.x;
  if (i >= n) return;
  const float* src = X + (size_t)rows[i] * d;
  float* dst = out + (size_t)i * d;
  for (int j = threadIdx.x; j < d; j += blockDim.x) dst[j] = src[j];
}

// Greedy k-means++ seeding (Arthur & Vassilvitskii 2007, with several
// sampled candidates per step and the one that lowers the potential most kept).
// State: closest[i] = squared distance of seeding row i to its nearest chosen
// centroid; partial[blk] = sum of closest over 256-row blocks (FP64).
constexpr int KPP_MAXL = 16;

// Per-block potentials potpart[blk][t] = sum_i min(closest[i], dcand[i][t])
// over 256-row blocks, from the candidate distances dcand (n x L, computed by
// the MFMA distance kernel).
__global__ __launch_bounds__(256) void kpp_pot_kernel(int64_t n, int L, const float* __restrict__ dcand,
                                                      const float* __restrict__ closest, int first,
                                                      double* __restrict__ potpart) {
  __shared__ double red[4][KPP_MAXL];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const float ci = (i < n && !first) ? closest[i] : __builtin_inff();
#pragma unroll
  for (int t = 0; t < KPP_MAXL; ++t) {
    if (t < L) {
      const double v = i < n ? (double)fminf(ci, dcand[(size_t)i * L + t]) : 0.0;
      const double w = wave_sum_d(v);
      if (lane == 0) red[wave][t] = w;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < L)
    potpart[(size_t)blockIdx.x * L + threadIdx.x] =
        red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

// Single workgroup: the candidate with the lowest potential (ties to the lower
// candidate slot) becomes centroid `step`.
__global__ __launch_bounds__(64) void kpp_choose_kernel(const float* __restrict__ Xs, int d,
                                                        const int32_t* __restrict__ cand, int L,
                                                        const double* __restrict__ potpart, int nblk,
                                                        int32_t* __restrict__ tstar, float* __restrict__ cent,
                                                        int step) {
  __shared__ int best_t;
  // potential of each candidate: the 64 lanes sum strided block partials, then
  // a butterfly reduction (fixed order, so the choice is reproducible)
  double acc[KPP_MAXL];
#pragma unroll
  for (int t = 0; t < KPP_MAXL; ++t) acc[t] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64)
#pragma unroll
    for (int t = 0; t < KPP_MAXL; ++t)
      if (t < L) acc[t] += potpart[(size_t)b * L + t];
#pragma unroll
  for (int t = 0; t < KPP_MAXL; ++t) acc[t] = wave_sum_d(acc[t]);
  if (threadIdx.x == 0) {
    double best = 0.0;
    int bt = 0;
    for (int t = 0; t < L; ++t)
      if (t == 0 || acc[t] < best) {
        best = acc[t];
        bt = t;
      }
    best_t = bt;
    *tstar = bt;
  }
  __syncthreads();
  const float* src = Xs + (size_t)cand[best_t] * d;
  for (int j = threadIdx.x; j < d; j += blockDim.x) cent[(size_t)step * d + j] = src[j];
}

// closest[i] = min(closest[i], dcand[i][t*]); per-block sums of closest.
__global__ __launch_bounds__(256) void kpp_apply_kernel(int64_t n, int L, const float* __restrict__ dcand,
                                                        const int32_t* __restrict__ tstar, int first,
                                                        float* __restrict__ closest, double* __restrict__ partial) {
  __shared__ double red[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    const float dc = dcand[(size_t)i * L + *tstar];
    const float c = first ? dc : fminf(closest[i], dc);
    closest[i] = c;
    v = (double)c;
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Single workgroup: L candidates sampled with probability proportional to
// closest[] (thread t draws candidate t from uniform u[t]).
__global__ __launch_bounds__(64) void kpp_sample_kernel(int64_t n, const float* __restrict__ closest,
                                                        const double* __restrict__ partial, int nblk,
                                                        const double* __restrict__ u, int L,
                                                        int32_t* __restrict__ cand) {
  const int t = threadIdx.x;
  if (t >= L) return;
  double tot = 0.0;
  for (int b = 0; b < nblk; ++b) tot += partial[b];
  int64_t pick = (int64_t)(u[t] * (double)n);
  if (tot > 0.0) {
    const double target = u[t] * tot;
    double run = 0.0;
    int b = 0;
    for (; b < nblk - 1; ++b) {
      if (run + partial[b] > target) break;
      run += partial[b];
    }
    const int64_t lo = (int64_t)b * 256, hi = n < lo + 256 ? n : lo + 256;
    pick = hi - 1;
    for (int64_t i = lo; i < hi; ++i) {
      run += (double)closest[i];
      if (run > target) {
        pick = i;
        break;
      }
    }
  }
  if (pick >= n) pick = n - 1;
  if (pick < 0) pick = 0;
  cand[t] = (int32_t)pick;
}

// FP64 mean of the rows listed in order[off[g]..off[g+1]) (fixed summation
// order); empty grains keep their centroid.  grid (G, ceil(d/256)).
__global__ __launch_bounds__(256) void segmented_mean_kernel(const float* __restrict__ Xs, int d,
                                                             const int32_t* __restrict__ order,
                                                             const int64_t* __restrict__ off,
                                                             const int* __restrict__ gmap,
                                                             float* __restrict__ cent) {
  const int g = gmap ? gmap[blockIdx.x] : (int)blockIdx.x;
  const int j = blockIdx.y * 256 + threadIdx.x;
  if (j >= d) return;
  const int64_t a = off[g], b = off[g + 1];
  if (b <= a) return;
  double s = 0.0;
  for (int64_t i = a; i < b; ++i) s += (double)Xs[(size_t)order[i] * d + j];
  cent[(size_t)g * d + j] = (float)(s / (double)(b - a));
}

// Grouped FP64 covariance of a chunk of grains (grain gmap[i] for chunk
// slot i).  grid (tile pair index, slot in chunk); 64x64 output tile per workgroup, 4x4 per thread; both the tile
// and its transpose are written.
constexpr int CT = 64, CK = 16;
__global__ __launch_bounds__(256) void covariance_kernel(const float* __restrict__ X, int d,
                                                         const int32_t* __restrict__ perm,
                                                         const int64_t* __restrict__ off, const float* __restrict__ mu,
                                                         const int* __restrict__ gmap, double* __restrict__ S,
                                                         const int* __restrict__ tiles) {
  __shared__ double Xi[CK][CT + 1];
  __shared__ double Xj[CK][CT + 1];
  const int gl = blockIdx.y, g = gmap[gl];
  const int ti = tiles[2 * blockIdx.x], tj = tiles[2 * blockIdx.x + 1];
  const int i0 = ti * CT, j0 = tj * CT;
  const int64_t a = off[g], n = off[g + 1] - off[g];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4] = {};
  const float* m = mu + (size_t)g * d;
  for (int64_t r0 = 0; r0 < n; r0 += CK) {
    for (int e = threadIdx.x; e < CK * CT; e += 256) {
      const int rr = e / CT, cc = e % CT;
      double vi = 0.0, vj = 0.0;
      if (r0 + rr < n) {
        const float* x = X + (size_t)perm[a + r0 + rr] * d;
        if (i0 + cc < d) vi = (double)x[i0 + cc] - (double)m[i0 + cc];
        if (j0 + cc < d) vj = (double)x[j0 + cc] - (double)m[j0 + cc];
      }
      Xi[rr][cc] = vi;
      Xj[rr][cc] = vj;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < CK; ++rr) {
      double ai[4], bj[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ai[u] = Xi[rr][ty * 4 + u];
        bj[u] = Xj[rr][tx * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(ai[u], bj[v], acc[u][v]);
    }
    __syncthreads();
  }
  const double inv = n > 0 ? 1.0 / (double)n : 0.0;
  double* Sg = S + (size_t)gl * d * d;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + ty * 4 + u, j = j0 + tx * 4 + v;
      if (i < d && j < d) {
        Sg[(size_t)i * d + j] = acc[u][v] * inv;
        Sg[(size_t)j * d + i] = acc[u][v] * inv;
      }
    }
}

// trace, shift S += delta I with delta = 1e-6 trace (+ tiny floor)
__global__ __launch_bounds__(256) void shift_kernel(double* __restrict__ S, int d, double* __restrict__ trace,
                                                    double* __restrict__ delta) {
  __shared__ double red[256];
  double* Sg = S + (size_t)blockIdx.x * d * d;
  double t = 0.0;
  for (int i = threadIdx.x; i < d; i += 256) t += Sg[(size_t)i * d + i];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double tr = red[0];
  const double dl = 1e-6 * tr + 1e-30;  // the floor keeps an all-zero covariance full rank
  for (int i = threadIdx.x; i < d; i += 256) Sg[(size_t)i * d + i] += dl;
  if (threadIdx.x == 0) {
    trace[blockIdx.x] = tr;
    delta[blockIdx.x] = dl;
  }
}

__global__ void randn_kernel(double* __restrict__ V, int64_t n, uint64_t seed, uint64_t stream) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) V[i] = 2.0 * u01(seed, stream, (uint64_t)i) - 1.0;
}

// Top-r Ritz vectors (columns b-1, b-2, ... of Wf, column-major d x b) ->
// sign-fixed FP64 rows Wd[slot][j][:] and FP32 basis rows of grain gmap[slot].
// grid (r, chunk).
__global__ __launch_bounds__(256) void extract_basis_kernel(const double* __restrict__ Wf, int d, int b, int r,
                                                            double* __restrict__ Wd, float* __restrict__ basis,
                                                            const int* __restrict__ gmap) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  const int j = blockIdx.x, gl = blockIdx.y;
  const double* col = Wf + (size_t)gl * d * b + (size_t)(b - 1 - j) * d;
  double best = -1.0;
  int besti = 0;
  for (int i = threadIdx.x; i < d; i += 256) {
    const double a = fabs(col[i]);
    if (a > best) {
      best = a;
      besti = i;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = besti;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      const double ov = bv[threadIdx.x + o];
      const int oi = bi[threadIdx.x + o];
      if (ov > bv[threadIdx.x] || (ov == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = ov;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const double sgn = col[bi[0]] < 0.0 ? -1.0 : 1.0;
  double* wd = Wd + ((size_t)gl * r + j) * d;
  float* bs = basis + ((size_t)gmap[gl] * r + j) * d;
  for (int i = threadIdx.x; i < d; i += 256) {
    const double v = sgn * col[i];
    wd[i] = v;
    bs[i] = (float)v;
  }
}

// Codes of one Block-SoA block: z = W_g^T (x - mu_g) and eps = ||x'||^2 - ||z||^2
// in FP64.  256 threads: member m = t & 63, coordinates j = (t >> 6) + 4u.
// blk_desc holds (grain, chunk slot of its FP64 basis, block of the grain)
// per workgroup; the block is written at boff[grain] + block.
constexpr int EK = 32;
__global__ __launch_bounds__(256) void encode_kernel(const float* __restrict__ X, int d, int r, int rp,
                                                     const int32_t* __restrict__ perm,
                                                     const int64_t* __restrict__ off, const float* __restrict__ mu,
                                                     const double* __restrict__ Wd, const int* __restrict__ blk_desc,
                                                     const int32_t* __restrict__ boff, float* __restrict__ codes,
                                                     float* __restrict__ eps) {
  __shared__ double xs[HNTL_WAVE][EK + 1];
  __shared__ double ws[HNTL_MAX_R][EK + 1];
  const int g = blk_desc[3 * blockIdx.x], slot = blk_desc[3 * blockIdx.x + 1];
  const int bi = blk_desc[3 * blockIdx.x + 2];
  const int blk = boff[g] + bi;
  const int t = threadIdx.x, m = t & 63, jq = t >> 6;
  const int64_t a = off[g], n = off[g + 1] - off[g];
  const int64_t mem = (int64_t)bi * B + m;
  const bool valid = mem < n;
  const float* mug = mu + (size_t)g * d;
  const double* W = Wd + (size_t)slot * r * d;
  double z[HNTL_MAX_R / 4];
#pragma unroll
  for (int u = 0; u < HNTL_MAX_R / 4; ++u) z[u] = 0.0;
  double sq = 0.0;
  for (int k0 = 0; k0 < d; k0 += EK) {
    for (int e = t; e < HNTL_WAVE * EK; e += 256) {
      const int mm = e / EK, kk = e % EK;
      const int64_t mi = (int64_t)bi * B + mm;
      double v = 0.0;
      if (mi < n && k0 + kk < d) v = (double)X[(size_t)perm[a + mi] * d + k0 + kk] - (double)mug[k0 + kk];
      xs[mm][kk] = v;
    }
    for (int e = t; e < r * EK; e += 256) {
      const int jj = e / EK, kk = e % EK;
      ws[jj][kk] = (k0 + kk < d) ? W[(size_t)jj * d + k0 + kk] : 0.0;
    }
    __syncthreads();
    for (int kk = 0; kk < EK; ++kk) {
      const double xv = xs[m][kk];
      if (jq == 0) sq = fma(xv, xv, sq);
#pragma unroll
      for (int u = 0; u < HNTL_MAX_R / 4; ++u) {
        const int j = jq + 4 * u;
        if (j < r) z[u] = fma(ws[j][kk], xv, z[u]);
      }
    }
    __syncthreads();
  }
  float* cb = codes + (size_t)blk * rp * B;
  double zz = 0.0;
#pragma unroll
  for (int u = 0; u < HNTL_MAX_R / 4; ++u) {
    const int j = jq + 4 * u;
    if (j < rp) cb[(size_t)j * B + m] = (valid && j < r) ? (float)z[u] : 0.f;
    if (j < r) zz += z[u] * z[u];
  }
  // ||z||^2 summed over the 4 thread groups through LDS
  __shared__ double zpart[4][HNTL_WAVE];
  zpart[jq][m] = zz;
  __syncthreads();
  if (jq == 0) {
    const double tot = zpart[0][m] + zpart[1][m] + zpart[2][m] + zpart[3][m];
    eps[(size_t)blk * B + m] = valid ? (float)fmax(sq - tot, 0.0) : __builtin_inff();
  }
}

// ---------------------------------------------------------------- host side
struct KMeansOut {
  std::vector<int32_t> label;  // per row (all N)
  int iters = 0;
};

// Phase timings on stderr when HNTL_VERBOSE is set to a positive number (each
// report waits for the stream, so timings are off unless asked for).
struct PhaseLog {
  bool on;
  hipStream_t s;
  std::chrono::steady_clock::time_point t0, t;
  explicit PhaseLog(hipStream_t s_) : s(s_) {
    const char* v = std::getenv("HNTL_VERBOSE");
    on = v && std::atoi(v) > 0;
    t0 = t = std::chrono::steady_clock::now();
  }
  void operator()(const char* what) {
    if (!on) return;
    (void)hipStreamSynchronize(s);
    const auto n = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[hntl_build] %-26s %8.2f s  (total %.2f s)\n", what,
                 std::chrono::duration<double>(n - t).count(), std::chrono::duration<double>(n - t0).count());
    std::fflush(stderr);
    t = n;
  }
};

std::vector<int64_t> counting_sort(const std::vector<int32_t>& lab, int G, std::vector<int32_t>& order) {
  std::vector<int64_t> off(G + 1, 0);
  for (int32_t l : lab) off[l + 1]++;
  for (int g = 0; g < G; ++g) off[g + 1] += off[g];
  std::vector<int64_t> cur(off.begin(), off.end() - 1);
  order.resize(lab.size());
  for (size_t i = 0; i < lab.size(); ++i) order[cur[lab[i]]++] = (int32_t)i;
  return off;
}

}  // namespace

// Local PCA of the grains in glist (FP64 covariance, subspace iteration on
// S_g + delta_g I with Cholesky-QR2, Rayleigh-Ritz), their FP32 basis rows,
// captured-variance fractions and the codes of every block they own.  Needs
// ix->X, perm, centroids, boff / boff_h, basis, codes, eps and captured (G
// entries) in place; d_off holds the G + 1 grain-order offsets on the device.
// The start vectors of the chunk from list position p0 come from counter
// stream stream_base + p0.
void pca_encode_grains(Index* ix, const int64_t* d_off, const std::vector<int32_t>& glist, uint32_t eig_iters,
                       uint64_t seed, uint64_t stream_base, hipStream_t s) {
  const uint32_t d = ix->d, r = ix->r;
  const int ng = (int)glist.size();
  if (ng == 0) return;
  struct Free {
    std::vector<void*> p;
    ~Free() {
      for (void* q : p) (void)hipFree(q);
    }
  } tmp;
  Blas blas(s);
  const int bsz = (int)std::min<uint32_t>(d, std::max<uint32_t>(r + 16, 2 * r));
  const int GC = (int)std::max<int64_t>(1, std::min<int64_t>(ng, ((int64_t)1 << 30) / ((int64_t)d * d * 8)));
  double* S = dev_alloc<double>(nullptr, (size_t)GC * d * d);
  tmp.p.push_back(S);
  double* V = dev_alloc<double>(nullptr, (size_t)GC * d * bsz);
  tmp.p.push_back(V);
  double* Y = dev_alloc<double>(nullptr, (size_t)GC * d * bsz);
  tmp.p.push_back(Y);
  double* M = dev_alloc<double>(nullptr, (size_t)GC * bsz * bsz);
  tmp.p.push_back(M);
  double* Wev = dev_alloc<double>(nullptr, (size_t)GC * bsz);
  tmp.p.push_back(Wev);
  double* res = dev_alloc<double>(nullptr, GC);
  tmp.p.push_back(res);
  int* nsw = dev_alloc<int>(nullptr, GC);
  tmp.p.push_back(nsw);
  int* info = dev_alloc<int>(nullptr, GC);
  tmp.p.push_back(info);
  double* trace = dev_alloc<double>(nullptr, GC);
  tmp.p.push_back(trace);
  double* delta = dev_alloc<double>(nullptr, GC);
  tmp.p.push_back(delta);
  double* Wd = dev_alloc<double>(nullptr, (size_t)GC * r * d);
  tmp.p.push_back(Wd);
  int* d_glist = dev_alloc<int>(nullptr, ng);
  tmp.p.push_back(d_glist);
  HIP_TRY(hipMemcpyAsync(d_glist, glist.data(), sizeof(int) * ng, hipMemcpyHostToDevice, s));
  // upper-triangle tile list
  const int nt = (int)((d + CT - 1) / CT);
  std::vector<int> tiles;
  for (int i = 0; i < nt; ++i)
    for (int j = i; j < nt; ++j) {
      tiles.push_back(i);
      tiles.push_back(j);
    }
  int* d_tiles = dev_alloc<int>(nullptr, tiles.size());
  tmp.p.push_back(d_tiles);
  HIP_TRY(hipMemcpyAsync(d_tiles, tiles.data(), sizeof(int) * tiles.size(), hipMemcpyHostToDevice, s));
  // per-block work descriptors (grain, chunk slot, block of the grain), all chunks
  int64_t nblk_all = 0;
  for (int32_t g : glist) nblk_all += ix->boff_h[g + 1] - ix->boff_h[g];
  int* d_desc = dev_alloc<int>(nullptr, (size_t)std::max<int64_t>(1, 3 * nblk_all));
  tmp.p.push_back(d_desc);
  std::vector<double> ev_h((size_t)GC * bsz), tr_h(GC), dl_h(GC);
  std::vector<int> desc;
  const double one = 1.0, zero = 0.0;
  int64_t desc_pos = 0;
  for (int p0 = 0; p0 < ng; p0 += GC) {
    const int gc = std::min(GC, ng - p0);
    const int* gmap = d_glist + p0;
    hipLaunchKernelGGL(covariance_kernel, dim3((unsigned)(tiles.size() / 2), gc), dim3(256), 0, s, ix->X, (int)d,
                       ix->perm, d_off, ix->centroids, gmap, S, d_tiles);
    hipLaunchKernelGGL(shift_kernel, dim3(gc), dim3(256), 0, s, S, (int)d, trace, delta);
    const int64_t nv = (int64_t)gc * d * bsz;
    hipLaunchKernelGGL(randn_kernel, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, s, V, nv, seed,
                       stream_base + (uint64_t)p0);
    HIP_TRY(hipGetLastError());
    const rocblas_stride sS = (rocblas_stride)d * d, sV = (rocblas_stride)d * bsz, sM = (rocblas_stride)bsz * bsz;
    auto cholqr = [&](double* Yp) {
      for (int rep = 0; rep < 2; ++rep) {
        rb(rocblas_dgemm_strided_batched(blas.h, rocblas_operation_transpose, rocblas_operation_none, bsz, bsz, (int)d,
                                         &one, Yp, (int)d, sV, Yp, (int)d, sV, &zero, M, bsz, sM, gc),
           "dgemm Y^T*Y");
        rb(rocsolver_dpotrf_strided_batched(blas.h, rocblas_fill_upper, bsz, M, bsz, sM, info, gc), "dpotrf");
        rb(rocblas_dtrsm_strided_batched(blas.h, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                                         rocblas_diagonal_non_unit, (int)d, bsz, &one, M, bsz, sM, Yp, (int)d, sV, gc),
           "dtrsm");
      }
    };
    cholqr(V);
    for (uint32_t itx = 0; itx < eig_iters; ++itx) {
      rb(rocblas_dgemm_strided_batched(blas.h, rocblas_operation_none, rocblas_operation_none, (int)d, bsz, (int)d,
                                       &one, S, (int)d, sS, V, (int)d, sV, &zero, Y, (int)d, sV, gc),
         "dgemm S*V");
      cholqr(Y);
      std::swap(V, Y);
    }
    // Rayleigh-Ritz: H = V^T S V, eigen-decomposed; W = V * U
    rb(rocblas_dgemm_strided_batched(blas.h, rocblas_operation_none, rocblas_operation_none, (int)d, bsz, (int)d, &one,
                                     S, (int)d, sS, V, (int)d, sV, &zero, Y, (int)d, sV, gc),
       "dgemm S*V");
    rb(rocblas_dgemm_strided_batched(blas.h, rocblas_operation_transpose, rocblas_operation_none, bsz, bsz, (int)d,
                                     &one, V, (int)d, sV, Y, (int)d, sV, &zero, M, bsz, sM, gc),
       "dgemm V^T*Y");
    rb(rocsolver_dsyevj_strided_batched(blas.h, rocblas_esort_ascending, rocblas_evect_original, rocblas_fill_upper,
                                        bsz, M, bsz, sM, 0.0, res, 100, nsw, Wev, bsz, info, gc),
       "dsyevj");
    rb(rocblas_dgemm_strided_batched(blas.h, rocblas_operation_none, rocblas_operation_none, (int)d, bsz, bsz, &one, V,
                                     (int)d, sV, M, bsz, sM, &zero, Y, (int)d, sV, gc),
       "dgemm V*U");
    hipLaunchKernelGGL(extract_basis_kernel, dim3(r, gc), dim3(256), 0, s, Y, (int)d, bsz, (int)r, Wd, ix->basis,
                       gmap);
    HIP_TRY(hipGetLastError());
    // codes of every block of the chunk's grains
    desc.clear();
    for (int gl = 0; gl < gc; ++gl) {
      const int g = glist[p0 + gl];
      for (int q = 0; q < ix->boff_h[g + 1] - ix->boff_h[g]; ++q) {
        desc.push_back(g);
        desc.push_back(gl);
        desc.push_back(q);
      }
    }
    const int nb = (int)(desc.size() / 3);
    if (nb > 0) {
      int* dd = d_desc + desc_pos;  // each chunk has its own range: no reuse while a copy is in flight
      desc_pos += (int64_t)desc.size();
      HIP_TRY(hipMemcpyAsync(dd, desc.data(), sizeof(int) * desc.size(), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(encode_kernel, dim3((unsigned)nb), dim3(256), 0, s, ix->X, (int)d, (int)r, (int)ix->rp,
                         ix->perm, d_off, ix->centroids, Wd, dd, ix->boff, ix->codes, ix->eps);
      HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipMemcpyAsync(ev_h.data(), Wev, sizeof(double) * gc * bsz, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(tr_h.data(), trace, sizeof(double) * gc, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(dl_h.data(), delta, sizeof(double) * gc, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int gl = 0; gl < gc; ++gl)
      for (int j = 0; j < bsz; ++j)
        if (!std::isfinite(ev_h[(size_t)gl * bsz + j]))
          throw HipError(hipErrorUnknown,
                         "eigensolver produced a non-finite value for grain " + std::to_string(glist[p0 + gl]));
    for (int gl = 0; gl < gc; ++gl) {
      double top = 0.0;
      for (uint32_t j = 0; j < r; ++j) top += ev_h[(size_t)gl * bsz + bsz - 1 - j] - dl_h[gl];
      ix->captured[glist[p0 + gl]] = tr_h[gl] > 0 ? top / tr_h[gl] : 1.0;
    }
  }
}

void launch_segmented_mean(const float* X, int d, const int32_t* order, const int64_t* off, const int* gmap, int ng,
                           float* cent, hipStream_t s) {
  if (ng <= 0) return;
  hipLaunchKernelGGL(segmented_mean_kernel, dim3(ng, (d + 255) / 256), dim3(256), 0, s, X, d, order, off, gmap, cent);
  HIP_TRY(hipGetLastError());
}

}  // namespace hntl

using namespace hntl;

extern "C" hntl_status hntl_build(const float* X, uint64_t N, uint32_t d, const hntl_build_params* params,
                                  void* stream, hntl_index** out) {
  set_error("");
  if (!out) return fail(HNTL_EINVAL, "out is NULL");
  *out = nullptr;
  if (!X || !params) return fail(HNTL_EINVAL, "null pointer");
  const uint32_t G = params->G, r = params->r;
  if (N == 0 || d == 0) return fail(HNTL_EINVAL, "N and d must be positive");
  if (G == 0 || G > N) return fail(HNTL_EINVAL, "need 1 <= G <= N");
  if (r == 0 || r > d) return fail(HNTL_EINVAL, "need 1 <= r <= d");
  if (r > HNTL_MAX_R) return fail(HNTL_EUNSUPPORTED, "r exceeds HNTL_MAX_R");
  if (N >= (1ull << 31)) return fail(HNTL_EUNSUPPORTED, "N must be below 2^31");
  hipStream_t s = (hipStream_t)stream;
  const uint32_t max_iter = params->kmeans_iters ? params->kmeans_iters : 25;
  const uint32_t tpg = params->train_per_grain ? params->train_per_grain : 256;
  const uint32_t eig_iters = params->eig_iters ? params->eig_iters : 40;
  const uint64_t seed = params->seed;
  hntl_index* h = nullptr;
  try {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(HNTL_EDEVICE, "no GPU device");
    h = new hntl_index();
    Index* ix = &h->ix;
    HIP_TRY(hipGetDevice(&ix->device));
    ix->N = N;
    ix->d = d;
    ix->G = G;
    ix->r = r;
    ix->rp = (r + 7) / 8 * 8;
    PhaseLog plog(s);
    ix->X = dev_alloc<float>(ix, (size_t)N * d);
    HIP_TRY(hipMemcpyAsync(ix->X, X, sizeof(float) * N * d, hipMemcpyDefault, s));
    ix->centroids = dev_alloc<float>(ix, (size_t)G * d);
    ix->cnorm = dev_alloc<float>(ix, G);

    // ---------------- k-means: training subset (partial Fisher-Yates)
    const int64_t n_train = std::min<int64_t>((int64_t)N, (int64_t)tpg * G);
    const int64_t n_seed = std::min<int64_t>(n_train, (int64_t)262144);
    std::vector<int32_t> tr_idx(n_train);
    {
      std::vector<int32_t> all(N);
      std::iota(all.begin(), all.end(), 0);
      for (int64_t i = 0; i < n_train; ++i) {
        const int64_t j = i + (int64_t)(u01(seed, 1, (uint64_t)i) * (double)(N - i));
        std::swap(all[i], all[std::min<int64_t>(j, N - 1)]);
        tr_idx[i] = all[i];
      }
    }
    int32_t* d_tr = dev_alloc<int32_t>(nullptr, n_train);
    float* Xt = dev_alloc<float>(nullptr, (size_t)n_train * d);
    float* xtn = dev_alloc<float>(nullptr, n_train);
    int32_t* lab_t = dev_alloc<int32_t>(nullptr, n_train);
    float* dmin_t = dev_alloc<float>(nullptr, n_train);
    struct Free {
      std::vector<void*> p;
      ~Free() {
        for (void* q : p) (void)hipFree(q);
      }
    } tmp;
    tmp.p = {d_tr, Xt, xtn, lab_t, dmin_t};
    HIP_TRY(hipMemcpyAsync(d_tr, tr_idx.data(), sizeof(int32_t) * n_train, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)n_train), dim3(256), 0, s, ix->X, (int)d, d_tr, n_train,
                       Xt);
    HIP_TRY(hipGetLastError());
    launch_row_norms(Xt, n_train, (int)d, xtn, s);

    // ---------------- seeding
    if (params->init_centroids) {
      HIP_TRY(hipMemcpyAsync(ix->centroids, params->init_centroids, sizeof(float) * G * d, hipMemcpyDefault, s));
    } else {
      const int nblk = (int)((n_seed + 255) / 256);
      const int L = KPP_MAXL;  // 2 + ln G candidates still merge well-separated clusters in about 1 run of 4
      float* closest = dev_alloc<float>(nullptr, n_seed);
      double* partial = dev_alloc<double>(nullptr, nblk);
      float* dcand = dev_alloc<float>(nullptr, (size_t)n_seed * L);
      double* potpart = dev_alloc<double>(nullptr, (size_t)nblk * L);
      int32_t* cand = dev_alloc<int32_t>(nullptr, KPP_MAXL);
      int32_t* tstar = dev_alloc<int32_t>(nullptr, 1);
      double* uu = dev_alloc<double>(nullptr, (size_t)G * KPP_MAXL);
      tmp.p.insert(tmp.p.end(), {closest, partial, dcand, potpart, cand, tstar, uu});
      // all uniforms of the seeding, drawn up front from the counter-based hash
      std::vector<double> uh((size_t)G * KPP_MAXL);
      for (uint32_t st = 0; st < G; ++st)
        for (int t = 0; t < KPP_MAXL; ++t) uh[(size_t)st * KPP_MAXL + t] = u01(seed, 2, (uint64_t)st * KPP_MAXL + t);
      HIP_TRY(hipMemcpyAsync(uu, uh.data(), sizeof(double) * uh.size(), hipMemcpyHostToDevice, s));
      // first centroid: a uniformly drawn seeding row
      const int32_t first = (int32_t)std::min<int64_t>(n_seed - 1, (int64_t)(uh[0] * (double)n_seed));
      HIP_TRY(hipMemcpyAsync(cand, &first, sizeof(int32_t), hipMemcpyHostToDevice, s));
      float* cand_rows = dev_alloc<float>(nullptr, (size_t)KPP_MAXL * d);
      float* cand_norm = dev_alloc<float>(nullptr, KPP_MAXL);
      tmp.p.insert(tmp.p.end(), {cand_rows, cand_norm});
      // candidate distances on the MFMA distance kernel, then potentials
      auto evaluate = [&](int Lc, int first_step) {
        hipLaunchKernelGGL(gather_rows_kernel, dim3(Lc), dim3(256), 0, s, Xt, (int)d, cand, (int64_t)Lc, cand_rows);
        launch_row_norms(cand_rows, Lc, (int)d, cand_norm, s);
        launch_dist_matrix(Xt, xtn, n_seed, cand_rows, cand_norm, Lc, (int)d, dcand, s);
        hipLaunchKernelGGL(kpp_pot_kernel, dim3(nblk), dim3(256), 0, s, n_seed, Lc, dcand, closest, first_step,
                           potpart);
      };
      evaluate(1, 1);
      hipLaunchKernelGGL(kpp_choose_kernel, dim3(1), dim3(64), 0, s, Xt, (int)d, cand, 1, potpart, nblk, tstar,
                         ix->centroids, 0);
      hipLaunchKernelGGL(kpp_apply_kernel, dim3(nblk), dim3(256), 0, s, n_seed, 1, dcand, tstar, 1, closest, partial);
      for (uint32_t step = 1; step < G; ++step) {
        hipLaunchKernelGGL(kpp_sample_kernel, dim3(1), dim3(64), 0, s, n_seed, closest, partial, nblk,
                           uu + (size_t)step * KPP_MAXL, L, cand);
        evaluate(L, 0);
        hipLaunchKernelGGL(kpp_choose_kernel, dim3(1), dim3(64), 0, s, Xt, (int)d, cand, L, potpart, nblk, tstar,
                           ix->centroids, (int)step);
        hipLaunchKernelGGL(kpp_apply_kernel, dim3(nblk), dim3(256), 0, s, n_seed, L, dcand, tstar, 0, closest,
                           partial);
      }
      HIP_TRY(hipGetLastError());
    }

    plog("k-means++ seeding");
    // ---------------- Lloyd iterations on the training rows
    std::vector<int32_t> lab_h(n_train), prev(n_train, -1), order_h;
    std::vector<float> dmin_h(n_train);
    int32_t* d_order = dev_alloc<int32_t>(nullptr, std::max<int64_t>(n_train, (int64_t)N));
    int64_t* d_off = dev_alloc<int64_t>(nullptr, G + 1);
    tmp.p.push_back(d_order);
    tmp.p.push_back(d_off);
    auto assign_train = [&]() {
      launch_row_norms(ix->centroids, G, (int)d, ix->cnorm, s);
      launch_argmin_rows(Xt, xtn, n_train, ix->centroids, ix->cnorm, (int)G, (int)d, lab_t, dmin_t, s);
      HIP_TRY(hipMemcpyAsync(lab_h.data(), lab_t, sizeof(int32_t) * n_train, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(dmin_h.data(), dmin_t, sizeof(float) * n_train, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
    };
    assign_train();
    uint32_t it = 0;
    for (it = 1; it <= max_iter; ++it) {
      auto off = counting_sort(lab_h, (int)G, order_h);
      HIP_TRY(hipMemcpyAsync(d_order, order_h.data(), sizeof(int32_t) * n_train, hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(d_off, off.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(segmented_mean_kernel, dim3(G, (d + 255) / 256), dim3(256), 0, s, Xt, (int)d, d_order, d_off,
                         nullptr, ix->centroids);
      HIP_TRY(hipGetLastError());
      // re-seed empty grains with the farthest training rows
      std::vector<char> taken;
      for (uint32_t g = 0; g < G; ++g) {
        if (off[g + 1] > off[g]) continue;
        if (taken.empty()) taken.assign(n_train, 0);
        int64_t best = -1;
        for (int64_t i = 0; i < n_train; ++i)
          if (!taken[i] && (best < 0 || dmin_h[i] > dmin_h[best])) best = i;
        if (best < 0) break;
        taken[best] = 1;
        dmin_h[best] = 0.f;
        HIP_TRY(hipMemcpyAsync(ix->centroids + (size_t)g * d, Xt + (size_t)best * d, sizeof(float) * d,
                               hipMemcpyDeviceToDevice, s));
      }
      prev.swap(lab_h);
      assign_train();
      int64_t changed = 0;
      for (int64_t i = 0; i < n_train; ++i) changed += prev[i] != lab_h[i];
      if (changed == 0) break;
    }
    ix->kmeans_iters_run = std::min(it, max_iter);
    plog("Lloyd iterations");

    // ---------------- final assignment of every row, exact member means
    {
      float* xn = dev_alloc<float>(nullptr, N);
      int32_t* lab = dev_alloc<int32_t>(nullptr, N);
      tmp.p.push_back(xn);
      tmp.p.push_back(lab);
      launch_row_norms(ix->X, N, (int)d, xn, s);
      launch_row_norms(ix->centroids, G, (int)d, ix->cnorm, s);
      launch_argmin_rows(ix->X, xn, N, ix->centroids, ix->cnorm, (int)G, (int)d, lab, nullptr, s);
      std::vector<int32_t> lab_all(N);
      HIP_TRY(hipMemcpyAsync(lab_all.data(), lab, sizeof(int32_t) * N, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      std::vector<int32_t> perm_h;
      ix->offsets_h = counting_sort(lab_all, (int)G, perm_h);
      ix->perm = dev_alloc<int32_t>(ix, N);
      HIP_TRY(hipMemcpyAsync(ix->perm, perm_h.data(), sizeof(int32_t) * N, hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(d_off, ix->offsets_h.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(segmented_mean_kernel, dim3(G, (d + 255) / 256), dim3(256), 0, s, ix->X, (int)d, ix->perm,
                         d_off, nullptr, ix->centroids);
      HIP_TRY(hipGetLastError());
      launch_row_norms(ix->centroids, G, (int)d, ix->cnorm, s);
    }

    plog("final assignment + means");
    // ---------------- block layout
    {
      ix->boff_h.assign(G + 1, 0);
      uint32_t maxg = 0;
      for (uint32_t g = 0; g < G; ++g) {
        const int64_t n = ix->offsets_h[g + 1] - ix->offsets_h[g];
        maxg = std::max<uint32_t>(maxg, (uint32_t)n);
        ix->boff_h[g + 1] = ix->boff_h[g] + (int32_t)((n + B - 1) / B);
      }
      ix->max_grain = maxg;
      ix->nblocks = (uint64_t)ix->boff_h[G];
      std::vector<int32_t> goff32(G + 1);
      for (uint32_t g = 0; g <= G; ++g) goff32[g] = (int32_t)ix->offsets_h[g];
      ix->goff = dev_alloc<int32_t>(ix, G + 1);
      ix->boff = dev_alloc<int32_t>(ix, G + 1);
      HIP_TRY(hipMemcpyAsync(ix->goff, goff32.data(), sizeof(int32_t) * (G + 1), hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(ix->boff, ix->boff_h.data(), sizeof(int32_t) * (G + 1), hipMemcpyHostToDevice, s));
      ix->codes = dev_alloc<float>(ix, (size_t)ix->nblocks * ix->rp * B);
      ix->eps = dev_alloc<float>(ix, (size_t)ix->nblocks * B);
      ix->basis = dev_alloc<float>(ix, (size_t)G * r * d);
    }

    // ---------------- local PCA per grain chunk + codes
    {
      std::vector<int32_t> all(G);
      std::iota(all.begin(), all.end(), 0);
      ix->captured.assign(G, -1.0);
      pca_encode_grains(ix, d_off, all, eig_iters, seed, 3, s);
    }
    plog("covariance, eigensolve, codes");
    launch_grain_bounds(*ix, s);
    ix->codes_mask = 1u;
    const uint32_t want =
        params->codes_mask & ((1u << HNTL_CODES_BF16) | (1u << HNTL_CODES_FP8_E4M3) | (1u << HNTL_CODES_INT16));
    if (want) {
      ix->codes_mask |= want;
      launch_derive_lowp(*ix, s);
    }
    HIP_TRY(hipStreamSynchronize(s));
    plog("bounds + reduced-precision codes");
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
