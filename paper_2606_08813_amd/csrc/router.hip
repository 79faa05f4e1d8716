// Learned router: a small MLP that maps a query to one score per grain, whose
// top-P grains replace centroid routing.  The paper routes by centroid
// distance (Section 2.3) and names learned partitioning as future work
// (Section 4); this is that extension.
//
//   xh = bf16((x - mean) / std)                      standardised input
//   h1 = bf16(gelu(W1 xh + b1)),  h2 = bf16(gelu(W2 h1 + b2))
//   s  = W3 h2 + b3                                   one score per grain
//
// GELU is the exact erf form (Hendrycks & Gimpel), computed with the device
// erff.  Weights are FP32 masters with BF16 copies; every GEMM takes BF16
// operands on the MFMA units (v_mfma_f32_16x16x32_bf16) and accumulates in
// FP32; bias, GELU, softmax, loss and Adam run in FP32.
//
// Training (softmax cross-entropy, Adam of Kingma & Ba with bias
// correction) targets the grain distribution of each training query's exact
// k nearest neighbours: the fraction of them in each grain.  Backward pass,
// per batch of B rows (rounding points as the forward: every GEMM operand
// rounded to BF16):
//
//   ds  = (softmax(s) - y) / B;   gW3 = bf16(ds)^T h2,  gb3 = sum_b ds
//   da2 = (bf16(ds) W3) * gelu'(a2);   gW2 = bf16(da2)^T h1,  gb2 = sum_b da2
//   da1 = (bf16(da2) W2) * gelu'(a1);  gW1 = bf16(da1)^T xh,  gb1 = sum_b da1
//
// The GEMM kernel below is the one contraction of all of this: C = A . B^T in
// the sense C[m][n] = sum_k A(m, k) B(n, k), with A and B each stored either
// k-contiguous or (transposed) m- / n-contiguous, staged through LDS.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <vector>

#include "hntl_device.h"
#include "hntl_internal.h"

namespace hntl {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// ------------------------------------------------------------------ GEMM
constexpr int GM = 128, GN = 128, GK = 64, GLD = GK + 8;  // LDS rows padded by 8 bf16

enum { EPI_F32 = 0, EPI_BIAS_GELU = 1, EPI_GELU_GRAD = 2, EPI_BIAS_F32 = 3, EPI_DIST = 4 };
struct Epi {
  float* C;            // FP32 output (EPI_F32, EPI_BIAS_F32: the result; EPI_BIAS_GELU: pre-activation, optional)
  int ldc;
  const float* bias;   // N
  uint16_t* H;         // BF16 output (EPI_BIAS_GELU: gelu(z); EPI_GELU_GRAD: bf16(acc * gelu'(z)))
  int ldh;
  const float* Z;      // EPI_GELU_GRAD: pre-activation
  int ldz;
  float* D;            // EPI_GELU_GRAD: FP32 acc * gelu'(z)
  int ldd;
  float scale;         // EPI_BIAS_F32: result = scale * (acc + bias)
  const float* an;     // EPI_DIST: C = max(an[row] + bn[col] - 2 acc, 0)
  const float* bn;
  int64_t row_base;    // rows from *mlim - row_base on are skipped
};

// Epilogue of one output element (row < M, col < N checked by the caller).
template <int EPI>
__device__ __forceinline__ void epi_store(const Epi& e, int row, int col, float v) {
  if constexpr (EPI == EPI_F32) {
    e.C[(size_t)row * e.ldc + col] = v;
  } else if constexpr (EPI == EPI_BIAS_F32) {
    e.C[(size_t)row * e.ldc + col] = e.scale * (v + e.bias[col]);
  } else if constexpr (EPI == EPI_BIAS_GELU) {
    const float z = v + e.bias[col];
    if (e.C) e.C[(size_t)row * e.ldc + col] = z;
    e.H[(size_t)row * e.ldh + col] = to_bf16(gelu(z));
  } else if constexpr (EPI == EPI_DIST) {
    e.C[(size_t)row * e.ldc + col] = fmaxf(e.an[row] + e.bn[col] - 2.f * v, 0.f);
  } else {
    const float gz = v * gelu_grad(e.Z[(size_t)row * e.ldz + col]);
    e.D[(size_t)row * e.ldd + col] = gz;
    e.H[(size_t)row * e.ldh + col] = to_bf16(gz);
  }
}

// The same epilogue with its per-row term rt (EPI_DIST: an[row]) and per-column
// term ct (EPI_DIST: bn[col]; the bias forms: bias[col]) loaded once per row
// and column by the caller instead of once per element; same arithmetic.
template <int EPI>
__device__ __forceinline__ float epi_row_term(const Epi& e, int row) {
  if constexpr (EPI == EPI_DIST) return e.an[row];
  return 0.f;
}
template <int EPI>
__device__ __forceinline__ float epi_col_term(const Epi& e, int col) {
  if constexpr (EPI == EPI_DIST) return e.bn[col];
  if constexpr (EPI == EPI_BIAS_F32 || EPI == EPI_BIAS_GELU) return e.bias[col];
  return 0.f;
}
template <int EPI>
__device__ __forceinline__ void epi_store_t(const Epi& e, int row, int col, float v, float rt, float ct) {
  if constexpr (EPI == EPI_F32) {
    e.C[(size_t)row * e.ldc + col] = v;
  } else if constexpr (EPI == EPI_BIAS_F32) {
    e.C[(size_t)row * e.ldc + col] = e.scale * (v + ct);
  } else if constexpr (EPI == EPI_BIAS_GELU) {
    const float z = v + ct;
    if (e.C) e.C[(size_t)row * e.ldc + col] = z;
    e.H[(size_t)row * e.ldh + col] = to_bf16(gelu(z));
  } else if constexpr (EPI == EPI_DIST) {
    e.C[(size_t)row * e.ldc + col] = fmaxf(rt + ct - 2.f * v, 0.f);
  } else {
    epi_store<EPI>(e, row, col, v);
  }
}

// One thread's share of a 128 x 64 tile of X(r, k) (rows r0.., depths k0..):
// 32 bf16 in four 16-byte words.  XT = false: X(r, k) = X[r * ld + k], the
// thread holds row t / 2, depths 32 (t % 2) .. + 31; XT = true:
// X(r, k) = X[k * ld + r], the thread holds depth t / 4, rows 32 (t % 4) .. + 31.
struct Frag {
  uint4 v[4];
};

template <bool XT>
__device__ __forceinline__ void gemm_fetch(Frag& f, const uint16_t* __restrict__ X, int ld, int R, int K, int r0,
                                           int k0) {
  const int t = threadIdx.x;
  const int a = XT ? (t >> 2) : (t >> 1);       // depth (XT) or row
  const int b0 = XT ? (t & 3) * 32 : (t & 1) * 32;  // first row (XT) or depth of the run
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int gr = XT ? r0 + b0 + 8 * h : r0 + a;  // row of element 0 of this word
    const int gk = XT ? k0 + a : k0 + b0 + 8 * h;  // depth of element 0
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (!XT) {
      if (gr < R && gk + 8 <= K) {
        v = *reinterpret_cast<const uint4*>(X + (size_t)gr * ld + gk);
      } else if (gr < R) {
        uint16_t e[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) e[u] = gk + u < K ? X[(size_t)gr * ld + gk + u] : 0;
        memcpy(&v, e, 16);
      }
    } else {
      if (gk < K && gr + 8 <= R) {
        v = *reinterpret_cast<const uint4*>(X + (size_t)gk * ld + gr);
      } else if (gk < K) {
        uint16_t e[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) e[u] = gr + u < R ? X[(size_t)gk * ld + gr + u] : 0;
        memcpy(&v, e, 16);
      }
    }
    f.v[h] = v;
  }
}

template <bool XT>
__device__ __forceinline__ void gemm_store(uint16_t (*S)[GLD], const Frag& f) {
  const int t = threadIdx.x;
  if (!XT) {
    const int r = t >> 1, kk = (t & 1) * 32;
#pragma unroll
    for (int h = 0; h < 4; ++h) *reinterpret_cast<uint4*>(&S[r][kk + 8 * h]) = f.v[h];
  } else {
    const int k = t >> 2, rr = (t & 3) * 32;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      uint16_t e[8];
      memcpy(e, &f.v[h], 16);
#pragma unroll
      for (int u = 0; u < 8; ++u) S[rr + 8 * h + u][k] = e[u];
    }
  }
}

// One workgroup (4 waves) per 128 x 128 tile of C; wave w owns a 64 x 64
// quarter as 4 x 4 MFMA 16x16 tiles.  Lane (i = lane % 16, kq = lane / 16)
// feeds depths 8 kq .. 8 kq + 7 of row / column i to each MFMA and holds
// C[4 kq + j][i] of each 16 x 16 output.  The next depth tile is fetched into
// registers while the MFMAs of the current one run.  Rows from *mlim on are
// skipped.
template <bool AT, bool BT, int EPI>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(const uint16_t* __restrict__ A, int lda,
                                                        const uint16_t* __restrict__ B, int ldb, int M, int N, int K,
                                                        Epi e, const int32_t* __restrict__ mlim) {
  __shared__ __attribute__((aligned(16))) uint16_t As[GM][GLD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[GN][GLD];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int m0 = blockIdx.y * GM, n0 = blockIdx.x * GN;
  if (mlim) {
    const int lim = (int)(*mlim - e.row_base);
    if (m0 >= lim) return;
    if (lim < M) M = lim;
  }
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int i = lane & 15, kq = lane >> 4;
  floatx4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  Frag fa, fb;
  gemm_fetch<AT>(fa, A, lda, M, K, m0, 0);
  gemm_fetch<BT>(fb, B, ldb, N, K, n0, 0);
  for (int k0 = 0; k0 < K; k0 += GK) {
    gemm_store<AT>(As, fa);
    gemm_store<BT>(Bs, fb);
    __syncthreads();
    if (k0 + GK < K) {
      gemm_fetch<AT>(fa, A, lda, M, K, m0, k0 + GK);
      gemm_fetch<BT>(fb, B, ldb, N, K, n0, k0 + GK);
    }
#pragma unroll
    for (int ks = 0; ks < GK; ks += 32) {
      bf16x8 af[4], bfv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        af[t] = *reinterpret_cast<const bf16x8*>(&As[wm + 16 * t + i][ks + 8 * kq]);
        bfv[t] = *reinterpret_cast<const bf16x8*>(&Bs[wn + 16 * t + i][ks + 8 * kq]);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = m0 + wm + 16 * a + 4 * kq + j;
        const int col = n0 + wn + 16 * b + i;
        if (row >= M || col >= N) continue;
        epi_store<EPI>(e, row, col, acc[a][b][j]);
      }
}

// ---------------------------------------------- large-tile GEMM, both k-contiguous
// C = A B^T with A (M x K) and B (N x K) both row-major (k contiguous, K % 8
// == 0), the shape of every forward product.  One workgroup of 8 waves per
// 256 x 128 tile of C; wave w owns rows 64 (w / 2) .. + 63 and columns
// 64 (w % 2) .. + 63 as 4 x 4 MFMA 16x16x32 tiles.  Depth tiles of 64 go
// global -> registers -> LDS into two LDS buffers: tile k + 1 loads while
// tile k feeds the MFMAs, one barrier per depth tile.  Tiles are handed to the
// 8 XCDs in contiguous runs (workgroup ids go round-robin over the XCDs), so
// the workgroups of one XCD share A row blocks in their L2.
constexpr int NM = 256, NN = 128, NK = 64, NLD = NK + 8;

struct NFrag {
  uint4 a[4];  // A: row t / 2, depths 32 (t % 2) + 8 h
  uint4 b[2];  // B: row t / 4, depths 16 (t % 4) + 8 h
};

// 8 consecutive bf16 of row r from depth k (K % 8 == 0: a run is wholly in or out).
__device__ __forceinline__ uint4 load8(const uint16_t* __restrict__ X, int ld, int R, int K, int r, int k) {
  uint4 v = make_uint4(0u, 0u, 0u, 0u);
  if (r < R && k < K) v = *reinterpret_cast<const uint4*>(X + (size_t)r * ld + k);
  return v;
}

__device__ __forceinline__ void nfetch(NFrag& f, const uint16_t* __restrict__ A, int lda, int M,
                                       const uint16_t* __restrict__ B, int ldb, int N, int K, int m0, int n0, int k0) {
  const int t = threadIdx.x;
#pragma unroll
  for (int h = 0; h < 4; ++h) f.a[h] = load8(A, lda, M, K, m0 + (t >> 1), k0 + (t & 1) * 32 + 8 * h);
#pragma unroll
  for (int h = 0; h < 2; ++h) f.b[h] = load8(B, ldb, N, K, n0 + (t >> 2), k0 + (t & 3) * 16 + 8 * h);
}

__device__ __forceinline__ void nstore(uint16_t (*As)[NLD], uint16_t (*Bs)[NLD], const NFrag& f) {
  const int t = threadIdx.x;
#pragma unroll
  for (int h = 0; h < 4; ++h) *reinterpret_cast<uint4*>(&As[t >> 1][(t & 1) * 32 + 8 * h]) = f.a[h];
#pragma unroll
  for (int h = 0; h < 2; ++h) *reinterpret_cast<uint4*>(&Bs[t >> 2][(t & 3) * 16 + 8 * h]) = f.b[h];
}

template <int EPI>
__global__ __launch_bounds__(512) void gemm_nn_kernel(const uint16_t* __restrict__ A, int lda,
                                                      const uint16_t* __restrict__ B, int ldb, int M, int N, int K,
                                                      Epi e, const int32_t* __restrict__ mlim, int tiles_n,
                                                      int ntiles) {
  extern __shared__ __attribute__((aligned(16))) uint16_t nsm[];
  uint16_t(*As0)[NLD] = reinterpret_cast<uint16_t(*)[NLD]>(nsm);
  uint16_t(*Bs0)[NLD] = reinterpret_cast<uint16_t(*)[NLD]>(nsm + NM * NLD);
  uint16_t(*As1)[NLD] = reinterpret_cast<uint16_t(*)[NLD]>(nsm + (NM + NN) * NLD);
  uint16_t(*Bs1)[NLD] = reinterpret_cast<uint16_t(*)[NLD]>(nsm + (2 * NM + NN) * NLD);
  // XCD-contiguous tile order: workgroup b runs on XCD b % 8
  const int nb = (int)gridDim.x, per = nb / 8;
  const int bid = (int)blockIdx.x;
  const int tile = (nb % 8 == 0) ? (bid % 8) * per + bid / 8 : bid;
  if (tile >= ntiles) return;
  const int m0 = (tile / tiles_n) * NM, n0 = (tile % tiles_n) * NN;
  if (mlim) {
    const int lim = (int)(*mlim - e.row_base);
    if (m0 >= lim) return;
    if (lim < M) M = lim;
  }
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int i = lane & 15, kq = lane >> 4;
  floatx4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int nk = (K + NK - 1) / NK;
  auto mma = [&](uint16_t (*As)[NLD], uint16_t (*Bs)[NLD]) {
#pragma unroll
    for (int ks = 0; ks < NK; ks += 32) {
      bf16x8 af[4], bfv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        af[t] = *reinterpret_cast<const bf16x8*>(&As[wm + 16 * t + i][ks + 8 * kq]);
        bfv[t] = *reinterpret_cast<const bf16x8*>(&Bs[wn + 16 * t + i][ks + 8 * kq]);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfv[b], acc[a][b], 0, 0, 0);
    }
  };
  NFrag f;
  nfetch(f, A, lda, M, B, ldb, N, K, m0, n0, 0);
  nstore(As0, Bs0, f);
  __syncthreads();
  // LDS buffer k % 2 holds depth tile k while tile k + 1 loads into registers;
  // the buffer written in a step was last read in the step before, which the
  // barrier closed
  for (int k = 0; k < nk; k += 2) {
    if (k + 1 < nk) nfetch(f, A, lda, M, B, ldb, N, K, m0, n0, (k + 1) * NK);
    mma(As0, Bs0);
    if (k + 1 < nk) nstore(As1, Bs1, f);
    __syncthreads();
    if (k + 1 >= nk) break;
    if (k + 2 < nk) nfetch(f, A, lda, M, B, ldb, N, K, m0, n0, (k + 2) * NK);
    mma(As1, Bs1);
    if (k + 2 < nk) nstore(As0, Bs0, f);
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = m0 + wm + 16 * a + 4 * kq + j;
        const int col = n0 + wn + 16 * b + i;
        if (row < M && col < N) epi_store<EPI>(e, row, col, acc[a][b][j]);
      }
}
constexpr size_t NN_LDS = (size_t)2 * (NM + NN) * NLD * sizeof(uint16_t);

// ------------------------------- 256 x 256 tiles, LDS filled by direct loads
// The same product as gemm_nn_kernel (both operands k-contiguous) for large
// shapes with K % 64 == 0.  One workgroup of 8 waves (two per SIMD) per
// 256 x 256 tile of C; wave w owns rows 128 (w / 4) .. + 127 and columns
// 64 (w % 4) .. + 63 as 8 x 4 MFMA 16x16x32 tiles.  Depth tiles of 64 go from
// global memory straight into the LDS (global_load_lds_dwordx4: lane l of a
// wave instruction writes 16 bytes at the instruction's LDS base + 16 l), into
// two buffers: tile k + 1 is requested before tile k is multiplied, so its
// latency hides behind a whole tile of MFMAs, with no registers holding it.
// A row of a depth tile is 8 chunks of 16 bytes; chunk c of row r sits at
// position c ^ (r % 8) of the row (an XOR swizzle), so the 16 rows read by
// one ds_read_b128 of an MFMA fragment spread over the LDS banks.  Rows past M
// or N load a valid clamped row (their results are never stored).  Every
// output element is accumulated in the same order as in gemm_nn_kernel (depth
// tiles of 64, MFMA steps of 32), so the kernels give identical results.
constexpr int BM = 256, BN = 256;
constexpr int BIG_GROUP = 4;  // row blocks per tile group
constexpr size_t DL_STAGE = (size_t)(BM + BN) * NK * sizeof(uint16_t);  // 64 KiB
constexpr size_t BIG_LDS = 2 * DL_STAGE;

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Requests one operand's 256 x 64 depth tile (rows r0.., depths k0..) into
// the LDS at `dst`: 2048 chunks, 4 wave instructions of 64 chunks per wave.
__device__ __forceinline__ void dl_fetch(uint16_t* dst, const uint16_t* __restrict__ X, int ld, int R, int r0,
                                         int k0) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int u = h * 8 + wave;         // instruction index: LDS bytes 1024 u .. + 1023
    const int c = u * 64 + lane;        // chunk of the tile in LDS order
    const int row = c >> 3, pos = c & 7;
    const int kc = pos ^ (row & 7);     // the depth chunk stored at that position
    const int gr = min(r0 + row, R - 1);
    __builtin_amdgcn_global_load_lds((const void*)(X + (size_t)gr * ld + k0 + kc * 8),
                                     (lds_ptr_t)(dst + (size_t)u * 512), 16, 0, 0);
  }
}

// 8 bf16 of row r, depths 8 kc .. 8 kc + 7, of a swizzled depth tile.
__device__ __forceinline__ bf16x8 dl_frag(const uint16_t* S, int r, int kc) {
  return *reinterpret_cast<const bf16x8*>(S + ((size_t)r * 8 + (kc ^ (r & 7))) * 8);
}

template <int EPI>
__global__ __launch_bounds__(512) void gemm_big_kernel(const uint16_t* __restrict__ A, int lda,
                                                       const uint16_t* __restrict__ B, int ldb, int M, int N, int K,
                                                       Epi e, const int32_t* __restrict__ mlim, int tiles_n,
                                                       int ntiles) {
  extern __shared__ __attribute__((aligned(16))) uint16_t dsm[];
  // XCD-contiguous tile order: workgroup b runs on XCD b % 8; inside an XCD's
  // range, tiles go in groups of BIG_GROUP row blocks (down a group's rows
  // first, then across its columns), so the tiles that run together on one
  // XCD read few distinct operand panels through its L2
  const int nb = (int)gridDim.x, per = nb / 8;
  const int bid = (int)blockIdx.x;
  const int tile = (nb % 8 == 0) ? (bid % 8) * per + bid / 8 : bid;
  if (tile >= ntiles) return;
  const int tiles_m = ntiles / tiles_n, in_group = BIG_GROUP * tiles_n;
  const int first = tile / in_group * BIG_GROUP, gsz = min(tiles_m - first, BIG_GROUP), r = tile % in_group;
  const int m0 = (first + r % gsz) * BM, n0 = (r / gsz) * BN;
  if (mlim) {
    const int lim = (int)(*mlim - e.row_base);
    if (m0 >= lim) return;
    if (lim < M) M = lim;
  }
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int wm = (wave >> 2) * 128, wn = (wave & 3) * 64;
  const int i = lane & 15, kq = lane >> 4;
  floatx4 acc[8][4];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int nk = K / NK;
  uint16_t* const st0 = dsm;
  uint16_t* const st1 = dsm + DL_STAGE / sizeof(uint16_t);
  dl_fetch(st0, A, lda, M, m0, 0);
  dl_fetch(st0 + BM * NK, B, ldb, N, n0, 0);
  for (int k = 0; k < nk; ++k) {
    __builtin_amdgcn_s_waitcnt(0);  // this wave's requests for tile k have landed
    __syncthreads();                // every wave's have, and every wave is done with tile k - 1
    if (k + 1 < nk) {               // the other buffer (last read for tile k - 1) takes tile k + 1
      uint16_t* nx = (k & 1) ? st0 : st1;
      dl_fetch(nx, A, lda, M, m0, (k + 1) * NK);
      dl_fetch(nx + BM * NK, B, ldb, N, n0, (k + 1) * NK);
    }
    const uint16_t* As = (k & 1) ? st1 : st0;
    const uint16_t* Bs = As + BM * NK;
#pragma unroll
    for (int ks = 0; ks < NK; ks += 32) {
      const int kc = (ks >> 3) + kq;
      bf16x8 bfv[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) bfv[t] = dl_frag(Bs, wn + 16 * t + i, kc);
#pragma unroll
      for (int a = 0; a < 8; ++a) {
        const bf16x8 af = dl_frag(As, wm + 16 * a + i, kc);
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfv[b], acc[a][b], 0, 0, 0);
      }
    }
  }
  float ct[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int col = n0 + wn + 16 * b + i;
    ct[b] = col < N ? epi_col_term<EPI>(e, col) : 0.f;
  }
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = m0 + wm + 16 * a + 4 * kq + j;
      const float rt = row < M ? epi_row_term<EPI>(e, row) : 0.f;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int col = n0 + wn + 16 * b + i;
        if (row < M && col < N) epi_store_t<EPI>(e, row, col, acc[a][b][j], rt, ct[b]);
      }
    }
}
constexpr int BIG_MIN_ROWS = 512;  // fewer rows: the 256 x 128 tiles keep more workgroups busy
constexpr int64_t BIG_MIN_TILES = 256;  // fewer 256 x 256 tiles than CUs: the 256 x 128 tiles

template <bool AT, bool BT, int EPI>
void gemm(const uint16_t* A, int lda, const uint16_t* B, int ldb, int M, int N, int K, const Epi& e, hipStream_t s,
          const int32_t* mlim = nullptr) {
  if (M <= 0 || N <= 0) return;
  if constexpr (!AT && !BT) {
    if ((K % 8) == 0 && (lda % 8) == 0 && (ldb % 8) == 0 && ((uintptr_t)A % 16) == 0 && ((uintptr_t)B % 16) == 0 &&
        M >= BIG_MIN_ROWS && N >= BN && (K % NK) == 0 &&
        (int64_t)((M + BM - 1) / BM) * ((N + BN - 1) / BN) >= BIG_MIN_TILES) {
      const int tn = (N + BN - 1) / BN, tm = (M + BM - 1) / BM;
      const int nt = tn * tm;
      const int grid = (nt + 7) / 8 * 8;  // a multiple of 8 for the XCD-contiguous order
      static bool lds_set = false;        // more than 64 KiB of dynamic LDS
      if (!lds_set) {
        HIP_TRY(hipFuncSetAttribute((const void*)gemm_big_kernel<EPI>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)BIG_LDS));
        lds_set = true;
      }
      hipLaunchKernelGGL((gemm_big_kernel<EPI>), dim3((unsigned)grid), dim3(512), BIG_LDS, s, A, lda, B, ldb, M, N, K,
                         e, mlim, tn, nt);
      HIP_TRY(hipGetLastError());
      return;
    }
    if ((K % 8) == 0 && (lda % 8) == 0 && (ldb % 8) == 0 && ((uintptr_t)A % 16) == 0 && ((uintptr_t)B % 16) == 0) {
      const int tn = (N + NN - 1) / NN, tm = (M + NM - 1) / NM;
      const int nt = tn * tm;
      const int grid = (nt + 7) / 8 * 8;  // a multiple of 8 for the XCD-contiguous order
      static bool lds_set = false;        // more than 64 KiB of dynamic LDS
      if (!lds_set) {
        HIP_TRY(hipFuncSetAttribute((const void*)gemm_nn_kernel<EPI>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)NN_LDS));
        lds_set = true;
      }
      hipLaunchKernelGGL((gemm_nn_kernel<EPI>), dim3((unsigned)grid), dim3(512), NN_LDS, s, A, lda, B, ldb, M, N, K, e,
                         mlim, tn, nt);
      HIP_TRY(hipGetLastError());
      return;
    }
  }
  const dim3 grid((unsigned)((N + GN - 1) / GN), (unsigned)((M + GM - 1) / GM));
  hipLaunchKernelGGL((gemm_bf16_kernel<AT, BT, EPI>), grid, dim3(256), 0, s, A, lda, B, ldb, M, N, K, e, mlim);
  HIP_TRY(hipGetLastError());
}

// ------------------------------------------------------ elementwise kernels
__global__ void to_bf16_kernel(const float* __restrict__ x, int64_t n, uint16_t* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = to_bf16(x[i]);
}

// xh[r][j] = bf16((X[rows[r]][j] - mean[j]) / std[j]) (rows == null: r itself)
// h = bf16(gelu(z + bias[col])) over a rows x cols block of FP32 dot products
__global__ void gelu_bias_bf16_kernel(const float* __restrict__ z, int64_t rows, int cols,
                                      const float* __restrict__ bias, uint16_t* __restrict__ h) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < rows * cols) h[i] = to_bf16(gelu(z[i] + bias[i % cols]));
}

__global__ void negate_kernel(const float* __restrict__ a, int64_t n, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = -a[i];
}

__global__ void standardize_kernel(const float* __restrict__ X, const int32_t* __restrict__ rows, int64_t n, int d,
                                   const float* __restrict__ mean, const float* __restrict__ stdv,
                                   uint16_t* __restrict__ xh, const int32_t* __restrict__ nlim) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * d) return;
  const int64_t r = i / d;
  const int j = (int)(i % d);
  if (nlim && r >= *nlim) return;
  const int64_t src = rows ? rows[r] : r;
  xh[i] = to_bf16((X[src * d + j] - mean[j]) / stdv[j]);
}

// Column mean and standard deviation (FP64 accumulation) of n x d rows.
__global__ void col_stats_kernel(const float* __restrict__ X, int64_t n, int d, float* __restrict__ mean,
                                 float* __restrict__ stdv) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  double s = 0.0;
  for (int64_t r = 0; r < n; ++r) s += X[r * d + j];
  const double mu = s / (double)n;
  double v = 0.0;
  for (int64_t r = 0; r < n; ++r) {
    const double t = X[r * d + j] - mu;
    v += t * t;
  }
  mean[j] = (float)mu;
  const double sd = sqrt(v / (double)n);
  stdv[j] = (float)(sd > 1e-12 ? sd : 1.0);
}

// Softmax cross-entropy of one row of scores against the target distribution
// of `kt` grain ids (each weighing 1 / kt): ds = (p - y) / B in FP32 and BF16,
// and the row's loss.  One workgroup of 256 per row.
__global__ __launch_bounds__(256) void softmax_ce_kernel(const float* __restrict__ S, int G,
                                                         const int32_t* __restrict__ tgt, int kt, float invB,
                                                         float* __restrict__ ds, uint16_t* __restrict__ dsb,
                                                         float* __restrict__ loss) {
  __shared__ float red[256];
  const int64_t r = blockIdx.x;
  const float* s = S + r * G;
  float m = -__builtin_inff();
  for (int g = threadIdx.x; g < G; g += 256) m = fmaxf(m, s[g]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  m = red[0];
  __syncthreads();
  float z = 0.f;
  for (int g = threadIdx.x; g < G; g += 256) z += expf(s[g] - m);
  red[threadIdx.x] = z;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  z = red[0];
  const float logz = logf(z);
  const int32_t* t = tgt + r * kt;
  const float w = 1.f / (float)kt;
  for (int g = threadIdx.x; g < G; g += 256) {
    float y = 0.f;
    for (int q = 0; q < kt; ++q) y += t[q] == g ? w : 0.f;
    const float p = expf(s[g] - m) / z;
    const float v = (p - y) * invB;
    ds[r * G + g] = v;
    dsb[r * G + g] = to_bf16(v);
  }
  if (threadIdx.x == 0) {
    float l = 0.f;
    for (int q = 0; q < kt; ++q) {
      const int g = t[q];
      if (g >= 0 && g < G) l -= w * (s[g] - m - logz);
    }
    atomicAdd(loss, l * invB);
  }
}

// out[n] = sum over rows of X[r][n] (bias gradients).
__global__ void col_sum_kernel(const float* __restrict__ X, int rows, int N, float* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float acc = 0.f;
  for (int r = 0; r < rows; ++r) acc += X[(size_t)r * N + n];
  out[n] = acc;
}

// One Adam step of a tensor, and its BF16 copy when given.
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2, uint16_t* __restrict__ wb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  if (wb) wb[i] = to_bf16(wi);
}

// Max softmax probability of each row of negated scores (1 / z, z from the
// top-P pass that read the row); rows below tau are appended to the fallback
// list.  One thread per row.
__global__ __launch_bounds__(256) void fallback_select_kernel(const float2* __restrict__ znorm, int64_t rows,
                                                              float tau, int32_t* __restrict__ fb_rows,
                                                              int32_t* __restrict__ fb_count,
                                                              const int32_t* __restrict__ nlim) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows || (nlim && r >= *nlim)) return;
  if (1.f / znorm[r].y < tau) fb_rows[atomicAdd(fb_count, 1)] = (int32_t)r;
}

// Probability-mass probe budget of one learned row (one wave): with
// m = max score and z = sum_g exp(s_g - m) over all G scores, slots are kept
// up to and including the first j at which sum_{i <= j} exp(s_{p_i} - m) / z
// reaches mass; later slots become probe -1 (pdist +inf).
__global__ __launch_bounds__(256) void mass_cut_kernel(const float* __restrict__ negS, const float2* __restrict__ znorm,
                                                       int64_t rows, int G, int P, float mass,
                                                       int32_t* __restrict__ probes, float* __restrict__ pdist,
                                                       const int32_t* __restrict__ nlim) {
  const int lane = lane_id();
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows || (nlim && r >= *nlim)) return;
  const float* s = negS + r * G;  // negated scores
  // m and z of the row, from the top-P pass that read the row
  const float2 mz = znorm[r];
  const float mn = mz.x, z = mz.y;
  // lane j < P: probability of slot j; an inclusive prefix sum over the lanes
  const int32_t pj = lane < P ? probes[r * P + lane] : -1;
  float p = pj >= 0 ? expf(mn - s[pj]) / z : 0.f;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const float t = __shfl_up(p, o, 64);
    if (lane >= o) p += t;
  }
  const uint64_t reached = __ballot(lane < P && p >= mass);
  if (!reached) return;
  const int cut = __builtin_ctzll(reached);  // the first slot that reaches the mass: kept
  if (lane > cut && lane < P) {
    probes[r * P + lane] = -1;
    if (pdist) pdist[r * P + lane] = __builtin_inff();
  }
}

// Copies the query rows of the fallback list into a compact block.
__global__ void gather_rows_kernel(const float* __restrict__ Q, int d, const int32_t* __restrict__ rows,
                                   const int32_t* __restrict__ count, float* __restrict__ out) {
  const int r = blockIdx.x;
  if (r >= *count) return;
  const float* src = Q + (size_t)rows[r] * d;
  for (int j = threadIdx.x; j < d; j += blockDim.x) out[(size_t)r * d + j] = src[j];
}

// Writes the centroid-routing probes of the fallback rows back in place.
__global__ void scatter_probes_kernel(const int32_t* __restrict__ rows, const int32_t* __restrict__ count, int P,
                                      const int32_t* __restrict__ src, const float* __restrict__ srcd,
                                      int32_t* __restrict__ probes, float* __restrict__ pdist) {
  const int r = blockIdx.x;
  if (r >= *count) return;
  const int q = rows[r];
  for (int j = threadIdx.x; j < P; j += blockDim.x) {
    probes[(size_t)q * P + j] = src[(size_t)r * P + j];
    if (pdist) pdist[(size_t)q * P + j] = srcd ? srcd[(size_t)r * P + j] : 0.f;
  }
}

// Grain of every original row: lab[perm[pos]] = grain holding position pos.
__global__ void row_grain_kernel(const int32_t* __restrict__ perm, const int32_t* __restrict__ goff, int G, int64_t N,
                                 int32_t* __restrict__ lab) {
  const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pos >= N) return;
  int lo = 0, hi = G;  // largest g with goff[g] <= pos
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (goff[mid] <= pos)
      lo = mid;
    else
      hi = mid;
  }
  lab[perm[pos]] = lo;
}

__global__ void map_ids_kernel(const int32_t* __restrict__ ids, int64_t n, const int32_t* __restrict__ lab,
                               int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = ids[i] >= 0 ? lab[ids[i]] : -1;
}

inline unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

uint64_t splitmix(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
double uni(uint64_t seed, uint64_t stream, uint64_t i) {
  return (double)(splitmix(splitmix(seed ^ (stream * 0xD1B54A32D192ED03ull)) + i) >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace

// ------------------------------------------------------------------ router
void Router::alloc(int d_, int h1_, int h2_, int G_) {
  d = d_;
  h1 = h1_;
  h2 = h2_;
  G = G_;
  const int64_t n[3] = {(int64_t)h1 * d, (int64_t)h2 * h1, (int64_t)G * h2};
  const int64_t nb[3] = {h1, h2, G};
  for (int l = 0; l < 3; ++l) {
    HIP_TRY(hipMalloc((void**)&W[l], sizeof(float) * n[l]));
    HIP_TRY(hipMalloc((void**)&b[l], sizeof(float) * nb[l]));
    HIP_TRY(hipMalloc((void**)&Wb[l], sizeof(uint16_t) * n[l]));
  }
  HIP_TRY(hipMalloc((void**)&mean, sizeof(float) * d));
  HIP_TRY(hipMalloc((void**)&stdv, sizeof(float) * d));
}

Router::~Router() {
  for (int l = 0; l < 3; ++l) {
    if (W[l]) (void)hipFree(W[l]);
    if (b[l]) (void)hipFree(b[l]);
    if (Wb[l]) (void)hipFree(Wb[l]);
  }
  if (mean) (void)hipFree(mean);
  if (stdv) (void)hipFree(stdv);
}

int64_t Router::wsize(int l) const { return l == 0 ? (int64_t)h1 * d : l == 1 ? (int64_t)h2 * h1 : (int64_t)G * h2; }
int64_t Router::bsize(int l) const { return l == 0 ? h1 : l == 1 ? h2 : G; }

void Router::refresh_bf16(hipStream_t s) {
  for (int l = 0; l < 3; ++l)
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(wsize(l))), dim3(256), 0, s, W[l], wsize(l), Wb[l]);
  HIP_TRY(hipGetLastError());
}

// Learned routing of nq rows of Q: probes (nq x P) by descending score (ties:
// lower grain), pdist = the negated scores; rows whose largest softmax
// probability is below tau use centroid routing instead.
namespace {
// FP32 rows split into BF16 high and low parts (nearest even): an output row is
// [hi | hi | lo] (queries) or [hi | lo | hi] (centroids, corder), so that one
// product over 3d depths gives q_hi c_hi + q_hi c_lo + q_lo c_hi.
__global__ void split3_kernel(const float* __restrict__ X, int64_t rows, int d, int corder,
                              uint16_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * d) return;
  const int64_t r = i / d;
  const int k = (int)(i - r * d);
  const float x = X[i];
  const uint16_t h = to_bf16(x);
  const uint16_t l = to_bf16(x - __uint_as_float((uint32_t)h << 16));
  uint16_t* o = out + r * 3 * d;
  o[k] = h;
  o[d + k] = corder ? l : h;
  o[2 * d + k] = corder ? h : l;
}
std::mutex g_split_mu;
}  // namespace

void ensure_centroid_split(Index& ix, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_split_mu);
  if (ix.cent_split) return;
  if (ix.d % 8 != 0) throw ArgError{HNTL_EUNSUPPORTED, "split-BF16 routing needs d % 8 == 0"};
  uint16_t* p = dev_alloc<uint16_t>(&ix, (size_t)ix.G * 3 * ix.d);
  const int64_t n = (int64_t)ix.G * ix.d;
  hipLaunchKernelGGL(split3_kernel, dim3(blocks(n)), dim3(256), 0, s, ix.centroids, (int64_t)ix.G, (int)ix.d, 1, p);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  ix.cent_split = p;
}

void launch_dist_bf16x3(const Index& ix, const float* A, const float* an, int64_t rows, uint16_t* As, float* D,
                        hipStream_t s, const int32_t* nlim, int64_t row_base) {
  if (rows <= 0) return;
  if (!ix.cent_split) throw ArgError{HNTL_ESTATE, "split-BF16 routing: centroid split not built"};
  const int64_t n = rows * ix.d;
  hipLaunchKernelGGL(split3_kernel, dim3(blocks(n)), dim3(256), 0, s, A, rows, (int)ix.d, 0, As);
  HIP_TRY(hipGetLastError());
  Epi e{};
  e.C = D;
  e.ldc = (int)ix.G;
  e.an = an;
  e.bn = ix.cnorm;
  e.row_base = row_base;
  const int K3 = 3 * (int)ix.d;
  gemm<false, false, EPI_DIST>(As, K3, ix.cent_split, K3, (int)rows, (int)ix.G, K3, e, s, nlim);
}

// Plain BF16 expansion distances: <a, mu> from bf16(a) . bf16(mu) (the high
// parts of the split centroid rows, row stride 3d), FP32 accumulation.
void launch_dist_bf16(const Index& ix, const float* A, const float* an, int64_t rows, uint16_t* As, float* D,
                      hipStream_t s, const int32_t* nlim, int64_t row_base) {
  if (rows <= 0) return;
  if (!ix.cent_split) throw ArgError{HNTL_ESTATE, "BF16 routing: centroid split not built"};
  const int64_t n = rows * ix.d;
  hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(n)), dim3(256), 0, s, A, n, As);
  HIP_TRY(hipGetLastError());
  Epi e{};
  e.C = D;
  e.ldc = (int)ix.G;
  e.an = an;
  e.bn = ix.cnorm;
  e.row_base = row_base;
  const int d = (int)ix.d;
  gemm<false, false, EPI_DIST>(As, d, ix.cent_split, 3 * d, (int)rows, (int)ix.G, d, e, s, nlim);
}

size_t RouteScratch::layout(char* base, const Index& ix, int64_t nq, int form_) {
  form = form_;
  chunk = std::min<int64_t>(std::max<int64_t>(nq, 1), std::max<int64_t>(64, ((int64_t)1 << 28) / ix.G));
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = (off + 255) / 256 * 256;
    char* p = base ? base + off : nullptr;
    off += std::max<size_t>(bytes, 1);
    return p;
  };
  qn = (float*)take(4 * (size_t)std::max<int64_t>(nq, 1));
  D = (float*)take(4 * (size_t)chunk * ix.G);
  const int w = form == ROUTE_BF16X3 ? 3 : form == ROUTE_BF16 ? 1 : 0;
  As = w ? (uint16_t*)take(2 * (size_t)chunk * w * ix.d) : nullptr;
  return off;
}

float route_err(int form) {
  // Bound on |expansion - exact| per entry, as a multiple of ||q||^2 + ||mu||^2
  // (|<q, mu>| <= (||q||^2 + ||mu||^2) / 2):
  //  - FP32 MFMA: products and sums in FP32 over d <= 1024 terms, about 1e-5;
  //  - split BF16: the dropped lo x lo term and the parts' own rounding (about
  //    3 x 2^-18) plus FP32 accumulation over 3d terms;
  //  - plain BF16: each operand rounded to nearest even (2^-9 relative each),
  //    2^-8 + 2^-18 of sum |q_j mu_j|, plus the FP32 accumulation.
  // Each factor also covers the FP32 norms and the final combination.
  return form == ROUTE_BF16 ? 4.0e-3f : 5.0e-5f;
}

void launch_route_centroid(const Index& ix, const float* Q, int64_t nq, int P, const RouteScratch& w,
                           int32_t* probes, float* pdist, hipStream_t s, const int32_t* nlim,
                           unsigned int* overflow) {
  if (nq <= 0) return;
  if (w.form != ROUTE_F32 && !ix.cent_split) throw ArgError{HNTL_ESTATE, "BF16 routing: centroid split not built"};
  const int G = (int)ix.G, d = (int)ix.d;
  launch_row_norms(Q, nq, d, w.qn, s);
  for (int64_t q0 = 0; q0 < nq; q0 += w.chunk) {
    const int64_t rows = std::min<int64_t>(w.chunk, nq - q0);
    const float* Qc = Q + q0 * d;
    if (rows <= 16 || w.form == ROUTE_F32)  // a few rows: exact direct differences (FP32 MFMA expansion otherwise)
      launch_dist_matrix(Qc, w.qn + q0, rows, ix.centroids, ix.cnorm, G, d, w.D, s, nlim, q0);
    else if (w.form == ROUTE_BF16X3)
      launch_dist_bf16x3(ix, Qc, w.qn + q0, rows, w.As, w.D, s, nlim, q0);
    else
      launch_dist_bf16(ix, Qc, w.qn + q0, rows, w.As, w.D, s, nlim, q0);
    launch_topk_rows(w.D, rows, G, P, probes + q0 * P, pdist ? pdist + q0 * P : nullptr, s, Qc, w.qn + q0,
                     ix.centroids, ix.cnorm, d, route_err(w.form), nlim, q0, overflow);
  }
}

void launch_route_learned(const Index& ix, const float* Q, int64_t nq, int P, float tau, int32_t* probes,
                          float* pdist, const RouterScratch& w, hipStream_t s, const int32_t* nlim, float mass) {
  const Router& rt = *ix.router;
  hipLaunchKernelGGL(standardize_kernel, dim3(blocks(nq * rt.d)), dim3(256), 0, s, Q, nullptr, nq, rt.d, rt.mean,
                     rt.stdv, w.xh, nlim);
  HIP_TRY(hipGetLastError());
  Epi e{};
  e.bias = rt.b[0];
  e.H = w.h1;
  e.ldh = rt.h1;
  gemm<false, false, EPI_BIAS_GELU>(w.xh, rt.d, rt.Wb[0], rt.d, (int)nq, rt.h1, rt.d, e, s, nlim);
  e.bias = rt.b[1];
  e.H = w.h2;
  e.ldh = rt.h2;
  gemm<false, false, EPI_BIAS_GELU>(w.h1, rt.h1, rt.Wb[1], rt.h1, (int)nq, rt.h2, rt.h1, e, s, nlim);
  // negS = -(h2 W3^T + b3): the P smallest are the P largest scores
  Epi o{};
  o.C = w.negS;
  o.ldc = rt.G;
  o.bias = rt.b[2];
  o.scale = -1.f;
  gemm<false, false, EPI_BIAS_F32>(w.h2, rt.h2, rt.Wb[2], rt.h2, (int)nq, rt.G, rt.h2, o, s, nlim);
  const bool budget = mass > 0.f && mass < 1.f && P > 1;
  launch_topk_rows(w.negS, nq, rt.G, P, probes, pdist, s, nullptr, nullptr, nullptr, nullptr, 0, 0.f, nlim, 0,
                   nullptr, (budget || tau > 0.f) ? w.znorm : nullptr);
  if (budget) {
    hipLaunchKernelGGL(mass_cut_kernel, dim3(blocks(nq, 4)), dim3(256), 0, s, w.negS, w.znorm, nq, rt.G, P, mass,
                       probes, pdist, nlim);
    HIP_TRY(hipGetLastError());
  }
  if (tau > 0.f) {
    launch_fill_i32(w.fb_count, 1, 0, s);
    hipLaunchKernelGGL(fallback_select_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, w.znorm, nq, tau,
                       w.fb_rows, w.fb_count, nlim);
    hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)nq), dim3(256), 0, s, Q, (int)ix.d, w.fb_rows, w.fb_count,
                       w.fb_Q);
    launch_row_norms(w.fb_Q, nq, (int)ix.d, w.fb_qn, s);
    const int64_t chunk = std::max<int64_t>(64, ((int64_t)1 << 28) / ix.G);
    for (int64_t q0 = 0; q0 < nq; q0 += chunk) {
      const int64_t rows = std::min<int64_t>(chunk, nq - q0);
      launch_dist_matrix(w.fb_Q + q0 * ix.d, w.fb_qn + q0, rows, ix.centroids, ix.cnorm, (int)ix.G, (int)ix.d,
                         w.negS, s, w.fb_count, q0);  // the scores are no longer needed: reuse as scratch
      launch_topk_rows(w.negS, rows, (int)ix.G, P, w.fb_probes + q0 * P, w.fb_pdist + q0 * P, s,
                       w.fb_Q + q0 * ix.d, w.fb_qn + q0, ix.centroids, ix.cnorm, (int)ix.d, route_err(ROUTE_F32),
                       w.fb_count, q0, nullptr);
    }
    hipLaunchKernelGGL(scatter_probes_kernel, dim3((unsigned)nq), dim3(64), 0, s, w.fb_rows, w.fb_count, P,
                       w.fb_probes, w.fb_pdist, probes, pdist);
    HIP_TRY(hipGetLastError());
  }
}

// Buffers of launch_route_learned carved from one block (base == nullptr:
// sizing pass); returns the bytes used.
size_t RouterScratch::layout(char* base, const Index& ix, int64_t nq, int P) {
  const Router& rt = *ix.router;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = (off + 255) / 256 * 256;
    char* p = base ? base + off : nullptr;
    off += std::max<size_t>(bytes, 1);
    return p;
  };
  xh = (uint16_t*)take(2 * (size_t)nq * rt.d);
  h1 = (uint16_t*)take(2 * (size_t)nq * rt.h1);
  h2 = (uint16_t*)take(2 * (size_t)nq * rt.h2);
  const int64_t chunk = std::min<int64_t>(nq, std::max<int64_t>(64, ((int64_t)1 << 28) / ix.G));
  negS = (float*)take(4 * (size_t)std::max<int64_t>(nq * rt.G, chunk * ix.G));
  fb_rows = (int32_t*)take(4 * (size_t)nq);
  fb_count = (int32_t*)take(4);
  fb_Q = (float*)take(4 * (size_t)nq * ix.d);
  fb_qn = (float*)take(4 * (size_t)nq);
  fb_probes = (int32_t*)take(4 * (size_t)nq * P);
  fb_pdist = (float*)take(4 * (size_t)nq * P);
  znorm = (float2*)take(sizeof(float2) * (size_t)nq);
  return off;
}

namespace {

// Training state: Adam moments, gradients, activations of one batch.
struct Trainer {
  Router& rt;
  int B;
  hipStream_t s;
  std::vector<void*> mem;
  float* m[6] = {};
  float* v[6] = {};
  float* g[6] = {};
  uint16_t *xh = nullptr, *h1 = nullptr, *h2 = nullptr, *dsb = nullptr, *da2b = nullptr, *da1b = nullptr;
  float *a1 = nullptr, *a2 = nullptr, *S = nullptr, *ds = nullptr, *da2 = nullptr, *da1 = nullptr, *loss = nullptr;
  int32_t* rows = nullptr;
  int32_t* tgt = nullptr;
  int step = 0;

  template <class T>
  T* alloc(size_t n) {
    void* p = nullptr;
    HIP_TRY(hipMalloc(&p, sizeof(T) * std::max<size_t>(n, 1)));
    mem.push_back(p);
    return (T*)p;
  }
  Trainer(Router& r, int B_, hipStream_t st) : rt(r), B(B_), s(st) {
    for (int l = 0; l < 3; ++l) {
      m[2 * l] = alloc<float>(rt.wsize(l));
      v[2 * l] = alloc<float>(rt.wsize(l));
      g[2 * l] = alloc<float>(rt.wsize(l));
      m[2 * l + 1] = alloc<float>(rt.bsize(l));
      v[2 * l + 1] = alloc<float>(rt.bsize(l));
      g[2 * l + 1] = alloc<float>(rt.bsize(l));
      HIP_TRY(hipMemsetAsync(m[2 * l], 0, sizeof(float) * rt.wsize(l), s));
      HIP_TRY(hipMemsetAsync(v[2 * l], 0, sizeof(float) * rt.wsize(l), s));
      HIP_TRY(hipMemsetAsync(m[2 * l + 1], 0, sizeof(float) * rt.bsize(l), s));
      HIP_TRY(hipMemsetAsync(v[2 * l + 1], 0, sizeof(float) * rt.bsize(l), s));
    }
    xh = alloc<uint16_t>((size_t)B * rt.d);
    h1 = alloc<uint16_t>((size_t)B * rt.h1);
    h2 = alloc<uint16_t>((size_t)B * rt.h2);
    a1 = alloc<float>((size_t)B * rt.h1);
    a2 = alloc<float>((size_t)B * rt.h2);
    S = alloc<float>((size_t)B * rt.G);
    ds = alloc<float>((size_t)B * rt.G);
    dsb = alloc<uint16_t>((size_t)B * rt.G);
    da2 = alloc<float>((size_t)B * rt.h2);
    da2b = alloc<uint16_t>((size_t)B * rt.h2);
    da1 = alloc<float>((size_t)B * rt.h1);
    da1b = alloc<uint16_t>((size_t)B * rt.h1);
    loss = alloc<float>(1);
    rows = alloc<int32_t>(B);
  }
  ~Trainer() {
    for (void* p : mem) (void)hipFree(p);
  }

  // Loss and gradients of the batch X[rows[0..B)] against targets tg (B x kt).
  void grad(const float* X, const int32_t* d_rows, const int32_t* tg, int kt) {
    const int d = rt.d, H1 = rt.h1, H2 = rt.h2, G = rt.G;
    hipLaunchKernelGGL(standardize_kernel, dim3(blocks((int64_t)B * d)), dim3(256), 0, s, X, d_rows, (int64_t)B, d,
                       rt.mean, rt.stdv, xh, nullptr);
    Epi e{};
    e.C = a1;
    e.ldc = H1;
    e.bias = rt.b[0];
    e.H = h1;
    e.ldh = H1;
    gemm<false, false, EPI_BIAS_GELU>(xh, d, rt.Wb[0], d, B, H1, d, e, s);
    e.C = a2;
    e.ldc = H2;
    e.bias = rt.b[1];
    e.H = h2;
    e.ldh = H2;
    gemm<false, false, EPI_BIAS_GELU>(h1, H1, rt.Wb[1], H1, B, H2, H1, e, s);
    Epi o{};
    o.C = S;
    o.ldc = G;
    o.bias = rt.b[2];
    o.scale = 1.f;
    gemm<false, false, EPI_BIAS_F32>(h2, H2, rt.Wb[2], H2, B, G, H2, o, s);
    HIP_TRY(hipMemsetAsync(loss, 0, sizeof(float), s));
    hipLaunchKernelGGL(softmax_ce_kernel, dim3(B), dim3(256), 0, s, S, G, tg, kt, 1.f / (float)B, ds, dsb, loss);
    HIP_TRY(hipGetLastError());
    // layer 3: gW3[g][k] = sum_b ds[b][g] h2[b][k]; dh2 = ds W3, times gelu'(a2)
    Epi w{};
    w.C = g[4];
    w.ldc = H2;
    gemm<true, true, EPI_F32>(dsb, G, h2, H2, G, H2, B, w, s);
    hipLaunchKernelGGL(col_sum_kernel, dim3(blocks(G)), dim3(256), 0, s, ds, B, G, g[5]);
    Epi gg{};
    gg.Z = a2;
    gg.ldz = H2;
    gg.D = da2;
    gg.ldd = H2;
    gg.H = da2b;
    gg.ldh = H2;
    gemm<false, true, EPI_GELU_GRAD>(dsb, G, rt.Wb[2], H2, B, H2, G, gg, s);
    // layer 2
    w.C = g[2];
    w.ldc = H1;
    gemm<true, true, EPI_F32>(da2b, H2, h1, H1, H2, H1, B, w, s);
    hipLaunchKernelGGL(col_sum_kernel, dim3(blocks(H2)), dim3(256), 0, s, da2, B, H2, g[3]);
    gg.Z = a1;
    gg.ldz = H1;
    gg.D = da1;
    gg.ldd = H1;
    gg.H = da1b;
    gg.ldh = H1;
    gemm<false, true, EPI_GELU_GRAD>(da2b, H2, rt.Wb[1], H1, B, H1, H2, gg, s);
    // layer 1
    w.C = g[0];
    w.ldc = d;
    gemm<true, true, EPI_F32>(da1b, H1, xh, d, H1, d, B, w, s);
    hipLaunchKernelGGL(col_sum_kernel, dim3(blocks(H1)), dim3(256), 0, s, da1, B, H1, g[1]);
    HIP_TRY(hipGetLastError());
  }

  void adam(float lr) {
    ++step;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    for (int l = 0; l < 3; ++l) {
      hipLaunchKernelGGL(adam_kernel, dim3(blocks(rt.wsize(l))), dim3(256), 0, s, rt.W[l], g[2 * l], m[2 * l],
                         v[2 * l], rt.wsize(l), lr, b1, b2, eps, c1, c2, rt.Wb[l]);
      hipLaunchKernelGGL(adam_kernel, dim3(blocks(rt.bsize(l))), dim3(256), 0, s, rt.b[l], g[2 * l + 1],
                         m[2 * l + 1], v[2 * l + 1], rt.bsize(l), lr, b1, b2, eps, c1, c2, (uint16_t*)nullptr);
    }
    HIP_TRY(hipGetLastError());
  }
};

template <class F>
hntl_status guarded_r(F&& f) {
  try {
    f();
    return HNTL_OK;
  } catch (const ArgError& e) {
    return fail(e.code, e.msg);
  } catch (const HipError& e) {
    return fail(e.code == hipErrorOutOfMemory || e.code == hipErrorMemoryAllocation ? HNTL_ENOMEM : HNTL_EDEVICE,
                e.msg);
  } catch (const std::bad_alloc&) {
    return fail(HNTL_ENOMEM, "host allocation failed");
  }
}

void init_router(Index& ix, int h1, int h2) {
  if (h1 < 1 || h2 < 1) throw ArgError{HNTL_EINVAL, "hidden sizes must be positive"};
  if (ix.d % 8 || h1 % 8 || h2 % 8 || ix.G % 8)
    throw ArgError{HNTL_EUNSUPPORTED, "the router needs d, hidden sizes and G to be multiples of 8"};
  ix.router.reset(new Router());
  ix.router->alloc((int)ix.d, h1, h2, (int)ix.G);
}

}  // namespace

}  // namespace hntl

using namespace hntl;

extern "C" {

hntl_status hntl_router_set(hntl_index* index, uint32_t h1, uint32_t h2, const float* W1, const float* b1,
                            const float* W2, const float* b2, const float* W3, const float* b3, const float* mean,
                            const float* stdv) {
  set_error("");
  if (!index || !W1 || !b1 || !W2 || !b2 || !W3 || !b3 || !mean || !stdv) return fail(HNTL_EINVAL, "null pointer");
  return guarded_r([&] {
    Index& ix = index->ix;
    HIP_TRY(hipSetDevice(ix.device));
    init_router(ix, (int)h1, (int)h2);
    Router& rt = *ix.router;
    const float* Ws[3] = {W1, W2, W3};
    const float* bs[3] = {b1, b2, b3};
    for (int l = 0; l < 3; ++l) {
      HIP_TRY(hipMemcpy(rt.W[l], Ws[l], sizeof(float) * rt.wsize(l), hipMemcpyDefault));
      HIP_TRY(hipMemcpy(rt.b[l], bs[l], sizeof(float) * rt.bsize(l), hipMemcpyDefault));
    }
    HIP_TRY(hipMemcpy(rt.mean, mean, sizeof(float) * ix.d, hipMemcpyDefault));
    HIP_TRY(hipMemcpy(rt.stdv, stdv, sizeof(float) * ix.d, hipMemcpyDefault));
    rt.refresh_bf16(nullptr);
    HIP_TRY(hipDeviceSynchronize());
    rt.trained = true;
  });
}

hntl_status hntl_router_export(const hntl_index* index, uint32_t* h1, uint32_t* h2, float* W1, float* b1, float* W2,
                               float* b2, float* W3, float* b3, float* mean, float* stdv) {
  set_error("");
  if (!index) return fail(HNTL_EINVAL, "null index");
  const Index& ix = index->ix;
  if (!ix.router) return fail(HNTL_ESTATE, "the index has no router");
  return guarded_r([&] {
    HIP_TRY(hipSetDevice(ix.device));
    const Router& rt = *ix.router;
    if (h1) *h1 = (uint32_t)rt.h1;
    if (h2) *h2 = (uint32_t)rt.h2;
    float* Ws[3] = {W1, W2, W3};
    float* bs[3] = {b1, b2, b3};
    HIP_TRY(hipDeviceSynchronize());
    for (int l = 0; l < 3; ++l) {
      if (Ws[l]) HIP_TRY(hipMemcpy(Ws[l], rt.W[l], sizeof(float) * rt.wsize(l), hipMemcpyDefault));
      if (bs[l]) HIP_TRY(hipMemcpy(bs[l], rt.b[l], sizeof(float) * rt.bsize(l), hipMemcpyDefault));
    }
    if (mean) HIP_TRY(hipMemcpy(mean, rt.mean, sizeof(float) * ix.d, hipMemcpyDefault));
    if (stdv) HIP_TRY(hipMemcpy(stdv, rt.stdv, sizeof(float) * ix.d, hipMemcpyDefault));
  });
}

hntl_status hntl_router_grad(hntl_index* index, const float* X, uint32_t n, const int32_t* targets, uint32_t kt,
                             float* loss, float* gW1, float* gb1, float* gW2, float* gb2, float* gW3, float* gb3,
                             void* stream) {
  set_error("");
  if (!index || !X || !targets) return fail(HNTL_EINVAL, "null pointer");
  Index& ix = index->ix;
  if (!ix.router) return fail(HNTL_ESTATE, "the index has no router");
  if (n == 0 || kt == 0) return fail(HNTL_EINVAL, "n and kt must be positive");
  return guarded_r([&] {
    HIP_TRY(hipSetDevice(ix.device));
    hipStream_t s = (hipStream_t)stream;
    Router& rt = *ix.router;
    Trainer tr(rt, (int)n, s);
    std::vector<int32_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    HIP_TRY(hipMemcpyAsync(tr.rows, idx.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    tr.grad(X, tr.rows, targets, (int)kt);
    float* outs[6] = {gW1, gb1, gW2, gb2, gW3, gb3};
    for (int l = 0; l < 3; ++l) {
      if (outs[2 * l]) HIP_TRY(hipMemcpyAsync(outs[2 * l], tr.g[2 * l], sizeof(float) * rt.wsize(l), hipMemcpyDefault, s));
      if (outs[2 * l + 1])
        HIP_TRY(hipMemcpyAsync(outs[2 * l + 1], tr.g[2 * l + 1], sizeof(float) * rt.bsize(l), hipMemcpyDefault, s));
    }
    if (loss) HIP_TRY(hipMemcpyAsync(loss, tr.loss, sizeof(float), hipMemcpyDefault, s));
    HIP_TRY(hipStreamSynchronize(s));
  });
}

hntl_status hntl_router_forward(const hntl_index* index, const float* Q, uint32_t nq, float* scores, void* stream) {
  set_error("");
  if (!index || !Q || !scores) return fail(HNTL_EINVAL, "null pointer");
  const Index& ix = index->ix;
  if (!ix.router) return fail(HNTL_ESTATE, "the index has no router");
  if (nq == 0) return HNTL_OK;
  return guarded_r([&] {
    HIP_TRY(hipSetDevice(ix.device));
    hipStream_t s = (hipStream_t)stream;
    const Router& rt = *ix.router;
    Scratch sc(s);
    uint16_t* xh = sc.get<uint16_t>((size_t)nq * rt.d);
    uint16_t* h1 = sc.get<uint16_t>((size_t)nq * rt.h1);
    uint16_t* h2 = sc.get<uint16_t>((size_t)nq * rt.h2);
    hipLaunchKernelGGL(standardize_kernel, dim3(blocks((int64_t)nq * rt.d)), dim3(256), 0, s, Q, nullptr,
                       (int64_t)nq, rt.d, rt.mean, rt.stdv, xh, nullptr);
    Epi e{};
    e.bias = rt.b[0];
    e.H = h1;
    e.ldh = rt.h1;
    gemm<false, false, EPI_BIAS_GELU>(xh, rt.d, rt.Wb[0], rt.d, (int)nq, rt.h1, rt.d, e, s);
    e.bias = rt.b[1];
    e.H = h2;
    e.ldh = rt.h2;
    gemm<false, false, EPI_BIAS_GELU>(h1, rt.h1, rt.Wb[1], rt.h1, (int)nq, rt.h2, rt.h1, e, s);
    Epi o{};
    o.C = scores;
    o.ldc = rt.G;
    o.bias = rt.b[2];
    o.scale = 1.f;
    gemm<false, false, EPI_BIAS_F32>(h2, rt.h2, rt.Wb[2], rt.h2, (int)nq, rt.G, rt.h2, o, s);
  });
}

hntl_status hntl_knn(const hntl_index* index, const float* Q, uint32_t nq, uint32_t k, int32_t* ids, float* dist,
                     void* stream) {
  set_error("");
  if (!index || !Q || !ids) return fail(HNTL_EINVAL, "null pointer");
  if (nq == 0) return HNTL_OK;
  const Index& ix = index->ix;
  if (!ix.X) return fail(HNTL_ESTATE, "this index holds no raw vectors");
  return guarded_r([&] {
    HIP_TRY(hipSetDevice(ix.device));
    launch_knn(Q, nq, ix.X, (int64_t)ix.N, (int)ix.d, (int)k, ids, dist, (hipStream_t)stream);
  });
}

hntl_status hntl_router_train(hntl_index* index, const float* Qtrain, uint32_t n, const int32_t* targets,
                              const hntl_router_params* rp, float* epoch_loss, void* stream) {
  set_error("");
  if (!index || !Qtrain || !rp) return fail(HNTL_EINVAL, "null pointer");
  Index& ix = index->ix;
  const uint32_t B = rp->batch ? rp->batch : 1024;
  const uint32_t kt = rp->knn ? rp->knn : 10;
  if (n < B) return fail(HNTL_EINVAL, "need at least one full batch of training queries");
  if (kt > 16) return fail(HNTL_EUNSUPPORTED, "targets from at most 16 neighbours");
  return guarded_r([&] {
    HIP_TRY(hipSetDevice(ix.device));
    hipStream_t s = (hipStream_t)stream;
    const bool keep = (rp->flags & HNTL_ROUTER_KEEP_WEIGHTS) && ix.router;
    if (!keep) {
      init_router(ix, (int)(rp->hidden1 ? rp->hidden1 : 1024), (int)(rp->hidden2 ? rp->hidden2 : 1024));
      Router& rt = *ix.router;
      // He-style uniform initialisation from the counter-based generator
      for (int l = 0; l < 3; ++l) {
        const int fan_in = l == 0 ? rt.d : l == 1 ? rt.h1 : rt.h2;
        const double bound = std::sqrt((l < 2 ? 6.0 : 3.0) / fan_in);
        std::vector<float> w(rt.wsize(l));
        for (size_t i = 0; i < w.size(); ++i) w[i] = (float)((2.0 * uni(rp->seed, 10 + l, i) - 1.0) * bound);
        HIP_TRY(hipMemcpy(rt.W[l], w.data(), sizeof(float) * w.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemset(rt.b[l], 0, sizeof(float) * rt.bsize(l)));
      }
      hipLaunchKernelGGL(col_stats_kernel, dim3(blocks(ix.d)), dim3(256), 0, s, Qtrain, (int64_t)n, (int)ix.d,
                         rt.mean, rt.stdv);
      rt.refresh_bf16(s);
    }
    Router& rt = *ix.router;
    // targets: grains of each training query's exact kt nearest neighbours
    int32_t* tg = nullptr;
    std::unique_ptr<int32_t, void (*)(int32_t*)> tg_own(nullptr, [](int32_t* p) { (void)hipFree(p); });
    if (targets) {
      tg = const_cast<int32_t*>(targets);
    } else {
      if (!ix.X) throw ArgError{HNTL_ESTATE, "kNN training targets need the raw vectors (pass targets instead)"};
      int32_t *ids = nullptr, *lab = nullptr;
      HIP_TRY(hipMalloc((void**)&tg, sizeof(int32_t) * (size_t)n * kt));
      tg_own.reset(tg);
      HIP_TRY(hipMalloc((void**)&ids, sizeof(int32_t) * (size_t)n * kt));
      HIP_TRY(hipMalloc((void**)&lab, sizeof(int32_t) * ix.N));
      launch_knn(Qtrain, n, ix.X, (int64_t)ix.N, (int)ix.d, (int)kt, ids, nullptr, s);
      hipLaunchKernelGGL(row_grain_kernel, dim3(blocks((int64_t)ix.N)), dim3(256), 0, s, ix.perm, ix.goff, (int)ix.G,
                         (int64_t)ix.N, lab);
      hipLaunchKernelGGL(map_ids_kernel, dim3(blocks((int64_t)n * kt)), dim3(256), 0, s, ids, (int64_t)n * kt, lab, tg);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipStreamSynchronize(s));
      (void)hipFree(ids);
      (void)hipFree(lab);
    }
    Trainer tr(rt, (int)B, s);
    const uint32_t nb = n / B;  // full batches per epoch
    const uint32_t epochs = rp->epochs ? rp->epochs : 1;
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    int32_t* d_order = nullptr;
    int32_t* tgb = nullptr;
    HIP_TRY(hipMalloc((void**)&d_order, sizeof(int32_t) * n));
    HIP_TRY(hipMalloc((void**)&tgb, sizeof(int32_t) * (size_t)B * kt));
    std::unique_ptr<int32_t, void (*)(int32_t*)> o1(d_order, [](int32_t* p) { (void)hipFree(p); });
    std::unique_ptr<int32_t, void (*)(int32_t*)> o2(tgb, [](int32_t* p) { (void)hipFree(p); });
    std::vector<int32_t> tg_h((size_t)n * kt);
    HIP_TRY(hipMemcpyAsync(tg_h.data(), tg, sizeof(int32_t) * tg_h.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<int32_t> tgb_h((size_t)B * kt);
    for (uint32_t ep = 0; ep < epochs; ++ep) {
      if (!(rp->flags & HNTL_ROUTER_NO_SHUFFLE))  // Fisher-Yates from the counter-based generator
        for (uint32_t i = n - 1; i > 0; --i) {
          const uint32_t j = (uint32_t)(uni(rp->seed, 100 + ep, i) * (double)(i + 1));
          std::swap(order[i], order[std::min(j, i)]);
        }
      HIP_TRY(hipMemcpyAsync(d_order, order.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
      double eloss = 0.0;
      for (uint32_t bi = 0; bi < nb; ++bi) {
        for (uint32_t r = 0; r < B; ++r)
          std::memcpy(&tgb_h[(size_t)r * kt], &tg_h[(size_t)order[bi * B + r] * kt], sizeof(int32_t) * kt);
        HIP_TRY(hipMemcpyAsync(tgb, tgb_h.data(), sizeof(int32_t) * tgb_h.size(), hipMemcpyHostToDevice, s));
        tr.grad(Qtrain, d_order + (size_t)bi * B, tgb, (int)kt);
        tr.adam(rp->lr > 0 ? rp->lr : 1e-3f);
        float l = 0.f;
        HIP_TRY(hipMemcpyAsync(&l, tr.loss, sizeof(float), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));  // also keeps tgb_h from being overwritten early
        eloss += l;
      }
      if (epoch_loss) epoch_loss[ep] = (float)(eloss / nb);
    }
    rt.trained = true;
  });
}

}  // extern "C"
