// Centroid routing (paper Section 2.1 step 1 and Section 2.3): squared
// Euclidean distance from every query to every grain centroid, then the P
// nearest grains per query.  The same distance tile also serves the k-means
// assignment of the build (nearest centroid per row).
//
// Distances use the expansion ||a||^2 + ||b||^2 - 2 a.b with the a.b term on
// MFMA: FP32 (v_mfma_f32_16x16x4_f32) here, BF16 (plain or split operands) in
// router.hip.  The expansion's rounding error is harmless for the k-means
// assignment; routing bounds it per entry and re-scores every shortlist entry
// that the bound leaves in reach of the P-th by direct differences before it
// picks the P probes.
#include <algorithm>

#include "hntl_device.h"
#include "hntl_internal.h"

namespace hntl {

namespace {

constexpr int TM = 64, TN = 64, TK = 32, LDT = TK + 1;

__global__ __launch_bounds__(256) void row_norms_kernel(const float* __restrict__ A, int64_t rows, int d,
                                                        float* __restrict__ out) {
  const int lane = lane_id();
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const float* a = A + row * d;
  float acc = 0.f;
  for (int j = lane; j < d; j += HNTL_WAVE) acc = fmaf(a[j], a[j], acc);
  acc = wave_sum(acc);
  if (lane == 0) out[row] = acc;
}

// One thread's 8 floats of a TM x TK tile of row-major M (rows x d) at
// (r0, k0): row tid / 4, depths 8 (tid % 4) .. + 7 (zero outside M).
__device__ __forceinline__ void fetch_tile(float4 (&v)[2], const float* __restrict__ M, int64_t nrows, int d,
                                           int64_t r0, int k0, bool vec4) {
  const int tid = threadIdx.x;
  const int rr = tid >> 2, cc = (tid & 3) * 8;
  const int64_t gr = r0 + rr;
  if (vec4) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int gk = k0 + cc + 4 * u;
      v[u] = (gr < nrows && gk < d) ? *reinterpret_cast<const float4*>(M + gr * d + gk)
                                    : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  } else {
    float e[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int gk = k0 + cc + u;
      e[u] = (gr < nrows && gk < d) ? M[gr * d + gk] : 0.f;
    }
    v[0] = make_float4(e[0], e[1], e[2], e[3]);
    v[1] = make_float4(e[4], e[5], e[6], e[7]);
  }
}

__device__ __forceinline__ void store_tile(float (*S)[LDT], const float4 (&v)[2]) {
  const int tid = threadIdx.x;
  const int rr = tid >> 2, cc = (tid & 3) * 8;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    S[rr][cc + 4 * u] = v[u].x;
    S[rr][cc + 4 * u + 1] = v[u].y;
    S[rr][cc + 4 * u + 2] = v[u].z;
    S[rr][cc + 4 * u + 3] = v[u].w;
  }
}

// One 64 x 64 tile of A.B^T accumulated over the full depth d; each of the 4
// waves owns a 32 x 32 quarter as 2 x 2 MFMA 16x16 tiles.  The next depth
// tile is fetched into registers while the MFMAs of the current one run.
__device__ __forceinline__ void tile_dot(floatx4 (&acc)[2][2], float (*As)[LDT], float (*Bs)[LDT],
                                         const float* __restrict__ A, int64_t rows, const float* __restrict__ Bm,
                                         int cols, int d, int64_t row0, int col0, bool vec4) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  float4 fa[2], fb[2];
  fetch_tile(fa, A, rows, d, row0, 0, vec4);
  fetch_tile(fb, Bm, cols, d, col0, 0, vec4);
  for (int k0 = 0; k0 < d; k0 += TK) {
    store_tile(As, fa);
    store_tile(Bs, fb);
    __syncthreads();
    if (k0 + TK < d) {
      fetch_tile(fa, A, rows, d, row0, k0 + TK, vec4);
      fetch_tile(fb, Bm, cols, d, col0, k0 + TK, vec4);
    }
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const int kr = kk + (lane >> 4);
      const float a0 = As[wr + (lane & 15)][kr];
      const float a1 = As[wr + 16 + (lane & 15)][kr];
      const float b0 = Bs[wc + (lane & 15)][kr];
      const float b1 = Bs[wc + 16 + (lane & 15)][kr];
      acc[0][0] = mfma16x16x4(a0, b0, acc[0][0]);
      acc[0][1] = mfma16x16x4(a0, b1, acc[0][1]);
      acc[1][0] = mfma16x16x4(a1, b0, acc[1][0]);
      acc[1][1] = mfma16x16x4(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void dist_matrix_kernel(const float* __restrict__ A, const float* __restrict__ an,
                                                          int64_t rows, const float* __restrict__ Bm,
                                                          const float* __restrict__ bn, int cols, int d,
                                                          float* __restrict__ D, bool vec4,
                                                          const int32_t* __restrict__ nlim, int64_t row_base) {
  __shared__ float As[TM][LDT];
  __shared__ float Bs[TN][LDT];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * TM;
  if (nlim) {  // rows from *nlim - row_base on are not part of this batch
    const int64_t lim = (int64_t)*nlim - row_base;
    if (row0 >= lim) return;
    if (lim < rows) rows = lim;
  }
  const int col0 = blockIdx.y * TN;
  floatx4 acc[2][2];
  tile_dot(acc, As, Bs, A, rows, Bm, cols, d, row0, col0, vec4);
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t row = row0 + wr + rt * 16 + 4 * (lane >> 4) + i;
        const int col = col0 + wc + ct * 16 + (lane & 15);
        if (row < rows && col < cols) {
          const float v = an[row] + bn[col] - 2.f * acc[rt][ct][i];
          D[row * cols + col] = fmaxf(v, 0.f);
        }
      }
}

// Small batches (<= 16 rows): exact distances by direct differences, one
// wave per column (centroid) held in registers (d <= 1024), every row of A
// against it.  Reads each centroid once instead of staging mostly empty
// 64-row MFMA tiles.
constexpr int DIRECT_ROWS = 16;
__global__ __launch_bounds__(256) void dist_direct_kernel(const float* __restrict__ A, int64_t rows,
                                                          const float* __restrict__ Bm, int cols, int d,
                                                          float* __restrict__ D, const int32_t* __restrict__ nlim,
                                                          int64_t row_base) {
  const int lane = lane_id();
  const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (col >= cols) return;
  int64_t nr = rows;
  if (nlim) {
    const int64_t lim = (int64_t)*nlim - row_base;
    if (lim < nr) nr = lim;
  }
  const float* b = Bm + (size_t)col * d;
  float bv[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int j = u * HNTL_WAVE + lane;
    bv[u] = j < d ? b[j] : 0.f;
  }
  for (int64_t r = 0; r < nr; ++r) {
    const float* a = A + r * d;
    float acc = 0.f;
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int j = u * HNTL_WAVE + lane;
      if (j < d) {
        const float df = a[j] - bv[u];
        acc = fmaf(df, df, acc);
      }
    }
    acc = wave_sum(acc);
    if (lane == 0) D[r * cols + col] = acc;
  }
}

__global__ __launch_bounds__(256) void argmin_rows_kernel(const float* __restrict__ A, const float* __restrict__ an,
                                                          int64_t rows, const float* __restrict__ Bm,
                                                          const float* __restrict__ bn, int cols, int d,
                                                          int32_t* __restrict__ label, float* __restrict__ dmin,
                                                          bool vec4) {
  __shared__ float As[TM][LDT];
  __shared__ float Bs[TN][LDT];
  __shared__ float red_d[4][32];
  __shared__ int red_i[4][32];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * TM;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  float bd[2][4];
  int bi[2][4];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      bd[rt][i] = __builtin_inff();
      bi[rt][i] = 0x7fffffff;
    }
  for (int col0 = 0; col0 < cols; col0 += TN) {
    floatx4 acc[2][2];
    tile_dot(acc, As, Bs, A, rows, Bm, cols, d, row0, col0, vec4);
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t row = row0 + wr + rt * 16 + 4 * (lane >> 4) + i;
          const int col = col0 + wc + ct * 16 + (lane & 15);
          if (row < rows && col < cols) {
            const float v = fmaxf(an[row] + bn[col] - 2.f * acc[rt][ct][i], 0.f);
            if (v < bd[rt][i] || (v == bd[rt][i] && col < bi[rt][i])) {
              bd[rt][i] = v;
              bi[rt][i] = col;
            }
          }
        }
  }
  // reduce over the 16 lanes that share a row, then over the two waves that
  // share the same rows
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float v = bd[rt][i];
      int c = bi[rt][i];
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        const float ov = __shfl_xor(v, o, 64);
        const int oc = __shfl_xor(c, o, 64);
        if (ov < v || (ov == v && oc < c)) {
          v = ov;
          c = oc;
        }
      }
      if ((lane & 15) == 0) {
        red_d[wave][rt * 16 + 4 * (lane >> 4) + i] = v;
        red_i[wave][rt * 16 + 4 * (lane >> 4) + i] = c;
      }
    }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int r = threadIdx.x;
    const int w0 = 2 * (r >> 5);
    float v = red_d[w0][r & 31];
    int c = red_i[w0][r & 31];
    const float v1 = red_d[w0 + 1][r & 31];
    const int c1 = red_i[w0 + 1][r & 31];
    if (v1 < v || (v1 == v && c1 < c)) {
      v = v1;
      c = c1;
    }
    const int64_t row = row0 + r;
    if (row < rows) {
      label[row] = c;
      if (dmin) dmin[row] = v;
    }
  }
}

// Top-P per row of D.  Without A/Bm: the P smallest entries of D.  With them
// (routing), D holds expansion distances ||a||^2 + ||b||^2 - 2 <a, b> whose
// error against the exact distance is at most err (||a||^2 + ||b||^2) per
// entry (the caller's bound for its product form).  A shortlist of the M
// smallest expansion values is kept; every entry j whose interval
// [D_j - bound_j, D_j + bound_j] reaches the P-th entry's upper end can still
// be among the P nearest, so exactly those are re-scored by direct
// differences ||a - b||^2 in FP32 and the P smallest exact distances are kept
// (ties: lower column).  Probe order and reported distances then carry
// direct-difference accuracy.  If the window reaches the end of the
// shortlist (entry M - 1 qualifies while columns remain beyond it), entries
// past M may qualify as well: the row is then re-read whole, and every column
// inside the window is re-scored.
//
// Rows per workgroup, one per wave.
constexpr int TOPK_ROWS = 8;

// Direct FP32 squared distance of row a and column row b (both d long), one
// wave, every lane ends with the total.
// With vec4 (d % 4 == 0, 16-byte aligned rows) lane l covers depths
// 4 l .. 4 l + 3 of every 256-wide chunk, in that order; otherwise depths l,
// l + 64, ...
__device__ __forceinline__ float wave_dist(const float* __restrict__ a, const float* __restrict__ b, int d,
                                           bool vec4) {
  float acc = 0.f;
  if (vec4) {
    for (int t = lane_id() * 4; t < d; t += 4 * HNTL_WAVE) {
      const float4 x = *reinterpret_cast<const float4*>(a + t), y = *reinterpret_cast<const float4*>(b + t);
      float df = x.x - y.x;
      acc = fmaf(df, df, acc);
      df = x.y - y.y;
      acc = fmaf(df, df, acc);
      df = x.z - y.z;
      acc = fmaf(df, df, acc);
      df = x.w - y.w;
      acc = fmaf(df, df, acc);
    }
  } else {
    for (int t = lane_id(); t < d; t += HNTL_WAVE) {
      const float df = a[t] - b[t];
      acc = fmaf(df, df, acc);
    }
  }
  return wave_sum(acc);
}

__global__ __launch_bounds__(TOPK_ROWS * 64) void topk_rows_kernel(
    const float* __restrict__ D, int64_t rows, int cols, int P, int M, const float* __restrict__ A,
    const float* __restrict__ an, const float* __restrict__ Bm, const float* __restrict__ bn, int d, float err,
    int32_t* __restrict__ idx, float* __restrict__ val, const int32_t* __restrict__ nlim, int64_t row_base,
    unsigned int* __restrict__ overflow, float2* __restrict__ znorm, bool vec4) {
  __shared__ uint64_t stage[TOPK_ROWS][64];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t row = (int64_t)blockIdx.x * TOPK_ROWS + wave;
  if (row >= rows) return;
  if (nlim && row >= (int64_t)*nlim - row_base) {  // not part of this batch: no probes
    if (lane < P) {
      idx[row * P + lane] = -1;
      if (val) val[row * P + lane] = __builtin_inff();
    }
    return;
  }
  const bool exact = A != nullptr;
  WaveTop64 L;
  L.init(stage[wave], exact ? M : P);
  const float* drow = D + row * cols;
  // Segments of U chunks of 64 columns, loaded together.  The 64 lanes'
  // minima over a segment are 64 entries of the row, so their maximum bounds
  // the row's 64th smallest value (>= its M-th and P-th) from above: entries
  // above the smallest such bound so far cannot be selected and are not
  // offered (fewer list flushes; the selection is unchanged).  Segments of
  // 16 chunks measured best (0.573 against 0.588 ms of routing without the
  // bound at 16,384 x 8,192; longer segments cost more in occupancy).
  constexpr int U = 16;
  float T = __builtin_inff();  // uniform
  // znorm (negated scores): the row's smallest value mn and z = sum exp(mn - D_c),
  // the softmax normaliser of the scores, accumulated per lane against the
  // lane's running minimum and rescaled when it drops
  float lmn = __builtin_inff(), lz = 0.f;
  for (int c0 = 0; c0 < cols; c0 += U * HNTL_WAVE) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + u * HNTL_WAVE + lane;
      v[u] = c < cols ? drow[c] : __builtin_inff();
    }
    float seg = v[0];
#pragma unroll
    for (int u = 1; u < U; ++u) seg = fminf(seg, v[u]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) seg = fmaxf(seg, __shfl_xor(seg, o, 64));
    T = fminf(T, seg);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + u * HNTL_WAVE + lane;
      L.offer_f(v[u], (uint32_t)c, c < cols && v[u] <= T);
    }
    if (znorm) {
      float cm = __builtin_inff();
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (c0 + u * HNTL_WAVE + lane < cols) cm = fminf(cm, v[u]);
      if (cm < __builtin_inff()) {
        const float nm = fminf(lmn, cm);
        lz = lmn < __builtin_inff() ? lz * expf(nm - lmn) : 0.f;
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (c0 + u * HNTL_WAVE + lane < cols) lz += expf(nm - v[u]);
        lmn = nm;
      }
    }
  }
  L.finish();
  if (znorm) {
    float mn = lmn;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mn = fminf(mn, __shfl_xor(mn, o, 64));
    const float z = wave_sum(lmn < __builtin_inff() ? lz * expf(mn - lmn) : 0.f);
    if (lane == 0) znorm[row] = make_float2(mn, z);
  }
  if (!exact) {
    if (lane < P) {
      idx[row * P + lane] = L.best == KEY_NONE ? -1 : (int32_t)key_id(L.best);
      if (val) val[row * P + lane] = L.best == KEY_NONE ? __builtin_inff() : key_dist(L.best);
    }
    return;
  }
  // entries j >= P qualify while D_j - bound_j <= D_{P-1} + bound_{P-1}
  const float arow = an[row];
  const uint64_t mine = L.best;
  const uint64_t kp = shfl_u64(mine, P - 1);
  const float hiP = key_dist(kp) + err * (arow + bn[key_id(kp)]);
  const bool in = lane >= P && lane < M && mine != KEY_NONE &&
                  key_dist(mine) - err * (arow + bn[key_id(mine)]) <= hiP;
  const uint64_t qual = __ballot(in);
  const int Mr = qual ? 64 - __clzll(qual) : P;  // re-score the prefix [0, Mr)
  const float* a = A + row * d;
  uint64_t ex = KEY_NONE;
  if (Mr == M && M < cols) {
    // the window may extend past the shortlist: every column of the row whose
    // interval reaches hiP is re-scored, into a fresh top-P list
    if (overflow && lane == 0) atomicAdd(overflow, 1u);
    WaveTop64 X;
    wave_sync();
    X.init(stage[wave], P);
    for (int c0 = 0; c0 < cols; c0 += HNTL_WAVE) {
      const int c = c0 + lane;
      const bool w = c < cols && drow[c] - err * (arow + bn[c]) <= hiP;
      uint64_t m = __ballot(w);
      uint64_t keyc = KEY_NONE;
      while (m) {  // wave-uniform loop over the window columns of this chunk
        const int j = __builtin_ctzll(m);
        m &= m - 1;
        const float dd = wave_dist(a, Bm + (size_t)(c0 + j) * d, d, vec4);
        if (lane == j) keyc = make_key(dd, (uint32_t)(c0 + j));
      }
      X.offer(keyc, w);
    }
    X.finish();
    ex = X.best;
  } else {
    constexpr int RB = 8;  // shortlist entries re-scored together
    for (int j0 = 0; j0 < Mr; j0 += RB) {
      int cs[RB];
      const float* bp[RB];
      float acc[RB];
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int j = j0 + u < Mr ? j0 + u : j0;
        cs[u] = (int)key_id(shfl_u64(mine, j));
        bp[u] = Bm + (size_t)cs[u] * d;
        acc[u] = 0.f;
      }
      if (vec4) {
        // 16-byte loads: a round of RB entries covers 256 depths per load
        // instruction (3 rounds for d = 768 instead of 12 with 4-byte loads)
        constexpr int CH = 1;
        for (int t0 = lane * 4; t0 < d; t0 += CH * 4 * HNTL_WAVE) {
          float4 av[CH], bv[CH][RB];
#pragma unroll
          for (int i = 0; i < CH; ++i) {
            const int t = t0 + i * 4 * HNTL_WAVE;
            av[i] = t < d ? *reinterpret_cast<const float4*>(a + t) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int u = 0; u < RB; ++u)
              bv[i][u] = t < d ? *reinterpret_cast<const float4*>(bp[u] + t) : make_float4(0.f, 0.f, 0.f, 0.f);
          }
#pragma unroll
          for (int i = 0; i < CH; ++i) {
            if (t0 + i * 4 * HNTL_WAVE >= d) break;  // uniform
#pragma unroll
            for (int u = 0; u < RB; ++u) {
              float df = av[i].x - bv[i][u].x;
              acc[u] = fmaf(df, df, acc[u]);
              df = av[i].y - bv[i][u].y;
              acc[u] = fmaf(df, df, acc[u]);
              df = av[i].z - bv[i][u].z;
              acc[u] = fmaf(df, df, acc[u]);
              df = av[i].w - bv[i][u].w;
              acc[u] = fmaf(df, df, acc[u]);
            }
          }
        }
      } else {
        for (int t = lane; t < d; t += HNTL_WAVE) {
          const float av = a[t];
#pragma unroll
          for (int u = 0; u < RB; ++u) {
            const float df = av - bp[u][t];
            acc[u] = fmaf(df, df, acc[u]);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const float tot = wave_sum(acc[u]);
        if (lane == j0 + u && lane < Mr) ex = make_key(tot, (uint32_t)cs[u]);
      }
    }
    ex = wave_sort64(ex);
  }
  if (lane < P) {
    idx[row * P + lane] = (int32_t)key_id(ex);
    if (val) val[row * P + lane] = key_dist(ex);
  }
}

// ------------------------------------------------------- brute-force kNN
// Exact k nearest rows of B for every row of A (the learned router's training
// targets).  Pass 1, grid (row tiles of 64, column splits): a workgroup walks
// its column range in 64-wide tiles of MFMA expansion distances, stages each
// 64 x 64 tile in LDS, and every wave keeps, for its 16 rows, the KNN_SHORT
// smallest (distance, column) keys in register lists.  Pass 2 merges the
// splits' lists per row, re-scores the merged shortlist by direct
// differences in FP32 and keeps the k smallest exact distances (ties: lower
// column).
constexpr int KNN_SHORT = 32;

__global__ __launch_bounds__(256) void knn_partial_kernel(const float* __restrict__ A, const float* __restrict__ an,
                                                          int64_t rows, const float* __restrict__ Bm,
                                                          const float* __restrict__ bn, int64_t cols, int d,
                                                          int64_t per_split, uint64_t* __restrict__ part,
                                                          bool vec4) {
  __shared__ float tiles[2 * TM * LDT];  // As and Bs; then the 64 x 64 distance tile
  __shared__ uint64_t stage[4][16][64];
  float(*As)[LDT] = reinterpret_cast<float(*)[LDT]>(tiles);
  float(*Bs)[LDT] = reinterpret_cast<float(*)[LDT]>(tiles + TM * LDT);
  float(*Dt)[TN + 1] = reinterpret_cast<float(*)[TN + 1]>(tiles);
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * TM;
  const int64_t c_begin = (int64_t)blockIdx.y * per_split;
  const int64_t c_end = c_begin + per_split < cols ? c_begin + per_split : cols;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  WaveTop64 L[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) L[r].init(stage[wave][r], KNN_SHORT);
  for (int64_t col0 = c_begin; col0 < c_end; col0 += TN) {
    floatx4 acc[2][2];
    tile_dot(acc, As, Bs, A, rows, Bm, (int)(c_end < cols ? c_end : cols), d, row0, (int)col0, vec4);
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int rl = wr + rt * 16 + 4 * (lane >> 4) + i;
          const int cl = wc + ct * 16 + (lane & 15);
          const int64_t row = row0 + rl, col = col0 + cl;
          Dt[rl][cl] = (row < rows && col < c_end) ? fmaxf(an[row] + bn[col] - 2.f * acc[rt][ct][i], 0.f)
                                                   : __builtin_inff();
        }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float v = Dt[16 * wave + r][lane];
      const int64_t col = col0 + lane;
      L[r].offer(make_key(v, (uint32_t)col), col < c_end);
    }
    __syncthreads();  // the next tile_dot overwrites the distance tile
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    L[r].finish();
    const int64_t row = row0 + 16 * wave + r;
    if (row < rows && lane < KNN_SHORT) part[((size_t)row * gridDim.y + blockIdx.y) * KNN_SHORT + lane] = L[r].best;
  }
}

// One wave per row: merge the splits' shortlists, exact re-score, top k.
__global__ __launch_bounds__(256) void knn_merge_kernel(const float* __restrict__ A, int64_t rows,
                                                        const float* __restrict__ Bm, int d, int splits,
                                                        const uint64_t* __restrict__ part, int k,
                                                        int32_t* __restrict__ ids, float* __restrict__ dist) {
  __shared__ uint64_t stage[4][64];
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  const int64_t row = (int64_t)blockIdx.x * 4 + wave;
  if (row >= rows) return;
  WaveTop64 L;
  L.init(stage[wave], KNN_SHORT);
  for (int sp = 0; sp < splits; ++sp) {
    const uint64_t key = lane < KNN_SHORT ? part[((size_t)row * splits + sp) * KNN_SHORT + lane] : KEY_NONE;
    L.offer(key, key != KEY_NONE);
  }
  L.finish();
  const uint64_t mine = L.best;
  const float* a = A + row * d;
  uint64_t ex = KEY_NONE;
  for (int j = 0; j < KNN_SHORT; ++j) {
    const uint64_t kj = shfl_u64(mine, j);
    if (kj == KEY_NONE) break;
    const uint32_t c = key_id(kj);
    const float* b = Bm + (size_t)c * d;
    float acc = 0.f;
    for (int t = lane; t < d; t += HNTL_WAVE) {
      const float df = a[t] - b[t];
      acc = fmaf(df, df, acc);
    }
    acc = wave_sum(acc);
    if (lane == j) ex = make_key(acc, c);
  }
  ex = wave_sort64(ex);
  if (lane < k) {
    ids[row * k + lane] = ex == KEY_NONE ? -1 : (int32_t)key_id(ex);
    if (dist) dist[row * k + lane] = ex == KEY_NONE ? __builtin_inff() : key_dist(ex);
  }
}

}  // namespace

void launch_row_norms(const float* A, int64_t rows, int d, float* out, hipStream_t s) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(row_norms_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, A, rows, d, out);
  HIP_TRY(hipGetLastError());
}

void launch_dist_matrix(const float* A, const float* an, int64_t rows, const float* Bm, const float* bn, int cols,
                        int d, float* D, hipStream_t s, const int32_t* nlim, int64_t row_base) {
  if (rows <= 0 || cols <= 0) return;
  if (rows <= DIRECT_ROWS && d <= 16 * HNTL_WAVE) {
    hipLaunchKernelGGL(dist_direct_kernel, dim3((unsigned)((cols + 3) / 4)), dim3(256), 0, s, A, rows, Bm, cols, d, D,
                       nlim, row_base);
    HIP_TRY(hipGetLastError());
    return;
  }
  const bool vec4 = (d % 4) == 0 && ((uintptr_t)A % 16) == 0 && ((uintptr_t)Bm % 16) == 0;
  dim3 grid((unsigned)((rows + TM - 1) / TM), (unsigned)((cols + TN - 1) / TN));
  hipLaunchKernelGGL(dist_matrix_kernel, grid, dim3(256), 0, s, A, an, rows, Bm, bn, cols, d, D, vec4, nlim,
                     row_base);
  HIP_TRY(hipGetLastError());
}

void launch_argmin_rows(const float* A, const float* an, int64_t rows, const float* Bm, const float* bn, int cols,
                        int d, int32_t* label, float* dmin, hipStream_t s) {
  if (rows <= 0) return;
  const bool vec4 = (d % 4) == 0 && ((uintptr_t)A % 16) == 0 && ((uintptr_t)Bm % 16) == 0;
  hipLaunchKernelGGL(argmin_rows_kernel, dim3((unsigned)((rows + TM - 1) / TM)), dim3(256), 0, s, A, an, rows, Bm,
                     bn, cols, d, label, dmin, vec4);
  HIP_TRY(hipGetLastError());
}

void launch_topk_rows(const float* D, int64_t rows, int cols, int P, int32_t* idx, float* val, hipStream_t s,
                      const float* A, const float* an, const float* Bm, const float* bn, int d, float err,
                      const int32_t* nlim, int64_t row_base, unsigned int* overflow, float2* znorm) {
  if (A && (!an || !bn || !Bm)) throw ArgError{HNTL_EINVAL, "routing re-score needs both norm vectors and the centroids"};
  if (A && znorm) throw ArgError{HNTL_EINVAL, "the softmax normaliser is for score rows (no re-score)"};
  if (rows <= 0) return;
  if (P > HNTL_MAX_P) throw ArgError{HNTL_EUNSUPPORTED, "routing supports P <= 48"};
  // shortlist: the window of the P-th entry plus 48 more (one key per lane)
  const int M = A ? std::min(cols, std::min(64, P + 48)) : P;
  // float4 re-score loads where rows allow them
  const bool vec4 = A && (d % 4) == 0 && ((uintptr_t)A % 16) == 0 && ((uintptr_t)Bm % 16) == 0;
  dim3 grid((unsigned)((rows + TOPK_ROWS - 1) / TOPK_ROWS)), block(TOPK_ROWS * 64);
  hipLaunchKernelGGL(topk_rows_kernel, grid, block, 0, s, D, rows, cols, P, M, A, an, Bm, bn, d, err, idx, val, nlim,
                     row_base, overflow, znorm, vec4);
  HIP_TRY(hipGetLastError());
}

int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

}  // namespace hntl

namespace hntl {

void launch_knn(const float* A, int64_t rows, const float* Bm, int64_t cols, int d, int k, int32_t* ids, float* dist,
                hipStream_t s) {
  if (rows <= 0) return;
  if (k < 1 || k > 16) throw ArgError{HNTL_EUNSUPPORTED, "brute-force kNN supports 1 <= k <= 16"};
  if (cols >= (1ll << 31)) throw ArgError{HNTL_EUNSUPPORTED, "brute-force kNN needs fewer than 2^31 rows"};
  const bool vec4 = (d % 4) == 0 && ((uintptr_t)A % 16) == 0 && ((uintptr_t)Bm % 16) == 0;
  const int64_t rt = (rows + TM - 1) / TM;
  int64_t splits = std::max<int64_t>(1, std::min<int64_t>((cols + TN - 1) / TN, 2048 / rt));
  int64_t per = ((cols + splits - 1) / splits + TN - 1) / TN * TN;
  splits = (cols + per - 1) / per;
  float *an = nullptr, *bn = nullptr;
  uint64_t* part = nullptr;
  HIP_TRY(hipMallocAsync((void**)&an, sizeof(float) * rows, s));
  HIP_TRY(hipMallocAsync((void**)&bn, sizeof(float) * cols, s));
  HIP_TRY(hipMallocAsync((void**)&part, sizeof(uint64_t) * rows * splits * KNN_SHORT, s));
  launch_row_norms(A, rows, d, an, s);
  launch_row_norms(Bm, cols, d, bn, s);
  hipLaunchKernelGGL(knn_partial_kernel, dim3((unsigned)rt, (unsigned)splits), dim3(256), 0, s, A, an, rows, Bm, bn,
                     cols, d, per, part, vec4);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(knn_merge_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, A, rows, Bm, d,
                     (int)splits, part, k, ids, dist);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipFreeAsync(an, s));
  HIP_TRY(hipFreeAsync(bn, s));
  HIP_TRY(hipFreeAsync(part, s));
}

}  // namespace hntl
