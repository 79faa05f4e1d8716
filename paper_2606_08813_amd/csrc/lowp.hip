// Reduced-precision tangent codes (the precision form): BF16 codes, and FP8
// E4M3 codes with one FP32 scale per grain, derived from the FP32 Block-SoA
// codes; plus a BF16 copy of the bases for the BF16 projection.
//
// Packed Block-SoA layouts (one 32-bit word per lane and row, so that a row
// of a block is still one coalesced 256-byte load):
//   BF16: word[blk][j2][lane] holds dims 2 j2 (low half) and 2 j2 + 1 (high half)
//   FP8:  word[blk][j4][lane] holds dims 4 j4 + i in byte i
//
// BF16: round-to-nearest-even of the FP32 bit pattern (drop 16 mantissa bits).
// FP8 E4M3 "fn" (OCP 8-bit float specification): bias 7, 3 mantissa bits,
// largest finite 448, no infinities.  Code = e4m3(z / s_g) rounded to nearest
// even with saturation to +-448, s_g = amax_{i in g, j < r} |z_ij| / 448
// (1 for an all-zero grain).  INT16 (the paper's own reduced form, eq. 5):
// two int16 codes per word as BF16, per-grain steps, decoded member residuals.
#include "hntl_device.h"
#include "hntl_internal.h"

namespace hntl {

__host__ __device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}

__host__ __device__ inline uint8_t f32_to_e4m3_rne_sat(float x) {
  const uint8_t sign = x < 0.f ? 0x80 : 0x00;
  float a = fabsf(x);
  if (!(a < 448.f)) return sign | 0x7E;  // saturate (also NaN -> max, inputs are finite)
  if (a < 0.015625f) {                   // below 2^-6: subnormal, quantum 2^-9
    const int m = (int)rintf(a * 512.f); // 0..8; 8 encodes 2^-6 (the first normal)
    return sign | (uint8_t)m;
  }
  int e;
  const float mant = frexpf(a, &e);  // a = mant * 2^e, mant in [0.5, 1)
  const int E = e - 1;               // a = (2 mant) * 2^E, 2 mant in [1, 2)
  int m = (int)rintf((2.f * mant - 1.f) * 8.f);
  int Eb = E + 7;
  if (m == 8) {
    m = 0;
    ++Eb;
  }
  int code = (Eb << 3) | m;
  if (code > 0x7E) code = 0x7E;
  return sign | (uint8_t)code;
}

namespace {

__global__ void bf16_kernel(const float* __restrict__ in, int64_t n, uint16_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = f32_to_bf16_rne(in[i]);
}

// codes [blk][rp][64] f32 -> words [blk][rp / 2][64]
__global__ void bf16_pack_kernel(const float* __restrict__ codes, int rp, int64_t nblocks,
                                 uint32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // word index
  const int64_t per = (int64_t)(rp / 2) * B;
  if (i >= nblocks * per) return;
  const int64_t blk = i / per, rem = i % per, j2 = rem / B, lane = rem % B;
  const float* c = codes + (size_t)blk * rp * B;
  const uint32_t lo = f32_to_bf16_rne(c[(2 * j2) * B + lane]);
  const uint32_t hi = f32_to_bf16_rne(c[(2 * j2 + 1) * B + lane]);
  out[i] = lo | (hi << 16);
}

// one workgroup per grain: amax over valid members and j < r
__global__ __launch_bounds__(256) void grain_scale_kernel(const float* __restrict__ codes, int rp, int r,
                                                          const int32_t* __restrict__ goff,
                                                          const int32_t* __restrict__ boff,
                                                          float* __restrict__ scales) {
  __shared__ float red[256];
  const int g = blockIdx.x;
  const int b0 = boff[g], nb = boff[g + 1] - b0, ng = goff[g + 1] - goff[g];
  float m = 0.f;
  for (int64_t e = threadIdx.x; e < (int64_t)nb * rp * B; e += 256) {
    const int blk = (int)(e / (rp * B)), rem = (int)(e % (rp * B)), j = rem / B, lane = rem % B;
    if (j < r && blk * B + lane < ng) m = fmaxf(m, fabsf(codes[(size_t)(b0 + blk) * rp * B + rem]));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) scales[g] = red[0] > 0.f ? red[0] / 448.f : 1.f;
}

// codes [blk][rp][64] f32 -> words [blk][rp / 4][64] of e4m3(z / s_g)
__global__ void fp8_pack_kernel(const float* __restrict__ codes, int rp, const int32_t* __restrict__ block_grain,
                                const float* __restrict__ scales, int64_t nblocks, uint32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)(rp / 4) * B;
  if (i >= nblocks * per) return;
  const int64_t blk = i / per, rem = i % per, j4 = rem / B, lane = rem % B;
  const float s = scales[block_grain[blk]];
  const float* c = codes + (size_t)blk * rp * B;
  uint32_t w = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) w |= (uint32_t)f32_to_e4m3_rne_sat(c[(4 * j4 + t) * B + lane] / s) << (8 * t);
  out[i] = w;
}

// int16 form (eq. 5), one workgroup per grain: inv_g = fl32(32767 / amax_g)
// over |z_ij| (j < r), rinv_g = fl32(65535 / max_i eps_i) (1 when the maximum
// is 0), computed as float64 divisions rounded once; also (1 / inv_g)^2 and
// 1 / rinv_g for the score.
__global__ __launch_bounds__(256) void int16_steps_kernel(const float* __restrict__ codes, const float* __restrict__ eps,
                                                          int rp, int r, const int32_t* __restrict__ goff,
                                                          const int32_t* __restrict__ boff, float* __restrict__ steps) {
  __shared__ float red[2][256];
  const int g = blockIdx.x;
  const int b0 = boff[g], nb = boff[g + 1] - b0, ng = goff[g + 1] - goff[g];
  float m = 0.f, em = 0.f;
  for (int64_t e = threadIdx.x; e < (int64_t)nb * rp * B; e += 256) {
    const int blk = (int)(e / (rp * B)), rem = (int)(e % (rp * B)), j = rem / B, lane = rem % B;
    if (j < r && blk * B + lane < ng) m = fmaxf(m, fabsf(codes[(size_t)(b0 + blk) * rp * B + rem]));
  }
  for (int i = threadIdx.x; i < ng; i += 256) em = fmaxf(em, eps[((size_t)b0 + i / B) * B + i % B]);
  red[0][threadIdx.x] = m;
  red[1][threadIdx.x] = em;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      red[0][threadIdx.x] = fmaxf(red[0][threadIdx.x], red[0][threadIdx.x + o]);
      red[1][threadIdx.x] = fmaxf(red[1][threadIdx.x], red[1][threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float inv = red[0][0] > 0.f ? (float)(32767.0 / (double)red[0][0]) : 1.f;
    const float rinv = red[1][0] > 0.f ? (float)(65535.0 / (double)red[1][0]) : 1.f;
    const double st = 1.0 / (double)inv;
    steps[(size_t)g * 4] = inv;
    steps[(size_t)g * 4 + 1] = rinv;
    steps[(size_t)g * 4 + 2] = (float)(st * st);
    steps[(size_t)g * 4 + 3] = (float)(1.0 / (double)rinv);
  }
}

__device__ __forceinline__ int q16(float x, float inv, int lo, int hi) {
  const float q = rintf(x * inv);  // float32 product, ties to even
  return (int)fminf(fmaxf(q, (float)lo), (float)hi);
}

// codes [blk][rp][64] f32 -> words [blk][rp / 2][64] of two int16; residuals
// decoded as r_hat / rinv (0 past the grain's members)
__global__ void int16_pack_kernel(const float* __restrict__ codes, const float* __restrict__ eps, int rp,
                                  const int32_t* __restrict__ block_grain, const int32_t* __restrict__ goff,
                                  const int32_t* __restrict__ boff, const float* __restrict__ steps, int64_t nblocks,
                                  uint32_t* __restrict__ out, float* __restrict__ eps_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)(rp / 2) * B;
  if (i >= nblocks * per) return;
  const int64_t blk = i / per, rem = i % per, j2 = rem / B, lane = rem % B;
  const int g = block_grain[blk];
  const float inv = steps[(size_t)g * 4];
  const float* c = codes + (size_t)blk * rp * B;
  const uint32_t lo = (uint16_t)(int16_t)q16(c[(2 * j2) * B + lane], inv, -32767, 32767);
  const uint32_t hi = (uint16_t)(int16_t)q16(c[(2 * j2 + 1) * B + lane], inv, -32767, 32767);
  out[i] = lo | (hi << 16);
  if (j2 == 0) {
    const bool valid = (blk - boff[g]) * B + lane < goff[g + 1] - goff[g];
    const float rh = (float)q16(eps[blk * B + lane], steps[(size_t)g * 4 + 1], 0, 65535);
    eps_out[blk * B + lane] = valid ? rh * steps[(size_t)g * 4 + 3] : 0.f;
  }
}

}  // namespace

void launch_derive_lowp(Index& ix, hipStream_t s) {
  const int64_t nw2 = (int64_t)ix.nblocks * (ix.rp / 2) * B;
  const int64_t nw4 = (int64_t)ix.nblocks * (ix.rp / 4) * B;
  if (ix.codes_mask & (1u << HNTL_CODES_BF16)) {
    if (!ix.codes_bf16) ix.codes_bf16 = dev_alloc<uint32_t>(&ix, nw2);
    hipLaunchKernelGGL(bf16_pack_kernel, dim3((unsigned)((nw2 + 255) / 256)), dim3(256), 0, s, ix.codes, (int)ix.rp,
                       (int64_t)ix.nblocks, ix.codes_bf16);
    HIP_TRY(hipGetLastError());
  }
  const bool fp8 = (ix.codes_mask & (1u << HNTL_CODES_FP8_E4M3)) != 0;
  const bool i16 = (ix.codes_mask & (1u << HNTL_CODES_INT16)) != 0;
  if (fp8 || i16) {
    std::vector<int32_t> bg(ix.nblocks);
    for (uint32_t g = 0; g < ix.G; ++g)
      for (int q = ix.boff_h[g]; q < ix.boff_h[g + 1]; ++q) bg[q] = (int32_t)g;
    int32_t* d_bg = nullptr;
    HIP_TRY(hipMalloc((void**)&d_bg, sizeof(int32_t) * std::max<size_t>(1, bg.size())));
    HIP_TRY(hipMemcpy(d_bg, bg.data(), sizeof(int32_t) * bg.size(), hipMemcpyHostToDevice));
    if (fp8) {
      if (!ix.scales) ix.scales = dev_alloc<float>(&ix, ix.G);
      if (!ix.codes_fp8) ix.codes_fp8 = dev_alloc<uint32_t>(&ix, nw4);
      hipLaunchKernelGGL(grain_scale_kernel, dim3(ix.G), dim3(256), 0, s, ix.codes, (int)ix.rp, (int)ix.r, ix.goff,
                         ix.boff, ix.scales);
      hipLaunchKernelGGL(fp8_pack_kernel, dim3((unsigned)((nw4 + 255) / 256)), dim3(256), 0, s, ix.codes, (int)ix.rp,
                         d_bg, ix.scales, (int64_t)ix.nblocks, ix.codes_fp8);
      HIP_TRY(hipGetLastError());
    }
    if (i16) {
      if (!ix.i16_steps) ix.i16_steps = dev_alloc<float>(&ix, (size_t)ix.G * 4);
      if (!ix.codes_i16) ix.codes_i16 = dev_alloc<uint32_t>(&ix, nw2);
      if (!ix.eps_i16) ix.eps_i16 = dev_alloc<float>(&ix, (size_t)ix.nblocks * B);
      hipLaunchKernelGGL(int16_steps_kernel, dim3(ix.G), dim3(256), 0, s, ix.codes, ix.eps, (int)ix.rp, (int)ix.r,
                         ix.goff, ix.boff, ix.i16_steps);
      hipLaunchKernelGGL(int16_pack_kernel, dim3((unsigned)((nw2 + 255) / 256)), dim3(256), 0, s, ix.codes, ix.eps,
                         (int)ix.rp, d_bg, ix.goff, ix.boff, ix.i16_steps, (int64_t)ix.nblocks, ix.codes_i16,
                         ix.eps_i16);
      HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipFree(d_bg));
  }
  if (!ix.basis_bf16) {
    const int64_t nb = (int64_t)ix.G * ix.r * ix.d;
    ix.basis_bf16 = dev_alloc<uint16_t>(&ix, nb);
    hipLaunchKernelGGL(bf16_kernel, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, ix.basis, nb, ix.basis_bf16);
    HIP_TRY(hipGetLastError());
  }
}

}  // namespace hntl
