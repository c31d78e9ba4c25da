// Operand conversion for the scoring paths: float32 rows -> bfloat16, float32
// rows -> bfloat16 (hi, lo) pairs, and float32 rows -> OCP FP8 E4M3 codes with
// one power-of-two scale per row (and the MX formats).
#include "device_common.hpp"
#include "gem_internal.h"

namespace gem {

// 8 elements per thread and step: two 16-byte loads, one 16-byte store.
__global__ __launch_bounds__(256) void convert_bf16_kernel(const float* __restrict__ x, int64_t n,
                                                           uint16_t* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * 256 * 8;
  for (int64_t i8 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 8; i8 < n; i8 += stride) {
    if (i8 + 8 <= n) {
      float4 a = *reinterpret_cast<const float4*>(x + i8);
      float4 b = *reinterpret_cast<const float4*>(x + i8 + 4);
      uint4 r;
      r.x = f32_to_bf16_rne(a.x) | ((uint32_t)f32_to_bf16_rne(a.y) << 16);
      r.y = f32_to_bf16_rne(a.z) | ((uint32_t)f32_to_bf16_rne(a.w) << 16);
      r.z = f32_to_bf16_rne(b.x) | ((uint32_t)f32_to_bf16_rne(b.y) << 16);
      r.w = f32_to_bf16_rne(b.z) | ((uint32_t)f32_to_bf16_rne(b.w) << 16);
      *reinterpret_cast<uint4*>(out + i8) = r;
    } else {
      for (int64_t i = i8; i < n; ++i) out[i] = f32_to_bf16_rne(x[i]);
    }
  }
}

hipError_t launch_convert_bf16(const float* x, int64_t n_elems, uint16_t* out, hipStream_t s) {
  if (n_elems == 0) return hipSuccess;
  const int64_t threads = (n_elems + 7) / 8;
  const int64_t grid = (threads + 255) / 256;
  hipLaunchKernelGGL(convert_bf16_kernel, dim3(capped_blocks(grid, 256)), dim3(256), 0, s, x, n_elems, out);
  return hipGetLastError();
}

// float32 rows -> bfloat16 (hi, lo) pairs: hi = bf16(x), lo = bf16(x - hi),
// both round to nearest even (x - hi is exact in float32). Row layout: four
// 128-byte blocks, block j = hi of elements 32j .. 32j + 31, then their lo.
// One thread per 8 consecutive elements of a row (a 16-byte store of hi and
// one of lo).
__global__ __launch_bounds__(256) void split_bf16x3_kernel(const float* __restrict__ x, int64_t n_rows,
                                                           uint16_t* __restrict__ out) {
  const int64_t n8 = n_rows * (kDim / 8);
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n8; i += (int64_t)gridDim.x * 256) {
    const int64_t row = i / (kDim / 8);
    const int e0 = (int)(i % (kDim / 8)) * 8;                 // first element of the eight
    const float4 a = *reinterpret_cast<const float4*>(x + row * kDim + e0);
    const float4 b = *reinterpret_cast<const float4*>(x + row * kDim + e0 + 4);
    const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    uint32_t h[4], lo[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint32_t hh[2], ll[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const float xv = v[2 * j + t];
        const uint16_t hb = f32_to_bf16_rne(xv);
        hh[t] = hb;
        ll[t] = f32_to_bf16_rne(xv - __uint_as_float((uint32_t)hb << 16));
      }
      h[j] = hh[0] | (hh[1] << 16);
      lo[j] = ll[0] | (ll[1] << 16);
    }
    // block of element e0: e0 / 32; hi at block * 64 + (e0 % 32), lo 32 elements later
    uint16_t* o = out + row * (2 * kDim) + (e0 / 32) * 64 + (e0 % 32);
    *reinterpret_cast<uint4*>(o) = make_uint4(h[0], h[1], h[2], h[3]);
    *reinterpret_cast<uint4*>(o + 32) = make_uint4(lo[0], lo[1], lo[2], lo[3]);
  }
}

hipError_t launch_split_bf16x3(const float* x, int64_t n_rows, uint16_t* out, hipStream_t s) {
  if (n_rows == 0) return hipSuccess;
  const int64_t grid = (n_rows * (kDim / 8) + 255) / 256;
  hipLaunchKernelGGL(split_bf16x3_kernel, dim3(capped_blocks(grid, 256)), dim3(256), 0, s, x, n_rows, out);
  return hipGetLastError();
}

// One wave per 128-wide row, two elements per lane: max |x| over the wave,
// the row's power-of-two scale, then each element's E4M3 code of x / scale.
__global__ __launch_bounds__(256) void quantize_fp8_kernel(const float* __restrict__ x, int64_t n_rows,
                                                           uint8_t* __restrict__ out, float* __restrict__ scales) {
  const int l = threadIdx.x & 63;
  for (int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); row < n_rows; row += (int64_t)gridDim.x * 4) {
    const float2 v = reinterpret_cast<const float2*>(x + row * kDim)[l];
    const float amax = wave_max(fmaxf(fabsf(v.x), fabsf(v.y)));
    const int e = pow2_scale_exponent(amax);
    const float inv = ldexpf(1.0f, -e);                      // exact: x * 2^-e == x / 2^e
    const uint32_t c0 = f32_to_e4m3_rne_sat(v.x * inv);
    const uint32_t c1 = f32_to_e4m3_rne_sat(v.y * inv);
    reinterpret_cast<uint16_t*>(out + row * kDim)[l] = (uint16_t)(c0 | (c1 << 8));
    if (l == 0) scales[row] = ldexpf(1.0f, e);
  }
}

hipError_t launch_quantize_fp8(const float* x, int64_t n_rows, uint8_t* out, float* scales, hipStream_t s) {
  if (n_rows == 0) return hipSuccess;
  const int64_t grid = (n_rows + 3) / 4;
  hipLaunchKernelGGL(quantize_fp8_kernel, dim3(capped_blocks(grid, 256)), dim3(256), 0, s, x, n_rows, out, scales);
  return hipGetLastError();
}

// float32 rows -> OCP MXFP4. One wave per row, two elements per lane; the 16
// lanes of a 32-element block share its scale 2^e, the smallest with
// max|x| <= 6 * 2^e. E2M1 code of y = x / 2^e: round to nearest on the grid
// 0, .5, 1, 1.5, 2, 3, 4, 6 with ties to the even code, i.e. the count of
// midpoints below |y| (a tie at .25, 1.25, 2.5 or 5 stays on the lower, even
// code; at .75, 1.75 or 3.5 it moves to the upper, even code).
__device__ __forceinline__ uint32_t e2m1_code(float y) {
  const float a = fabsf(y);
  const uint32_t m = (uint32_t)(a > 0.25f) + (uint32_t)(a >= 0.75f) + (uint32_t)(a > 1.25f) + (uint32_t)(a >= 1.75f) +
                     (uint32_t)(a > 2.5f) + (uint32_t)(a >= 3.5f) + (uint32_t)(a > 5.0f);
  return m | ((y < 0.0f && m != 0u) ? 8u : 0u);
}

// Smallest e in [-127, 127] with amax <= top * 2^e (top: the element
// format's largest magnitude, 6 for E2M1 and 7.5 for E2M3; 0 for amax = 0).
__device__ __forceinline__ int mx_block_exponent(float amax, float top) {
  if (!(amax > 0.0f)) return 0;
  int E;
  (void)frexpf(amax, &E);                                   // amax = f * 2^E, f in [0.5, 1)
  int e = E - 4;                                            // below the answer for top < 8
  while (amax > ldexpf(top, e)) ++e;
  return e < -127 ? -127 : (e > 127 ? 127 : e);
}

__global__ __launch_bounds__(256) void quantize_mxfp4_kernel(const float* __restrict__ x, int64_t n_rows,
                                                             uint8_t* __restrict__ out, uint8_t* __restrict__ exps) {
  const int l = threadIdx.x & 63;
  for (int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); row < n_rows; row += (int64_t)gridDim.x * 4) {
    const float2 v = reinterpret_cast<const float2*>(x + row * kDim)[l];
    float amax = fmaxf(fabsf(v.x), fabsf(v.y));
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) amax = fmaxf(amax, __shfl_xor(amax, o));   // within the 16-lane block
    const int e = mx_block_exponent(amax, 6.0f);
    // x * 2^-e, exact: two steps keep the factor a normal float for e = 127
    const float y0 = ldexpf(ldexpf(v.x, -e / 2), -(e - e / 2));
    const float y1 = ldexpf(ldexpf(v.y, -e / 2), -(e - e / 2));
    out[row * 64 + l] = (uint8_t)(e2m1_code(y0) | (e2m1_code(y1) << 4));
    if ((l & 15) == 0) exps[row * 4 + (l >> 4)] = (uint8_t)(e + 127);
  }
}

hipError_t launch_quantize_mxfp4(const float* x, int64_t n_rows, uint8_t* out, uint8_t* exps, hipStream_t s) {
  if (n_rows == 0) return hipSuccess;
  hipLaunchKernelGGL(quantize_mxfp4_kernel, dim3(capped_blocks((n_rows + 3) / 4, 256)), dim3(256), 0, s, x, n_rows, out,
                     exps);
  return hipGetLastError();
}

// float32 rows -> OCP MXFP6 (E2M3 elements). As for MXFP4, one wave per row,
// two elements per lane, and a 32-element block's scale 2^e the smallest with
// max|x| <= 7.5 * 2^e. The E2M3 magnitudes are the multiples of 1/8 in [0, 2),
// of 1/4 in [2, 4) and of 1/2 in [4, 7.5]; on each of these uniform pieces the
// code index is the piece's first index (even) plus y rounded on the piece's
// step, half to even, so ties go to the even code. Each scaling is exact.
__device__ __forceinline__ uint32_t e2m3_code(float y) {
  const float a = fminf(fabsf(y), 7.5f);
  uint32_t idx;
  if (a < 2.0f) idx = (uint32_t)__builtin_rintf(a * 8.0f);                     // 0 .. 16
  else if (a < 4.0f) idx = 16u + (uint32_t)__builtin_rintf((a - 2.0f) * 4.0f);  // 16 .. 24
  else idx = 24u + (uint32_t)__builtin_rintf((a - 4.0f) * 2.0f);                // 24 .. 31
  return idx | ((y < 0.0f && idx != 0u) ? 0x20u : 0u);
}

// Packing: lane i of a block (i = l % 16) holds the block's bits 12i .. 12i + 11
// (its two codes, the even element low); the first lane of every four writes
// their 48 bits as three 16-bit words at byte 6 (i / 4) of the block.
__global__ __launch_bounds__(256) void quantize_mxfp6_kernel(const float* __restrict__ x, int64_t n_rows,
                                                             uint8_t* __restrict__ out, uint8_t* __restrict__ exps) {
  const int l = threadIdx.x & 63;
  for (int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); row < n_rows; row += (int64_t)gridDim.x * 4) {
    const float2 v = reinterpret_cast<const float2*>(x + row * kDim)[l];
    float amax = fmaxf(fabsf(v.x), fabsf(v.y));
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) amax = fmaxf(amax, __shfl_xor(amax, o));   // within the 16-lane block
    const int e = mx_block_exponent(amax, 7.5f);
    const float y0 = ldexpf(ldexpf(v.x, -e / 2), -(e - e / 2));
    const float y1 = ldexpf(ldexpf(v.y, -e / 2), -(e - e / 2));
    const uint32_t bits = e2m3_code(y0) | (e2m3_code(y1) << 6);                 // 12 bits
    const uint32_t b1 = __shfl_down(bits, 1), b2 = __shfl_down(bits, 2), b3 = __shfl_down(bits, 3);
    if ((l & 3) == 0) {
      const uint64_t u = (uint64_t)bits | ((uint64_t)b1 << 12) | ((uint64_t)b2 << 24) | ((uint64_t)b3 << 36);
      uint16_t* dst = reinterpret_cast<uint16_t*>(out + row * 96 + (l >> 4) * 24 + ((l & 15) >> 2) * 6);
      dst[0] = (uint16_t)u;
      dst[1] = (uint16_t)(u >> 16);
      dst[2] = (uint16_t)(u >> 32);
    }
    if ((l & 15) == 0) exps[row * 4 + (l >> 4)] = (uint8_t)(e + 127);
  }
}

hipError_t launch_quantize_mxfp6(const float* x, int64_t n_rows, uint8_t* out, uint8_t* exps, hipStream_t s) {
  if (n_rows == 0) return hipSuccess;
  hipLaunchKernelGGL(quantize_mxfp6_kernel, dim3(capped_blocks((n_rows + 3) / 4, 256)), dim3(256), 0, s, x, n_rows, out,
                     exps);
  return hipGetLastError();
}

// Row copies: dst row (dst_idx ? dst_idx[i] : i) = src row (src_idx ? src_idx[i] : i)
// for i < n, rows of `units` W-byte units (W = 16 or 4). One 64-lane wave per
// row (a row of more than 64 units takes several steps).
template <typename W>
__global__ __launch_bounds__(256) void copy_rows_kernel(const W* __restrict__ src, const int64_t* __restrict__ src_idx,
                                                        W* __restrict__ dst, const int64_t* __restrict__ dst_idx,
                                                        int64_t n, int64_t units) {
  const int l = threadIdx.x & 63;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n; i += (int64_t)gridDim.x * 4) {
    const int64_t s = src_idx ? src_idx[i] : i;
    const int64_t d = dst_idx ? dst_idx[i] : i;
    for (int64_t u = l; u < units; u += 64) dst[d * units + u] = src[s * units + u];
  }
}

hipError_t launch_copy_rows(const void* src, const int64_t* src_idx, void* dst, const int64_t* dst_idx, int64_t n,
                            int64_t row_bytes, hipStream_t s) {
  if (n == 0 || row_bytes == 0) return hipSuccess;
  const unsigned grid = capped_blocks((n + 3) / 4, 256);
  if (row_bytes % 16 == 0 && ((uintptr_t)src % 16) == 0 && ((uintptr_t)dst % 16) == 0) {
    hipLaunchKernelGGL(copy_rows_kernel<uint4>, dim3(grid), dim3(256), 0, s, static_cast<const uint4*>(src), src_idx,
                       static_cast<uint4*>(dst), dst_idx, n, row_bytes / 16);
  } else {
    hipLaunchKernelGGL(copy_rows_kernel<uint32_t>, dim3(grid), dim3(256), 0, s, static_cast<const uint32_t*>(src),
                       src_idx, static_cast<uint32_t*>(dst), dst_idx, n, row_bytes / 4);
  }
  return hipGetLastError();
}

}  // namespace gem
