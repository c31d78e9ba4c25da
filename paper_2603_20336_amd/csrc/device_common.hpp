// Device-side helpers shared by the gfx950 kernels of the scoring library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gem {

constexpr int kDim = 128;
constexpr int kWave = 64;

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) int i32x8;
typedef __attribute__((ext_vector_type(4))) int i32x4;

__device__ __forceinline__ float neg_inf() { return __int_as_float(0xff800000u); }

// ----------------------------------------------------------------- number formats
// bfloat16: keep the top 16 bits of the binary32 pattern, rounding the dropped
// half to nearest, ties to even; NaN becomes a quiet NaN with the same sign.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)(((u >> 16) & 0x8000u) | 0x7fc0u);
  uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)((u + 0x7fffu + lsb) >> 16);
}

// OCP FP8 E4M3 (bias 7, no infinities, S.1111.111 = NaN, max 448): nearest
// value, ties to the even code, magnitudes >= 448 saturate to 448.
__device__ __forceinline__ uint32_t f32_to_e4m3_rne_sat(float x) {
  uint32_t u = __float_as_uint(x);
  uint32_t sign = (u >> 24) & 0x80u;
  uint32_t mag = u & 0x7fffffffu;
  if (mag > 0x7f800000u) return 0x7fu;                      // NaN
  if (mag >= 0x43e00000u) return sign | 0x7eu;              // |x| >= 448
  if (mag < 0x3c800000u) {                                  // |x| < 2^-6: subnormal grid 2^-9
    float a = __uint_as_float(mag) * 512.0f;                // exact power-of-two scaling
    uint32_t m = (uint32_t)__builtin_rintf(a);              // ties to even; 8 -> code 0x08
    return sign | m;
  }
  int e = (int)(mag >> 23) - 127;                           // -6 .. 8
  uint32_t man = mag & 0x7fffffu;
  uint32_t m = man >> 20;
  uint32_t rem = man & 0xfffffu;
  if (rem > 0x80000u || (rem == 0x80000u && (m & 1u))) m += 1;
  if (m == 8) { m = 0; e += 1; }
  return sign | ((uint32_t)(e + 7) << 3) | m;
}

// Smallest e in [-126, 127] with amax <= 448 * 2^e (e = 0 for amax = 0).
__device__ __forceinline__ int pow2_scale_exponent(float amax) {
  if (!(amax > 0.0f)) return 0;
  int E;
  (void)frexpf(amax, &E);                                   // amax = f * 2^E, f in [0.5, 1)
  int e = E - 12;
  while (amax > ldexpf(448.0f, e)) ++e;
  return e < -126 ? -126 : (e > 127 ? 127 : e);
}

// Float -> unsigned key whose unsigned order is the float order.
__device__ __forceinline__ uint32_t float_order_key(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float float_from_order_key(uint32_t k) {
  uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __uint_as_float(u);
}

// ----------------------------------------------------------------- wave helpers
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// 64-bit values of one lane (both halves read as unsigned: the builtins return
// int, which would sign-extend into the high half)
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int lane) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)(v >> 32), lane) << 32) |
         (uint64_t)(uint32_t)__builtin_amdgcn_readlane((uint32_t)v, lane);
}
__device__ __forceinline__ uint64_t readfirstlane_u64(uint64_t v) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
         (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
}

__device__ __forceinline__ float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// Max across the four 16-lane groups (lanes l, l^16, l^32, l^48).
__device__ __forceinline__ float max_across_groups(float v) {
  v = fmaxf(v, __shfl_xor(v, 16));
  v = fmaxf(v, __shfl_xor(v, 32));
  return v;
}

__device__ __forceinline__ float max4(f32x4 a) {
  return fmaxf(fmaxf(a[0], a[1]), fmaxf(a[2], a[3]));
}

// Binary search: largest i in [lo, hi) with a[i] <= x (a non-decreasing), lo if none.
__device__ __forceinline__ int64_t upper_index(const int64_t* a, int64_t lo, int64_t hi, int64_t x) {
  int64_t l = lo, h = hi;          // invariant: a[l] <= x (caller guarantees a[lo] <= x)
  while (h - l > 1) {
    int64_t m = (l + h) >> 1;
    if (a[m] <= x) l = m; else h = m;
  }
  return l;
}

}  // namespace gem
