// MFMA operand fragments of 16-row tiles of 128-d vectors, for the gfx950
// kernels of the scoring library (scorers and nearest-centroid assignment).
#pragma once

#include "device_common.hpp"
#include "../../include/gem.h"

namespace gem {

// --------------------------------------------------------------------------
// Operand fragments. For every type, lane l loads row (l % 16) of a 16-row tile
// and lane group g = l / 16 loads dimensions [32g, 32g + 32) of that row. Inside
// each MFMA the k-slots a lane feeds are a permutation of those dimensions; A
// and B use the same permutation, so each dot product covers all 128 terms.
// Output layout: lane l holds D[4g + v][l % 16], v = 0..3.
template <int DT> struct Op;

template <> struct Op<GEM_F32> {
  static constexpr int kRowBytes = 512;
  struct Frag { float v[32]; };
  static __device__ __forceinline__ void load(Frag& f, const void* vecs, const float*, int64_t row, int g) {
    const float4* p = reinterpret_cast<const float4*>(static_cast<const char*>(vecs) + row * kRowBytes + g * 128);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      float4 t = p[i];
      f.v[4 * i + 0] = t.x; f.v[4 * i + 1] = t.y; f.v[4 * i + 2] = t.z; f.v[4 * i + 3] = t.w;
    }
  }
  static __device__ __forceinline__ void zero(Frag& f) {
#pragma unroll
    for (int i = 0; i < 32; ++i) f.v[i] = 0.0f;
  }
  static __device__ __forceinline__ f32x4 mma(const Frag& a, const Frag& b, f32x4 acc, int s) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[s], b.v[s], acc, 0, 0, 0);
  }
  static constexpr int kSteps = 32;
  static constexpr bool kColumnScale = false;
  static __device__ __forceinline__ void load_b(Frag& f, const void* v, const float* sc, int64_t row, int g) { load(f, v, sc, row, g); }
};

template <> struct Op<GEM_BF16> {
  static constexpr int kRowBytes = 256;
  struct Frag { bf16x8 v[4]; };
  static __device__ __forceinline__ void load(Frag& f, const void* vecs, const float*, int64_t row, int g) {
    const uint4* p = reinterpret_cast<const uint4*>(static_cast<const char*>(vecs) + row * kRowBytes + g * 64);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      uint4 t = p[i];
      f.v[i] = __builtin_bit_cast(bf16x8, t);
    }
  }
  static __device__ __forceinline__ void zero(Frag& f) {
#pragma unroll
    for (int i = 0; i < 4; ++i) f.v[i] = __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
  }
  static __device__ __forceinline__ f32x4 mma(const Frag& a, const Frag& b, f32x4 acc, int s) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v[s], b.v[s], acc, 0, 0, 0);
  }
  static constexpr int kSteps = 4;
  static constexpr bool kColumnScale = false;
  static __device__ __forceinline__ void load_b(Frag& f, const void* v, const float* sc, int64_t row, int g) { load(f, v, sc, row, g); }
};

// float32 values as bfloat16 pairs (hi, lo): lane group g reads block g of
// the row (hi of dims 32g .. 32g + 31, then lo of the same dims), and each
// bf16 step s multiplies lo x hi, hi x lo, then hi x hi into one float32
// accumulator (the small terms first), so a product a*b becomes
// ah*bh + ah*bl + al*bh with every partial product exact.
template <> struct Op<GEM_BF16X3> {
  static constexpr int kRowBytes = 512;
  struct Frag { bf16x8 h[4]; bf16x8 l[4]; };
  static __device__ __forceinline__ void load(Frag& f, const void* vecs, const float*, int64_t row, int g) {
    const uint4* p = reinterpret_cast<const uint4*>(static_cast<const char*>(vecs) + row * kRowBytes + g * 128);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      f.h[i] = __builtin_bit_cast(bf16x8, p[i]);
      f.l[i] = __builtin_bit_cast(bf16x8, p[4 + i]);
    }
  }
  static __device__ __forceinline__ void zero(Frag& f) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      f.h[i] = __builtin_bit_cast(bf16x8, make_uint4(0, 0, 0, 0));
      f.l[i] = f.h[i];
    }
  }
  static __device__ __forceinline__ f32x4 mma(const Frag& a, const Frag& b, f32x4 acc, int s) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l[s], b.h[s], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h[s], b.l[s], acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h[s], b.h[s], acc, 0, 0, 0);
  }
  static constexpr int kSteps = 4;
  static constexpr bool kColumnScale = false;
  static __device__ __forceinline__ void load_b(Frag& f, const void* v, const float* sc, int64_t row, int g) { load(f, v, sc, row, g); }
};

template <> struct Op<GEM_FP8_E4M3> {
  static constexpr int kRowBytes = 128;
  struct Frag { i32x8 v; int scale; };   // scale: E8M0 exponent byte of the row's power-of-two scale
  static __device__ __forceinline__ void load(Frag& f, const void* vecs, const float* scales, int64_t row, int g) {
    const uint4* p = reinterpret_cast<const uint4*>(static_cast<const char*>(vecs) + row * kRowBytes + g * 32);
    uint4 a = p[0], b = p[1];
    f.v = i32x8{(int)a.x, (int)a.y, (int)a.z, (int)a.w, (int)b.x, (int)b.y, (int)b.z, (int)b.w};
    f.scale = (int)((__float_as_uint(scales[row]) >> 23) & 0xffu);
  }
  static __device__ __forceinline__ void zero(Frag& f) {
    f.v = i32x8{0, 0, 0, 0, 0, 0, 0, 0};
    f.scale = 127;
  }
  // Query (B) side: codes only, unit block scale; the query vector's own
  // power-of-two scale multiplies its column after the max over the document
  // (max(s * x) = s * max(x) exactly for s = 2^e > 0).
  static __device__ __forceinline__ void load_b(Frag& f, const void* vecs, const float*, int64_t row, int g) {
    const uint4* p = reinterpret_cast<const uint4*>(static_cast<const char*>(vecs) + row * kRowBytes + g * 32);
    uint4 a = p[0], b = p[1];
    f.v = i32x8{(int)a.x, (int)a.y, (int)a.z, (int)a.w, (int)b.x, (int)b.y, (int)b.z, (int)b.w};
    f.scale = 127;
  }
  static constexpr bool kColumnScale = true;
  static __device__ __forceinline__ f32x4 mma(const Frag& a, const Frag& b, f32x4 acc, int) {
    // OCP E4M3 for both operands (format code 0); E8M0 block scales: each
    // lane's document row (A; all four 32-wide blocks of a row share it) and
    // the unit scale 2^0 for the query side (B), whose scale applies later.
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a.v, b.v, acc, 0, 0, 0, a.scale, 0, 127);
  }
  static constexpr int kSteps = 1;
};

// OCP MXFP4: lane group g holds block g of the row (dims 32g .. 32g + 31, 16
// bytes of E2M1 codes) with that block's E8M0 exponent as the lane's MFMA
// scale, for A and B alike, so the instruction applies the microscaling
// blocks itself. The FP4 operand takes four registers.
template <> struct Op<GEM_MXFP4> {
  static constexpr int kRowBytes = 64;
  struct Frag { i32x4 v; int scale; };
  static __device__ __forceinline__ void load(Frag& f, const void* vecs, const float* scales, int64_t row, int g) {
    const uint4 a = *reinterpret_cast<const uint4*>(static_cast<const char*>(vecs) + row * kRowBytes + g * 16);
    f.v = i32x4{(int)a.x, (int)a.y, (int)a.z, (int)a.w};
    f.scale = (int)reinterpret_cast<const uint8_t*>(scales)[row * 4 + g];
  }
  static __device__ __forceinline__ void zero(Frag& f) {
    f.v = i32x4{0, 0, 0, 0};
    f.scale = 127;
  }
  static __device__ __forceinline__ void load_b(Frag& f, const void* v, const float* sc, int64_t row, int g) {
    load(f, v, sc, row, g);
  }
  static constexpr bool kColumnScale = false;
  static __device__ __forceinline__ f32x4 mma(const Frag& a, const Frag& b, f32x4 acc, int) {
    // E2M1 for both operands (format code 4); each lane's block exponent
    const i32x8 av = i32x8{a.v.x, a.v.y, a.v.z, a.v.w, 0, 0, 0, 0};
    const i32x8 bv = i32x8{b.v.x, b.v.y, b.v.z, b.v.w, 0, 0, 0, 0};
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, acc, 4, 4, 0, a.scale, 0, b.scale);
  }
  static constexpr int kSteps = 1;
};

// OCP MXFP6 (E2M3 elements): lane group g holds block g of the row, 24 bytes
// of 6-bit codes (element t of the block in bits 6t .. 6t + 5), in the six
// low registers of the operand, with that block's E8M0 exponent as the
// lane's MFMA scale, for A and B alike.
template <> struct Op<GEM_MXFP6> {
  static constexpr int kRowBytes = 96;
  struct Frag { i32x8 v; int scale; };
  static __device__ __forceinline__ void load(Frag& f, const void* vecs, const float* scales, int64_t row, int g) {
    const uint2* p = reinterpret_cast<const uint2*>(static_cast<const char*>(vecs) + row * kRowBytes + g * 24);
    const uint2 a = p[0], b = p[1], c = p[2];
    f.v = i32x8{(int)a.x, (int)a.y, (int)b.x, (int)b.y, (int)c.x, (int)c.y, 0, 0};
    f.scale = (int)reinterpret_cast<const uint8_t*>(scales)[row * 4 + g];
  }
  static __device__ __forceinline__ void zero(Frag& f) {
    f.v = i32x8{0, 0, 0, 0, 0, 0, 0, 0};
    f.scale = 127;
  }
  static __device__ __forceinline__ void load_b(Frag& f, const void* v, const float* sc, int64_t row, int g) {
    load(f, v, sc, row, g);
  }
  static constexpr bool kColumnScale = false;
  static __device__ __forceinline__ f32x4 mma(const Frag& a, const Frag& b, f32x4 acc, int) {
    // E2M3 for both operands (format code 2); each lane's block exponent
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a.v, b.v, acc, 2, 2, 0, a.scale, 0, b.scale);
  }
  static constexpr int kSteps = 1;
};

}  // namespace gem
