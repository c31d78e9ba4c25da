// Codebook kernels for the quantized Chamfer estimate (GEM, arXiv 2603.20336):
// the nearest-centroid map NN(x) onto the k-means vocabulary C_quant
// (Secs. 4.1, 4.2) on MFMA, and the k-means centroid update.
//
// NN(x) = argmin_j ||x - c_j||^2 = argmax_j (<x, c_j> - ||c_j||^2 / 2), ties to
// the smallest j. The rows x are the MFMA B operand (columns, held in
// registers), the centroids the A operand (16-row tiles streamed through a
// register ring), so each lane's four accumulators are four centroids of one
// row. A (value, index) pair is packed into one 64-bit key whose unsigned order
// is "larger value, then smaller index"; partial results of centroid slices
// merge with an atomic max, which does not depend on their order, so the codes
// are the same for any launch split.
#include "device_common.hpp"
#include "gem_internal.h"
#include "mfma_ops.hpp"

namespace gem {

namespace {
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
int64_t tiles_of(int64_t k) { return (k + 15) / 16; }
}  // namespace

// --------------------------------------------------------------------------
// Nearest centroid

// Workspace: [n_rows] 64-bit keys, then the half squared norms of the
// centroids padded to whole 16-row tiles.
size_t nearest_centroid_ws_bytes(int64_t n_rows, int64_t n_centroids) {
  return align256((size_t)n_rows * 8) + align256((size_t)tiles_of(n_centroids) * 16 * 4);
}

// 0.5 ||c_j||^2 in the operand dtype's values (a wave per row, two elements
// per lane, a fixed shuffle tree). Padding rows of the last tile get +inf, so
// their value <x, c> - inf never wins.
template <int DT>
__global__ __launch_bounds__(256) void half_norms_kernel(const void* __restrict__ C, int64_t k, int64_t k_pad,
                                                         float* __restrict__ hn) {
  const int l = threadIdx.x & 63;
  for (int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); j < k_pad; j += (int64_t)gridDim.x * 4) {
    if (j >= k) {
      if (l == 0) hn[j] = __int_as_float(0x7f800000);
      continue;
    }
    float a, b;
    if constexpr (DT == GEM_F32) {
      const float2 v = reinterpret_cast<const float2*>(static_cast<const float*>(C) + j * kDim)[l];
      a = v.x;
      b = v.y;
    } else {
      const uint32_t u = reinterpret_cast<const uint32_t*>(static_cast<const uint16_t*>(C) + j * kDim)[l];
      a = __uint_as_float(u << 16);
      b = __uint_as_float(u & 0xffff0000u);
    }
    float s = a * a + b * b;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (l == 0) hn[j] = 0.5f * s;
  }
}

__global__ __launch_bounds__(256) void zero_u64_kernel(unsigned long long* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0ull;
}

__global__ __launch_bounds__(256) void decode_keys_kernel(const unsigned long long* __restrict__ keys, int64_t n,
                                                          int32_t* __restrict__ codes) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    codes[i] = (int32_t)(0xffffffffu - (uint32_t)(keys[i] & 0xffffffffull));
}

// Larger value first, then the smaller centroid index.
__device__ __forceinline__ unsigned long long assign_key(float v, int j) {
  return ((unsigned long long)float_order_key(v) << 32) | (unsigned long long)(0xffffffffu - (uint32_t)j);
}

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int m) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m);
  return ((unsigned long long)hi << 32) | lo;
}

// kNT: 16-row column tiles of x per wave; kDepth: centroid tiles in flight.
template <int DT> struct AssignCfg;
template <> struct AssignCfg<GEM_F32> { static constexpr int kNT = 4; static constexpr int kDepth = 2; };
template <> struct AssignCfg<GEM_BF16> { static constexpr int kNT = 8; static constexpr int kDepth = 3; };

struct AssignParams {
  const void* x;
  int64_t n;                   // rows of x
  const void* C;
  int64_t k;                   // centroids
  int64_t n_tiles;             // 16-row centroid tiles (the last one padded)
  const float* hn;             // [n_tiles * 16] half squared norms (+inf padding)
  unsigned long long* keys;    // [n] best key per row, merged by atomic max
  int64_t n_rb;                // row blocks of 16 * kNT rows
  int64_t n_slices;            // centroid slices
  int64_t tiles_per_slice;
};

// Workgroup b takes centroid slice b % n_slices for four consecutive row
// blocks (one per wave), so that its waves read the same centroid tiles at
// about the same time.
template <int DT>
__global__ __launch_bounds__(256) void nearest_centroid_kernel(AssignParams P) {
  using O = Op<DT>;
  using Frag = typename O::Frag;
  constexpr int NT = AssignCfg<DT>::kNT, PF = AssignCfg<DT>::kDepth;
  const int l = threadIdx.x & 63, g = l >> 4, c16 = l & 15;
  const int64_t slice = blockIdx.x % P.n_slices;
  const int64_t rb = (blockIdx.x / P.n_slices) * 4 + (threadIdx.x >> 6);
  if (rb >= P.n_rb) return;
  const int64_t t0 = slice * P.tiles_per_slice;
  const int64_t t1 = min(P.n_tiles, t0 + P.tiles_per_slice);
  if (t0 >= t1) return;
  const int64_t r0 = rb * 16 * NT;

  Frag B[NT];
#pragma unroll
  for (int ct = 0; ct < NT; ++ct) O::load_b(B[ct], P.x, nullptr, min(r0 + 16 * ct + c16, P.n - 1), g);

  // row of centroid tile t that this lane loads (tiles clamped into the slice,
  // rows past the last centroid repeat it)
  auto crow = [&](int64_t t) -> int64_t { return min(min(t, t1 - 1) * 16 + c16, P.k - 1); };
  const float4* hn4 = reinterpret_cast<const float4*>(P.hn);
  Frag A[PF];
  float4 H[PF];
#pragma unroll
  for (int j = 0; j < PF; ++j) {
    O::load(A[j], P.C, nullptr, crow(t0 + j), g);
    H[j] = hn4[min(t0 + j, t1 - 1) * 4 + g];
    __builtin_amdgcn_sched_barrier(0);
  }
  float bv[NT];
  int bi[NT];
#pragma unroll
  for (int ct = 0; ct < NT; ++ct) { bv[ct] = neg_inf(); bi[ct] = 0; }

  for (int64_t T0 = t0; T0 < t1; T0 += PF) {
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int64_t t = T0 + j;
      const bool live = t < t1;
      f32x4 acc[NT];
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
      if (live) {
#pragma unroll
        for (int s = 0; s < O::kSteps; ++s)
#pragma unroll
          for (int ct = 0; ct < NT; ++ct) acc[ct] = O::mma(A[j], B[ct], acc[ct], s);
      }
      const float4 h = H[j];
      // the slot is free once its products are issued: load the tile PF ahead
      // (unconditionally, clamped, so that every step issues the same loads)
      O::load(A[j], P.C, nullptr, crow(t + PF), g);
      H[j] = hn4[min(t + PF, t1 - 1) * 4 + g];
      if (live) {
        // lane (g, c16) holds centroids 16t + 4g + v of row r0 + 16ct + c16;
        // strict > over increasing indices keeps the first of equal values
        const int jb = (int)(t * 16 + 4 * g);
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
          const float v0 = acc[ct][0] - h.x, v1 = acc[ct][1] - h.y;
          const float v2 = acc[ct][2] - h.z, v3 = acc[ct][3] - h.w;
          if (v0 > bv[ct]) { bv[ct] = v0; bi[ct] = jb; }
          if (v1 > bv[ct]) { bv[ct] = v1; bi[ct] = jb + 1; }
          if (v2 > bv[ct]) { bv[ct] = v2; bi[ct] = jb + 2; }
          if (v3 > bv[ct]) { bv[ct] = v3; bi[ct] = jb + 3; }
        }
      }
    }
  }
#pragma unroll
  for (int ct = 0; ct < NT; ++ct) {
    unsigned long long key = assign_key(bv[ct], bi[ct]);
    key = max(key, shfl_xor_u64(key, 16));
    key = max(key, shfl_xor_u64(key, 32));
    const int64_t row = r0 + 16 * ct + c16;
    if (g == 0 && row < P.n) atomicMax(&P.keys[row], key);
  }
}

hipError_t launch_nearest_centroid(int dtype, const void* x, int64_t n_rows, const void* C, int64_t k, int32_t* codes,
                                   void* ws, int n_cu, hipStream_t s) {
  if (n_rows == 0) return hipSuccess;
  if (k <= 0 || (dtype != GEM_F32 && dtype != GEM_BF16)) return hipErrorInvalidValue;
  unsigned long long* keys = static_cast<unsigned long long*>(ws);
  float* hn = reinterpret_cast<float*>(static_cast<char*>(ws) + align256((size_t)n_rows * 8));
  const int64_t n_tiles = tiles_of(k);
  const int64_t k_pad = n_tiles * 16;
  const unsigned norm_grid = capped_blocks((k_pad + 3) / 4, 256);
  if (dtype == GEM_F32) hipLaunchKernelGGL(half_norms_kernel<GEM_F32>, dim3(norm_grid), dim3(256), 0, s, C, k, k_pad, hn);
  else hipLaunchKernelGGL(half_norms_kernel<GEM_BF16>, dim3(norm_grid), dim3(256), 0, s, C, k, k_pad, hn);
  hipLaunchKernelGGL(zero_u64_kernel, dim3(capped_blocks((n_rows + 255) / 256, 256)), dim3(256), 0, s, keys, n_rows);

  const int nt = dtype == GEM_F32 ? AssignCfg<GEM_F32>::kNT : AssignCfg<GEM_BF16>::kNT;
  AssignParams P;
  P.x = x; P.n = n_rows; P.C = C; P.k = k; P.n_tiles = n_tiles; P.hn = hn; P.keys = keys;
  P.n_rb = (n_rows + 16 * nt - 1) / (16 * nt);
  // centroid slices: about 16 waves per CU in all, no slice under 8 tiles
  const int64_t want_waves = (int64_t)(n_cu > 0 ? n_cu : 256) * 16;
  int64_t ns = (want_waves + P.n_rb - 1) / P.n_rb;
  ns = std::max<int64_t>(1, std::min<int64_t>(ns, n_tiles / 8));
  P.tiles_per_slice = (n_tiles + ns - 1) / ns;
  P.n_slices = (n_tiles + P.tiles_per_slice - 1) / P.tiles_per_slice;
  const int64_t grid = ((P.n_rb + 3) / 4) * P.n_slices;
  if (grid > kMaxGridThreads / 256) return hipErrorInvalidValue;
  if (dtype == GEM_F32)
    hipLaunchKernelGGL(nearest_centroid_kernel<GEM_F32>, dim3((unsigned)grid), dim3(256), 0, s, P);
  else
    hipLaunchKernelGGL(nearest_centroid_kernel<GEM_BF16>, dim3((unsigned)grid), dim3(256), 0, s, P);
  hipLaunchKernelGGL(decode_keys_kernel, dim3(capped_blocks((n_rows + 255) / 256, 256)), dim3(256), 0, s, keys, n_rows,
                     codes);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// k-means centroid update
//
// Each element x is added as the integer rint(x 2^sh), with sh chosen from
// max |x| and the row count so that no sum can reach 2^62: integer adds are
// exact, so the sums, and the means computed from them, do not depend on the
// order in which rows arrive.

// Workspace: [k][128] int64 sums, [k] int32 counts, one word for max |x|.
size_t centroid_update_ws_bytes(int64_t n_rows, int64_t n_centroids) {
  (void)n_rows;
  return align256((size_t)n_centroids * kDim * 8) + align256((size_t)n_centroids * 4) + 256;
}

__device__ __forceinline__ int fixed_point_shift(uint32_t amax_bits, int64_t n_rows) {
  const float amax = __uint_as_float(amax_bits);
  int e = 0;                                                  // amax < 2^e
  if (amax > 0.0f) (void)frexpf(amax, &e);
  int ln = 0;                                                 // n_rows <= 2^ln
  while (ln < 62 && (int64_t(1) << ln) < n_rows) ++ln;
  return 62 - e - ln;
}

__global__ __launch_bounds__(256) void zero_words_kernel(uint32_t* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0u;
}

__global__ __launch_bounds__(256) void absmax_kernel(const float* __restrict__ x, int64_t n_elems,
                                                     uint32_t* __restrict__ amax_bits) {
  uint32_t m = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n_elems; i += (int64_t)gridDim.x * 256)
    m = max(m, __float_as_uint(x[i]) & 0x7fffffffu);          // |x| bit patterns order like the values
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(amax_bits, m);
}

// One wave per row, two elements per lane.
__global__ __launch_bounds__(256) void centroid_accumulate_kernel(const float* __restrict__ x, int64_t n,
                                                                  const int32_t* __restrict__ codes,
                                                                  const uint32_t* __restrict__ amax_bits,
                                                                  unsigned long long* __restrict__ sums,
                                                                  int32_t* __restrict__ counts) {
  const int l = threadIdx.x & 63;
  const int sh = fixed_point_shift(*amax_bits, n);
  for (int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); row < n; row += (int64_t)gridDim.x * 4) {
    const int64_t c = codes[row];
    const float2 v = reinterpret_cast<const float2*>(x + row * kDim)[l];
    const long long a = (long long)rintf(ldexpf(v.x, sh));
    const long long b = (long long)rintf(ldexpf(v.y, sh));
    atomicAdd(&sums[c * kDim + 2 * l], (unsigned long long)a);
    atomicAdd(&sums[c * kDim + 2 * l + 1], (unsigned long long)b);
    if (l == 0) atomicAdd(&counts[c], 1);
  }
}

// One wave per centroid: the mean of its rows, or its old value when it has none.
__global__ __launch_bounds__(256) void centroid_finalize_kernel(const unsigned long long* __restrict__ sums,
                                                                const int32_t* __restrict__ counts,
                                                                const uint32_t* __restrict__ amax_bits, int64_t n,
                                                                const float* old, int64_t k, float* out) {
  const int l = threadIdx.x & 63;
  const int sh = fixed_point_shift(*amax_bits, n);
  for (int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); j < k; j += (int64_t)gridDim.x * 4) {
    const int cnt = counts[j];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t i = j * kDim + 2 * l + h;
      const float prev = old[i];
      out[i] = cnt > 0 ? (float)(ldexp((double)(long long)sums[i], -sh) / (double)cnt) : prev;
    }
  }
}

hipError_t launch_centroid_update(const float* x, int64_t n_rows, const int32_t* codes, const float* centroids,
                                  int64_t k, float* new_centroids, int32_t* counts, void* ws, hipStream_t s) {
  if (k == 0) return hipSuccess;
  unsigned long long* sums = static_cast<unsigned long long*>(ws);
  char* p = static_cast<char*>(ws) + align256((size_t)k * kDim * 8);
  int32_t* cnt = counts ? counts : reinterpret_cast<int32_t*>(p);
  uint32_t* amax = reinterpret_cast<uint32_t*>(p + align256((size_t)k * 4));
  hipLaunchKernelGGL(zero_u64_kernel, dim3(capped_blocks((k * kDim + 255) / 256, 256)), dim3(256), 0, s, sums,
                     k * kDim);
  hipLaunchKernelGGL(zero_words_kernel, dim3(capped_blocks((k + 255) / 256, 256)), dim3(256), 0, s,
                     reinterpret_cast<uint32_t*>(cnt), k);
  hipLaunchKernelGGL(zero_words_kernel, dim3(1), dim3(256), 0, s, amax, (int64_t)1);
  if (n_rows > 0) {
    hipLaunchKernelGGL(absmax_kernel, dim3(capped_blocks(std::min<int64_t>((n_rows * kDim + 255) / 256, 4096), 256)),
                       dim3(256), 0, s, x, n_rows * kDim, amax);
    hipLaunchKernelGGL(centroid_accumulate_kernel, dim3(capped_blocks((n_rows + 3) / 4, 256)), dim3(256), 0, s, x,
                       n_rows, codes, amax, sums, cnt);
  }
  hipLaunchKernelGGL(centroid_finalize_kernel, dim3(capped_blocks((k + 3) / 4, 256)), dim3(256), 0, s, sums, cnt, amax,
                     n_rows, centroids, k, new_centroids);
  return hipGetLastError();
}

}  // namespace gem
