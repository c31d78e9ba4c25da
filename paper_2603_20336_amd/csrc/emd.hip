// Entropic Earth Mover's Distance between vector sets (GEM, arXiv 2603.20336,
// Sec. 4.2, Eq. EMD; for code sets Eq. qEMD), batched over pairs of sets.
//
// EMD(P1, P2) = min_T sum_ij t_ij d(p_i, p'_j) with row sums 1/m1 and column
// sums 1/m2, d the Euclidean distance. The GPU solves its entropic form (the
// Sinkhorn iteration of Cuturi, 2013) in the log domain: from g = 0, n_iter
// rounds of
//   f_i <- -log m1 - logsumexp_j (g_j - C_ij / eps)
//   g_j <- -log m2 - logsumexp_i (f_i - C_ij / eps)
// then the cost sum_ij exp(f_i + g_j - C_ij / eps) C_ij of that plan.
//
// One workgroup per pair. Thread i < m1 holds row i of the first set in
// registers; the second set streams through LDS in chunks of 16 rows; the
// matrix -C / eps stays in LDS for the whole iteration (at most kMaxEmdCost
// entries), or for larger pairs in a slice of the workspace (a second pass
// over the pairs the first one flagged). Every reduction runs in a fixed
// order, so the result does not depend on the batch.
#include <algorithm>

#include "device_common.hpp"
#include "gem_internal.h"

namespace gem {

namespace {
constexpr int kEmdThreads = 256;
constexpr int kChunk = 16;
}  // namespace

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ float wave_max_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// kBig = false: pairs whose matrix fits LDS (kMaxEmdCost entries); larger
// pairs are flagged for the second pass. kBig = true: the flagged pairs, the
// matrix in this workgroup's slice of the workspace (kMaxSetLen^2 floats).
template <bool kBig>
__global__ __launch_bounds__(kEmdThreads) void emd_sinkhorn_kernel(EmdParams P) {
  __shared__ float K_lds[kBig ? 1 : kMaxEmdCost];   // -C / eps, row-major [m1][m2]
  __shared__ float fpot[kEmdMaxSet], gpot[kEmdMaxSet];
  __shared__ float brow[kChunk][kDim];
  __shared__ float red[kEmdThreads / 64];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const float inv_eps = 1.0f / P.eps;
  float* K = kBig ? P.big + (int64_t)blockIdx.x * kEmdMaxSet * kEmdMaxSet : K_lds;
  for (int64_t pr = blockIdx.x; pr < P.n_pairs; pr += gridDim.x) {
    if (kBig && !P.flags[pr]) continue;
    const int64_t ia = P.a_idx[pr], ib = P.b_idx[pr];
    const int64_t a0 = P.A.off[ia], b0 = P.B.off[ib];
    const int m1 = (int)(P.A.off[ia + 1] - a0), m2 = (int)(P.B.off[ib + 1] - b0);
    if (!kBig) {
      const bool big = m1 * m2 > kMaxEmdCost && m1 <= kEmdMaxSet && m2 <= kEmdMaxSet;
      if (t == 0) P.flags[pr] = big ? 1 : 0;
      // no transport plan for an empty set, nor for a set longer than the
      // bound the host checked: NaN; large matrices wait for the second pass
      if (m1 == 0 || m2 == 0 || m1 > kEmdMaxSet || m2 > kEmdMaxSet || big) {
        if (t == 0) P.out[pr] = __int_as_float(0x7fc00000);
        continue;
      }
    }
    // row t of the first set in registers
    float a[kDim];
    if (t < m1) {
      const int64_t r = P.A.codes ? (int64_t)P.A.codes[a0 + t] : a0 + t;
      const float4* src = reinterpret_cast<const float4*>(static_cast<const float*>(P.A.vecs) + r * kDim);
#pragma unroll
      for (int i = 0; i < kDim / 4; ++i) {
        const float4 v = src[i];
        a[4 * i] = v.x; a[4 * i + 1] = v.y; a[4 * i + 2] = v.z; a[4 * i + 3] = v.w;
      }
    }
    // -C / eps, 16 rows of the second set at a time
    for (int j0 = 0; j0 < m2; j0 += kChunk) {
      const int nj = min(kChunk, m2 - j0);
      for (int e = t; e < nj * kDim; e += kEmdThreads) {
        const int jj = e / kDim, d = e % kDim;
        const int64_t r = P.B.codes ? (int64_t)P.B.codes[b0 + j0 + jj] : b0 + j0 + jj;
        brow[jj][d] = static_cast<const float*>(P.B.vecs)[r * kDim + d];
      }
      __syncthreads();
      if (t < m1) {
        for (int jj = 0; jj < nj; ++jj) {
          float s = 0.0f;
#pragma unroll
          for (int d = 0; d < kDim; ++d) {
            const float df = a[d] - brow[jj][d];
            s = fmaf(df, df, s);
          }
          K[t * m2 + j0 + jj] = -sqrtf(s) * inv_eps;
        }
      }
      __syncthreads();
    }
    const float la = -logf((float)m1), lb = -logf((float)m2);
    for (int j = t; j < m2; j += kEmdThreads) gpot[j] = 0.0f;
    __syncthreads();
    for (int it = 0; it < P.n_iter; ++it) {
      // rows: one wave per row, lanes over the columns
      for (int i = w; i < m1; i += kEmdThreads / 64) {
        float mx = neg_inf();
        for (int j = l; j < m2; j += 64) mx = fmaxf(mx, gpot[j] + K[i * m2 + j]);
        mx = wave_max_f(mx);
        float s = 0.0f;
        for (int j = l; j < m2; j += 64) s += expf(gpot[j] + K[i * m2 + j] - mx);
        s = wave_sum(s);
        if (l == 0) fpot[i] = la - (mx + logf(s));
      }
      __syncthreads();
      // columns: one wave per column, lanes over the rows
      for (int j = w; j < m2; j += kEmdThreads / 64) {
        float mx = neg_inf();
        for (int i = l; i < m1; i += 64) mx = fmaxf(mx, fpot[i] + K[i * m2 + j]);
        mx = wave_max_f(mx);
        float s = 0.0f;
        for (int i = l; i < m1; i += 64) s += expf(fpot[i] + K[i * m2 + j] - mx);
        s = wave_sum(s);
        if (l == 0) gpot[j] = lb - (mx + logf(s));
      }
      __syncthreads();
    }
    // cost of the plan: rows over the waves, then the waves in order
    float acc = 0.0f;
    for (int i = w; i < m1; i += kEmdThreads / 64) {
      float s = 0.0f;
      for (int j = l; j < m2; j += 64) {
        const float k = K[i * m2 + j];
        s += expf(fpot[i] + gpot[j] + k) * (-k * P.eps);
      }
      acc += wave_sum(s);
    }
    if (l == 0) red[w] = acc;
    __syncthreads();
    if (t == 0) {
      float tot = 0.0f;
      for (int i = 0; i < kEmdThreads / 64; ++i) tot += red[i];
      P.out[pr] = tot;
    }
    __syncthreads();
  }
}

size_t emd_ws_bytes(int64_t n_pairs) {
  return (((size_t)n_pairs + 255) & ~(size_t)255) + (size_t)kEmdBigBlocks * kEmdMaxSet * kEmdMaxSet * 4;
}

hipError_t launch_emd_sinkhorn(EmdParams P, void* ws, hipStream_t s) {
  if (P.n_pairs == 0) return hipSuccess;
  P.flags = static_cast<uint8_t*>(ws);
  P.big = reinterpret_cast<float*>(static_cast<char*>(ws) + (((size_t)P.n_pairs + 255) & ~(size_t)255));
  hipLaunchKernelGGL(emd_sinkhorn_kernel<false>, dim3(capped_blocks(P.n_pairs, kEmdThreads)), dim3(kEmdThreads), 0, s, P);
  hipLaunchKernelGGL(emd_sinkhorn_kernel<true>, dim3((unsigned)std::min<int64_t>(P.n_pairs, kEmdBigBlocks)),
                     dim3(kEmdThreads), 0, s, P);
  return hipGetLastError();
}

}  // namespace gem
