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
// One workgroup per pair. To build the matrix, each lane group of row i holds
// row i of the first set in registers while the second set streams through
// LDS in chunks of 16 rows; the matrix of -C / eps (base 2) stays in LDS for the
// whole iteration (at most kMaxEmdCost entries), or for larger pairs in a
// slice of the workspace (a second pass over the pairs the first one flagged). Every reduction runs in
// a fixed order, so the result does not depend on the batch.
#include <algorithm>

#include "device_common.hpp"
#include "gem_internal.h"

namespace gem {

namespace {
constexpr int kEmdThreads = 256;
constexpr int kChunk = 16;
}  // namespace

// A group of up to eight consecutive lanes per row (then per column) of the
// matrix, as many as the 256 threads allow: each logsumexp is a two-pass loop
// (max, then the sum of powers) over the group's interleaved share of the row,
// then a butterfly over the group. The matrix is stored with an odd row
// stride, so the row pass (lanes walk rows) and the column pass (lanes walk
// columns) both read distinct LDS banks. The iteration runs in base 2: with L_ij = -C_ij
// log2(e) / eps and potentials in log2 units it is the same iteration (every
// term scaled by log2 e), evaluated with the hardware exp2 / log2.
__device__ __forceinline__ float hw_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float hw_log2(float x) { return __builtin_amdgcn_logf(x); }

// log2 of sum_k 2^(p[k * ps] + q[k * qs]) over k < n, split over s lanes (s
// a power of two, the group's lanes consecutive): lane j of the group takes
// k = j, j + s, ..., first the maximum, then the sum of powers, each over U
// interleaved partial results (loads in flight: a workgroup per CU leaves few
// waves to hide the latency); the lanes' partial maxima and sums are then
// combined across the group by an xor butterfly (a fixed order), and every
// lane of the group returns the total.
template <int U, int s>
__device__ __forceinline__ float lse2_split(const float* p, int ps, const float* q, int qs, int n, int j,
                                            bool active) {
  float m[U], sm[U];
#pragma unroll
  for (int u = 0; u < U; ++u) { m[u] = -INFINITY; sm[u] = 0.0f; }
  if (active) {
    int k = j;
    for (; k + (U - 1) * s < n; k += U * s) {
#pragma unroll
      for (int u = 0; u < U; ++u) m[u] = fmaxf(m[u], p[(k + u * s) * ps] + q[(k + u * s) * qs]);
    }
    for (int u = 0; k < n; ++u, k += s) m[u] = fmaxf(m[u], p[k * ps] + q[k * qs]);
  }
  float mx = m[0];
#pragma unroll
  for (int u = 1; u < U; ++u) mx = fmaxf(mx, m[u]);
  if (active && mx > -INFINITY) {
    int k = j;
    for (; k + (U - 1) * s < n; k += U * s) {
#pragma unroll
      for (int u = 0; u < U; ++u) sm[u] += hw_exp2(p[(k + u * s) * ps] + q[(k + u * s) * qs] - mx);
    }
    for (int u = 0; k < n; ++u, k += s) sm[u] += hw_exp2(p[k * ps] + q[k * qs] - mx);
  }
  float sum = sm[0];
#pragma unroll
  for (int u = 1; u < U; ++u) sum += sm[u];
  for (int o = 1; o < s; o <<= 1) {
    const float om = __shfl_xor(mx, o), os = __shfl_xor(sum, o);
    const float nm = fmaxf(mx, om);
    sum = (mx > -INFINITY ? sum * hw_exp2(mx - nm) : 0.0f) + (om > -INFINITY ? os * hw_exp2(om - nm) : 0.0f);
    mx = nm;
  }
  return mx + hw_log2(sum);
}

// lanes per row (or column) for n rows: as many as 256 threads allow, a power of two up to 8
__device__ __forceinline__ int lse_split(int n) { return n > 128 ? 1 : (n > 64 ? 2 : (n > 32 ? 4 : 8)); }

// lse2_split with the group size s (uniform over the workgroup) as a constant
__device__ __forceinline__ float lse2_groups(const float* p, int ps, const float* q, int qs, int n, int j, int s,
                                             bool active) {
  switch (s) {
    case 1: return lse2_split<8, 1>(p, ps, q, qs, n, j, active);
    case 2: return lse2_split<8, 2>(p, ps, q, qs, n, j, active);
    case 4: return lse2_split<8, 4>(p, ps, q, qs, n, j, active);
    default: return lse2_split<8, 8>(p, ps, q, qs, n, j, active);
  }
}

// kBig = false: pairs whose matrix fits LDS (kMaxEmdCost entries, stride
// included); larger pairs are flagged for the second pass. kBig = true: the
// flagged pairs, the matrix in this workgroup's slice of the workspace.
template <bool kBig>
__global__ __launch_bounds__(kEmdThreads) void emd_sinkhorn_kernel(EmdParams P) {
  __shared__ float K_lds[kBig ? 1 : kMaxEmdCost];   // L = -C log2(e) / eps, [m1][stride]
  __shared__ float fpot[kEmdMaxSet], gpot[kEmdMaxSet];
  __shared__ float brow[kChunk][kDim];
  __shared__ float red[kEmdThreads];
  const int t = threadIdx.x;
  const float kLog2e = 1.4426950408889634f;
  const float scale = kLog2e / P.eps;                // L = -C * scale
  float* K = kBig ? P.big + (int64_t)blockIdx.x * kEmdMaxSet * (kEmdMaxSet + 1) : K_lds;
  for (int64_t pr = blockIdx.x; pr < P.n_pairs; pr += gridDim.x) {
    if (kBig && !P.flags[pr]) continue;
    const int64_t ia = P.a_idx[pr], ib = P.b_idx[pr];
    const int64_t a0 = P.A.off[ia], b0 = P.B.off[ib];
    const int m1 = (int)(P.A.off[ia + 1] - a0), m2 = (int)(P.B.off[ib + 1] - b0);
    const int ld = m2 | 1;                                    // odd row stride
    if (!kBig) {
      const bool big = m1 * ld > kMaxEmdCost && m1 <= kEmdMaxSet && m2 <= kEmdMaxSet;
      if (t == 0) P.flags[pr] = big ? 1 : 0;
      // no transport plan for an empty set, nor for a set longer than the
      // bound the host checked: NaN; large matrices wait for the second pass
      if (m1 == 0 || m2 == 0 || m1 > kEmdMaxSet || m2 > kEmdMaxSet || big) {
        if (t == 0) P.out[pr] = __int_as_float(0x7fc00000);
        continue;
      }
    }
    // groups of sr (sc) consecutive lanes per row (column) of the matrix
    const int sr = lse_split(m1), sc = lse_split(m2);
    const int ri = t / sr, rj = t % sr, ci = t / sc, cj = t % sc;
    // row ri of the first set in registers (in every lane of its group)
    float a[kDim];
    if (ri < m1) {
      const int64_t r = P.A.codes ? (int64_t)P.A.codes[a0 + ri] : a0 + ri;
      const float4* src = reinterpret_cast<const float4*>(static_cast<const float*>(P.A.vecs) + r * kDim);
#pragma unroll
      for (int i = 0; i < kDim / 4; ++i) {
        const float4 v = src[i];
        a[4 * i] = v.x; a[4 * i + 1] = v.y; a[4 * i + 2] = v.z; a[4 * i + 3] = v.w;
      }
    }
    // L, 16 rows of the second set at a time; lane rj of row ri's group
    // takes the chunk's rows rj, rj + sr, ...
    for (int j0 = 0; j0 < m2; j0 += kChunk) {
      const int nj = min(kChunk, m2 - j0);
      for (int e = t; e < nj * kDim; e += kEmdThreads) {
        const int jj = e / kDim, d = e % kDim;
        const int64_t r = P.B.codes ? (int64_t)P.B.codes[b0 + j0 + jj] : b0 + j0 + jj;
        brow[jj][d] = static_cast<const float*>(P.B.vecs)[r * kDim + d];
      }
      __syncthreads();
      if (ri < m1) {
        for (int jj = rj; jj < nj; jj += sr) {
          float s = 0.0f;
#pragma unroll
          for (int d = 0; d < kDim; ++d) {
            const float df = a[d] - brow[jj][d];
            s = fmaf(df, df, s);
          }
          K[ri * ld + j0 + jj] = -sqrtf(s) * scale;
        }
      }
      __syncthreads();
    }
    const float la = -hw_log2((float)m1), lb = -hw_log2((float)m2);
    if (t < m2) gpot[t] = 0.0f;
    __syncthreads();
    for (int it = 0; it < P.n_iter; ++it) {
      const float fr = la - lse2_groups(gpot, 1, K + min(ri, m1 - 1) * ld, 1, m2, rj, sr, ri < m1);
      if (ri < m1 && rj == 0) fpot[ri] = fr;
      __syncthreads();
      const float gc = lb - lse2_groups(fpot, 1, K + min(ci, m2 - 1), ld, m1, cj, sc, ci < m2);
      if (ci < m2 && cj == 0) gpot[ci] = gc;
      __syncthreads();
    }
    // cost of the plan: each thread its row, then the rows in order
    float acc = 0.0f;
    if (t < m1) {
      const float* row = K + t * ld;
      for (int j = 0; j < m2; ++j) acc += hw_exp2(fpot[t] + gpot[j] + row[j]) * (-row[j] / scale);
    }
    red[t] = acc;
    __syncthreads();
    if (t == 0) {
      float tot = 0.0f;
      for (int i = 0; i < m1; ++i) tot += red[i];
      P.out[pr] = tot;
    }
    __syncthreads();
  }
}

size_t emd_ws_bytes(int64_t n_pairs) {
  return (((size_t)n_pairs + 255) & ~(size_t)255) + (size_t)kEmdBigBlocks * kEmdMaxSet * (kEmdMaxSet + 1) * 4;
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
