// Cluster-guided beam search (GEM, arXiv 2603.20336, Alg. 5) for a batch of
// queries at once, and the set-level clustering it prunes with (Sec. 4.1).
//
// Set-level clustering: TF(j, P) = vectors of P whose nearest C_index centroid
// is j; IDF(j) = log(N / (1 + sets touching j)); C_top(P) = the r clusters of
// P with the largest TF * IDF (ties to the smaller cluster). C_top(P) is a
// bit mask; a cluster's members are the sets whose mask holds it, in id order.
//
// Search state per query: the result set R (a gem_beam row, sorted), a visited
// and an expanded bit map over the sets, and the C_query mask. One step takes
// the w best unexpanded entries of R (all of Alg. 5's paths advance at once),
// marks them expanded, and lists their neighbours that are unvisited and
// share a cluster with C_query (marking them visited); the gathered scorer
// then scores the list and the beam merge folds it into R. A query whose R
// holds no unexpanded entry lists nothing; the host stops when no query did.
//
// Every kernel here gives each query (or set, or cluster) one wave or one
// workgroup; all bounds come from the host-checked sizes.
#include "device_common.hpp"
#include "gem_internal.h"

namespace gem {

namespace {
constexpr int kMaxClusters = 1024;
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(capped_blocks((n + 255) / 256, 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void fill_i32_kernel(int32_t* __restrict__ p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}


// ------------------------------------------------------------------ clustering

// One wave per set: its cluster histogram in LDS; every cluster it touches
// adds one to df.
__global__ __launch_bounds__(256) void set_df_kernel(const int32_t* __restrict__ vc, const int64_t* __restrict__ off,
                                                     int64_t n_sets, int k2, int32_t* __restrict__ df) {
  __shared__ int hist[4][kMaxClusters];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  // rounds over the workgroup's base index: every wave runs the same rounds,
  // so the barriers stay uniform
  for (int64_t base = (int64_t)blockIdx.x * 4; base < n_sets; base += (int64_t)gridDim.x * 4) {
    const int64_t s = base + w;
    const bool live = s < n_sets;
    for (int j = l; j < k2; j += 64) hist[w][j] = 0;
    __syncthreads();
    if (live) {
      for (int64_t i = off[s] + l; i < off[s + 1]; i += 64) atomicAdd(&hist[w][vc[i]], 1);
    }
    __syncthreads();
    if (live) {
      for (int j = l; j < k2; j += 64)
        if (hist[w][j] > 0) atomicAdd(&df[j], 1);
    }
    __syncthreads();
  }
}

// One wave per set: scores TF * IDF of the clusters it touches, r rounds of a
// wave arg-max (larger score, then smaller cluster), bits into its mask.
__global__ __launch_bounds__(256) void set_top_clusters_kernel(const int32_t* __restrict__ vc,
                                                               const int64_t* __restrict__ off, int64_t n_sets, int k2,
                                                               int r, const int32_t* __restrict__ df,
                                                               uint32_t* __restrict__ mask) {
  __shared__ int hist[4][kMaxClusters];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int words = (k2 + 31) / 32;
  const float n = (float)n_sets;
  for (int64_t base = (int64_t)blockIdx.x * 4; base < n_sets; base += (int64_t)gridDim.x * 4) {
    const int64_t s = base + w;
    const bool live = s < n_sets;
    for (int j = l; j < k2; j += 64) hist[w][j] = 0;
    __syncthreads();
    if (live) {
      for (int64_t i = off[s] + l; i < off[s + 1]; i += 64) atomicAdd(&hist[w][vc[i]], 1);
    }
    __syncthreads();
    if (live) {
      uint32_t m = 0;                                          // lane l < words: word l of the mask
      for (int round = 0; round < r; ++round) {
        float best = neg_inf();
        int bj = 0x7fffffff;
        for (int j = l; j < k2; j += 64) {
          const int tf = hist[w][j];
          if (tf <= 0) continue;
          const float sc = (float)tf * logf(n / (1.0f + (float)df[j]));
          if (sc > best || (sc == best && j < bj)) { best = sc; bj = j; }
        }
        // wave arg-max: larger score, then smaller cluster
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          const float ob = __shfl_xor(best, o);
          const int oj = __shfl_xor(bj, o);
          if (ob > best || (ob == best && oj < bj)) { best = ob; bj = oj; }
        }
        if (bj == 0x7fffffff) break;                           // fewer touched clusters than r
        if (l == (bj >> 5)) m |= 1u << (bj & 31);
        if (l == (bj & 63)) hist[w][bj] = 0;                   // taken
        __builtin_amdgcn_wave_barrier();
      }
      if (l < words) mask[s * words + l] = m;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void member_count_kernel(const uint32_t* __restrict__ mask, int64_t n_sets, int k2,
                                                           int32_t* __restrict__ counts) {
  const int words = (k2 + 31) / 32;
  for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < n_sets; s += (int64_t)gridDim.x * 256)
    for (int wd = 0; wd < words; ++wd) {
      uint32_t m = mask[s * words + wd];
      while (m) {
        const int b = __builtin_ctz(m);
        m &= m - 1;
        atomicAdd(&counts[wd * 32 + b], 1);
      }
    }
}

// Exclusive scan of the k2 (<= 1024) member counts, one workgroup.
__global__ __launch_bounds__(1024) void member_offsets_kernel(const int32_t* __restrict__ counts, int k2,
                                                              int64_t* __restrict__ offs) {
  __shared__ int64_t s[1024];
  const int t = threadIdx.x;
  s[t] = t < k2 ? counts[t] : 0;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t v = t >= o ? s[t - o] : 0;
    __syncthreads();
    s[t] += v;
    __syncthreads();
  }
  if (t < k2) offs[t + 1] = s[t];
  if (t == 0) offs[0] = 0;
}

// One workgroup per cluster: its members in set order (a block scan per
// chunk of 256 sets).
__global__ __launch_bounds__(256) void member_fill_kernel(const uint32_t* __restrict__ mask, int64_t n_sets, int k2,
                                                          const int64_t* __restrict__ offs,
                                                          int32_t* __restrict__ members) {
  __shared__ int scan[256];
  const int words = (k2 + 31) / 32;
  for (int j = blockIdx.x; j < k2; j += gridDim.x) {
    int64_t pos = offs[j];
    for (int64_t s0 = 0; s0 < n_sets; s0 += 256) {
      const int64_t s = s0 + threadIdx.x;
      const int f = (s < n_sets && ((mask[s * words + (j >> 5)] >> (j & 31)) & 1u)) ? 1 : 0;
      scan[threadIdx.x] = f;
      __syncthreads();
      for (int o = 1; o < 256; o <<= 1) {
        const int v = threadIdx.x >= o ? scan[threadIdx.x - o] : 0;
        __syncthreads();
        scan[threadIdx.x] += v;
        __syncthreads();
      }
      if (f) members[pos + scan[threadIdx.x] - 1] = (int32_t)s;
      pos += scan[255];
      __syncthreads();
    }
  }
}

hipError_t launch_set_clusters(const int32_t* vec_clusters, const int64_t* set_off, int64_t n_sets, int k2, int r,
                               uint32_t* mask, int64_t* member_off, int32_t* members, int32_t* ws, hipStream_t s) {
  if (k2 < 1 || k2 > kMaxClusters) return hipErrorInvalidValue;
  int32_t* df = ws;
  int32_t* counts = ws + kMaxClusters;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(256), 0, s, ws, (int64_t)(2 * kMaxClusters), 0);
  const unsigned g = capped_blocks((n_sets + 3) / 4, 256);
  if (n_sets > 0) {
    hipLaunchKernelGGL(set_df_kernel, dim3(g), dim3(256), 0, s, vec_clusters, set_off, n_sets, k2, df);
    hipLaunchKernelGGL(set_top_clusters_kernel, dim3(g), dim3(256), 0, s, vec_clusters, set_off, n_sets, k2, r, df,
                       mask);
    hipLaunchKernelGGL(member_count_kernel, dim3(capped_blocks((n_sets + 255) / 256, 256)), dim3(256), 0, s, mask,
                       n_sets, k2, counts);
  }
  hipLaunchKernelGGL(member_offsets_kernel, dim3(1), dim3(1024), 0, s, counts, k2, member_off);
  hipLaunchKernelGGL(member_fill_kernel, dim3((unsigned)k2), dim3(256), 0, s, mask, n_sets, k2, member_off, members);
  return hipGetLastError();
}

// ------------------------------------------------------------------ cluster filter

// One workgroup per query: S = C Q^T for each query vector (lane j of a wave
// computes <c_j, q> for j = l, l + 64, ...), its top-t centroids (larger,
// then smaller index), their union as the query's mask.
__global__ __launch_bounds__(256) void query_clusters_kernel(const int64_t* __restrict__ q_off,
                                                             const float* __restrict__ q, int64_t n_q,
                                                             const float* __restrict__ C, int k2, int t,
                                                             uint32_t* __restrict__ qmask) {
  __shared__ float qv[4][kDim];
  __shared__ uint32_t m[kMaxClusters / 32];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int words = (k2 + 31) / 32;
  for (int64_t qi = blockIdx.x; qi < n_q; qi += gridDim.x) {
    for (int i = threadIdx.x; i < words; i += 256) m[i] = 0;
    __syncthreads();
    const int64_t r0 = q_off[qi], r1 = q_off[qi + 1];
    for (int64_t rb = r0; rb < r1; rb += 4) {                 // (uniform trip count across the waves)
      const int64_t row = rb + w;
      const bool live = row < r1;
      if (live) {
        qv[w][2 * l] = q[row * kDim + 2 * l];
        qv[w][2 * l + 1] = q[row * kDim + 2 * l + 1];
      }
      __syncthreads();
      if (live) {
        float sc[kMaxClusters / 64];
#pragma unroll
        for (int i = 0; i < kMaxClusters / 64; ++i) {
          const int j = l + 64 * i;
          float a = neg_inf();
          if (j < k2) {
            a = 0.0f;
            for (int d = 0; d < kDim; ++d) a = fmaf(C[(int64_t)j * kDim + d], qv[w][d], a);
          }
          sc[i] = a;
        }
        for (int round = 0; round < t && round < k2; ++round) {
          float best = neg_inf();
          int bj = 0x7fffffff;
#pragma unroll
          for (int i = 0; i < kMaxClusters / 64; ++i) {
            const int j = l + 64 * i;
            if (j < k2 && (sc[i] > best || (sc[i] == best && j < bj))) { best = sc[i]; bj = j; }
          }
#pragma unroll
          for (int o = 32; o > 0; o >>= 1) {
            const float ob = __shfl_xor(best, o);
            const int oj = __shfl_xor(bj, o);
            if (ob > best || (ob == best && oj < bj)) { best = ob; bj = oj; }
          }
          if (bj >= k2) break;
          if (l == (bj & 63)) {
#pragma unroll
            for (int i = 0; i < kMaxClusters / 64; ++i)
              if (i == (bj >> 6)) sc[i] = neg_inf();               // taken (the wave's copy in lane bj % 64)
            atomicOr(&m[bj >> 5], 1u << (bj & 31));
          }
        }
      }
      __syncthreads();
    }
    for (int i = threadIdx.x; i < words; i += 256) qmask[qi * words + i] = m[i];
    __syncthreads();
  }
}

hipError_t launch_query_clusters(const int64_t* q_off, const float* q, int64_t n_q, const float* C, int k2, int t,
                                 uint32_t* qmask, hipStream_t s) {
  if (n_q == 0) return hipSuccess;
  if (k2 < 1 || k2 > kMaxClusters) return hipErrorInvalidValue;
  hipLaunchKernelGGL(query_clusters_kernel, dim3(capped_blocks(n_q, 256)), dim3(256), 0, s, q_off, q, n_q, C, k2, t,
                     qmask);
  return hipGetLastError();
}

// ------------------------------------------------------------------ search steps

// One wave per query: one entry per cluster of C_query (member
// floor(u * count / 2^32) for the caller's random word u), each set once
// (the visited map decides), in cluster order; the rest of the row is padding.
__global__ __launch_bounds__(256) void search_entries_kernel(SearchView S, int64_t n_q, const uint32_t* __restrict__ u,
                                                             int32_t* __restrict__ cand, int32_t stride) {
  const int l = threadIdx.x & 63;
  const int words = (S.k2 + 31) / 32;
  for (int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); q < n_q; q += (int64_t)gridDim.x * 4) {
    int pos = 0;
    for (int j0 = 0; j0 < S.k2; j0 += 64) {
      const int j = j0 + l;
      int pick = -1;
      if (j < S.k2 && ((S.qmask[q * words + (j >> 5)] >> (j & 31)) & 1u)) {
        const int64_t a = S.member_off[j], cnt = S.member_off[j + 1] - a;
        if (cnt > 0) {
          const int64_t k = (int64_t)(((uint64_t)u[q * S.k2 + j] * (uint64_t)cnt) >> 32);   // < cnt
          pick = S.members[a + k];
          const uint32_t bit = 1u << (pick & 31);
          const uint32_t old = atomicOr(&S.visited[q * S.bitmap_words + (pick >> 5)], bit);
          if (old & bit) pick = -1;                              // already an entry
        }
      }
      const uint64_t keep = __ballot(pick >= 0);
      const int before = __popcll(keep & ((1ull << l) - 1));
      if (pick >= 0) cand[q * stride + pos + before] = pick;
      pos += __popcll(keep);
    }
    for (int i = pos + l; i < stride; i += 64) cand[q * stride + i] = -1;
  }
}

// One wave per query, one step of the search:
// - select: the first w entries of R (sorted, padding at the end) that are
//   not expanded become the frontier and are marked expanded; lane f keeps
//   frontier entry f (w <= 64), which is also written to S.frontier;
// - expand: the neighbours of the frontier (lists in order) that share a
//   cluster with C_query and were not visited (marked now), compacted into
//   the query's candidate row; the rest is padding.
__global__ __launch_bounds__(256) void search_step_kernel(SearchView S, int64_t n_q, const int32_t* __restrict__ beam_ids,
                                                          int32_t ef, int32_t* __restrict__ cand, int32_t stride) {
  const int l = threadIdx.x & 63;
  const int words = (S.k2 + 31) / 32;
  for (int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); q < n_q; q += (int64_t)gridDim.x * 4) {
    int taken = 0;
    int fr = -1;                                                 // lane f: frontier entry f
    for (int e0 = 0; e0 < ef && taken < S.width; e0 += 64) {
      const int e = e0 + l;
      const int id = e < ef ? beam_ids[q * ef + e] : -1;
      const bool open = id >= 0 && !((S.expanded[q * S.bitmap_words + (id >> 5)] >> (id & 31)) & 1u);
      const uint64_t bal = __ballot(open);
      const int rank = taken + __popcll(bal & ((1ull << l) - 1));
      if (open && rank < S.width) {
        S.frontier[q * S.width + rank] = id;
        atomicOr(&S.expanded[q * S.bitmap_words + (id >> 5)], 1u << (id & 31));
      }
      // the entries taken here move to lanes taken, taken + 1, ... in order
      uint64_t rest = bal;
      for (int f = taken; f < S.width && rest != 0; ++f) {
        const int src = __builtin_ctzll(rest);
        rest &= rest - 1;
        const int v = __builtin_amdgcn_readlane(id, src);
        if (l == f) fr = v;
      }
      taken += __popcll(bal);
      if (__ballot(id < 0 && e < ef)) break;                     // reached the padding
    }
    taken = min(taken, S.width);
    for (int i = taken + l; i < S.width; i += 64) S.frontier[q * S.width + i] = -1;
    if (l == 0 && taken > 0) atomicAdd(S.active, 1u);
    int pos = 0;
    for (int f = 0; f < taken; ++f) {
      const int p = __builtin_amdgcn_readlane(fr, f);
      for (int d0 = 0; d0 < S.degree; d0 += 64) {
        const int d = d0 + l;
        int nb = d < S.degree ? S.neighbors[(int64_t)p * S.degree + d] : -1;
        if (nb >= 0) {
          bool share = false;
          for (int i = 0; i < words; ++i)
            share |= (S.set_mask[(int64_t)nb * words + i] & S.qmask[q * words + i]) != 0u;
          if (!share) nb = -1;
        }
        if (nb >= 0) {
          const uint32_t bit = 1u << (nb & 31);
          const uint32_t old = atomicOr(&S.visited[q * S.bitmap_words + (nb >> 5)], bit);
          if (old & bit) nb = -1;
        }
        const uint64_t keep = __ballot(nb >= 0);
        const int before = __popcll(keep & ((1ull << l) - 1));
        if (nb >= 0) cand[q * stride + pos + before] = nb;
        pos += __popcll(keep);
      }
    }
    for (int i = pos + l; i < stride; i += 64) cand[q * stride + i] = -1;
  }
}

hipError_t launch_search_clear(const SearchView& S, int64_t n_q, hipStream_t s) {
  const int64_t n = n_q * S.bitmap_words;
  if (n > 0) {
    hipLaunchKernelGGL(fill_u32_kernel, dim3(capped_blocks((n + 255) / 256, 256)), dim3(256), 0, s, S.visited, n, 0u);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(capped_blocks((n + 255) / 256, 256)), dim3(256), 0, s, S.expanded, n, 0u);
  }
  return hipGetLastError();
}

hipError_t launch_search_entries(const SearchView& S, int64_t n_q, const uint32_t* u, int32_t* cand, int32_t stride,
                                 hipStream_t s) {
  if (n_q == 0) return hipSuccess;
  hipLaunchKernelGGL(search_entries_kernel, dim3(capped_blocks((n_q + 3) / 4, 256)), dim3(256), 0, s, S, n_q, u, cand,
                     stride);
  return hipGetLastError();
}

hipError_t launch_search_step(const SearchView& S, int64_t n_q, const int32_t* beam_ids, int32_t ef, int32_t* cand,
                              int32_t stride, hipStream_t s) {
  hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(256), 0, s, S.active, (int64_t)1, 0u);
  if (n_q == 0) return hipGetLastError();
  hipLaunchKernelGGL(search_step_kernel, dim3(capped_blocks((n_q + 3) / 4, 256)), dim3(256), 0, s, S, n_q, beam_ids,
                     ef, cand, stride);
  return hipGetLastError();
}

}  // namespace gem
