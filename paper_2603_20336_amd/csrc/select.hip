// Selection kernels: segmented top-k (the k-argmax of the retrieval problem,
// GEM Sec. 3.1) and the bounded result-set update of beam search (the set R of
// Alg. 5: insert the scored neighbours, keep at most ef, evict the worst).
//
// Entries are ranked by a 64-bit key: the score's order-preserving bits above
// the complemented id, so a larger key is a higher score or, on equal scores,
// a smaller id. A repeated id keeps its best entry; identical (score, id)
// copies have identical keys.
#include <algorithm>

#include "device_common.hpp"
#include "gem_internal.h"

namespace gem {

constexpr int kSelThreads = 512;
constexpr int kSelCap = 4096;     // entries a workgroup can hold in LDS
constexpr int kSelUnroll = 8;     // score loads in flight per thread in the radix passes
constexpr int kSelVec = 4;        // 16-byte score loads in flight per thread in the sampled collect pass
constexpr int kTopkSample = 2048; // entries sampled for the threshold of a long positional segment

__device__ __forceinline__ uint64_t rank_key(float s, int32_t id) {
  return ((uint64_t)float_order_key(s) << 32) | (uint64_t)(~(uint32_t)id);
}
__device__ __forceinline__ int32_t key_id(uint64_t k) { return (int32_t)(~(uint32_t)k); }
__device__ __forceinline__ float key_score(uint64_t k) { return float_from_order_key((uint32_t)(k >> 32)); }
// Same entry keyed by id first (ascending), best score first among equal ids.
__device__ __forceinline__ uint64_t id_key(uint64_t k) {
  return ((uint64_t)(uint32_t)key_id(k) << 32) | (uint64_t)(~(uint32_t)(k >> 32));
}
__device__ __forceinline__ uint64_t rank_from_id_key(uint64_t ik) {
  return ((uint64_t)(~(uint32_t)ik) << 32) | (uint64_t)(~(uint32_t)(ik >> 32));
}

// One compare-exchange stage of merge k with partner distance j over
// a[0..n): n / 2 pairs, thread t takes pairs t, t + T, ... (pair p is
// elements i = 2 j (p / j) + p % j and i + j).
__device__ __forceinline__ void bitonic_stage(uint64_t* a, int half, int k, int j, bool desc) {
  for (int p = threadIdx.x; p < half; p += blockDim.x) {
    const int i = ((p & ~(j - 1)) << 1) | (p & (j - 1));
    const int ixj = i + j;
    const uint64_t x = a[i], y = a[ixj];
    const bool up = ((i & k) == 0) != desc;             // this pair ascending?
    if ((x > y) == up) { a[i] = y; a[ixj] = x; }
  }
}

// Bitonic sort with the stages of partner distance below E in registers:
// thread t holds elements [t E, t E + E) (t < n / E), so those stages pair
// only its own elements. The merges k <= E run wholly in registers; every
// later merge runs its stages j >= E through LDS, one pass each, then its
// last log2(E) stages in registers (for k > E the direction is the same over
// a thread's E elements). The same network as stage by stage, with one LDS
// pass for the last log2(E) stages of each merge.
template <int E>
__device__ void bitonic_sort_regs(uint64_t* a, int n, bool desc) {
  const int half = n >> 1;
  const bool owner = (int)threadIdx.x < n / E;
  const int i0 = (int)threadIdx.x * E;
  uint64_t v[E];
  auto cx = [&](int e, int j, bool up) {
    const uint64_t x = v[e], y = v[e + j];
    if ((x > y) == up) { v[e] = y; v[e + j] = x; }
  };
  if (owner) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = a[i0 + e];
#pragma unroll
    for (int k = 2; k <= E; k <<= 1)
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
        for (int e = 0; e < E; ++e)
          if ((e & j) == 0) cx(e, j, (((i0 | e) & k) == 0) != desc);
#pragma unroll
    for (int e = 0; e < E; ++e) a[i0 + e] = v[e];
  }
  __syncthreads();
  for (int k = 2 * E; k <= n; k <<= 1) {
    for (int j = k >> 1; j >= E; j >>= 1) {
      bitonic_stage(a, half, k, j, desc);
      __syncthreads();
    }
    if (owner) {
      const bool up = ((i0 & k) == 0) != desc;
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = a[i0 + e];
#pragma unroll
      for (int j = E >> 1; j > 0; j >>= 1)
#pragma unroll
        for (int e = 0; e < E; ++e)
          if ((e & j) == 0) cx(e, j, up);
#pragma unroll
      for (int e = 0; e < E; ++e) a[i0 + e] = v[e];
    }
    __syncthreads();
  }
}

// Bitonic sort of a[0..n) (n a power of two), descending if `desc`; every
// thread of the block takes part, and a[] is published at the end.
__device__ void block_bitonic_sort(uint64_t* a, int n, bool desc) {
  if (n < 2) return;
  const int per = n / (int)blockDim.x;                  // elements per thread
  if (per <= 2) bitonic_sort_regs<2>(a, n, desc);
  else if (per == 4) bitonic_sort_regs<4>(a, n, desc);
  else if (per == 8) bitonic_sort_regs<8>(a, n, desc);
  else {
    for (int k = 2; k <= n; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) {
        bitonic_stage(a, n >> 1, k, j, desc);
        __syncthreads();
      }
  }
}

__device__ __forceinline__ int pow2_ceil(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// keys[0..n): rank keys (0 = empty). Removes repeated ids (keeping the best
// entry of each), then sorts descending. Returns the number of distinct entries.
template <int kCap, int kThreads>
__device__ int dedup_and_sort(uint64_t* keys, int n, bool may_repeat, int* s_cnt) {
  const int np = pow2_ceil(max(n, 1));
  if (may_repeat) {
    for (int i = threadIdx.x; i < np; i += blockDim.x) keys[i] = (i < n && keys[i]) ? id_key(keys[i]) : ~0ull;
    __syncthreads();
    block_bitonic_sort(keys, np, false);
    // after the ascending id sort, copies of an id are adjacent, best first
    uint64_t keep_key[kCap / kThreads];
    int c = 0;
    for (int i = threadIdx.x; i < np; i += blockDim.x, ++c) {
      const uint64_t ik = keys[i];
      bool keep = ik != ~0ull;
      if (keep && i > 0 && (uint32_t)(keys[i - 1] >> 32) == (uint32_t)(ik >> 32)) keep = false;
      keep_key[c] = keep ? rank_from_id_key(ik) : 0ull;
    }
    __syncthreads();
    c = 0;
    for (int i = threadIdx.x; i < np; i += blockDim.x, ++c) keys[i] = keep_key[c];
    __syncthreads();
  } else {
    for (int i = threadIdx.x + n; i < np; i += blockDim.x) keys[i] = 0ull;
    __syncthreads();
  }
  block_bitonic_sort(keys, np, true);
  if (threadIdx.x == 0) *s_cnt = 0;
  __syncthreads();
  int c = 0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) c += keys[i] != 0ull;
  atomicAdd(s_cnt, c);
  __syncthreads();
  const int d = *s_cnt;
  __syncthreads();
  return d;
}

struct SegAccess {
  const float* sc;
  const int32_t* ids;
  int64_t n;
  __device__ __forceinline__ int32_t id(int64_t j) const { return ids ? ids[j] : (int32_t)j; }
};

// Histogram add with one atomic per wave when all active lanes hit one bin.
__device__ __forceinline__ void hist_add(uint32_t* hist, bool active, uint32_t bin) {
  const uint64_t act = __ballot(active);
  if (act == 0) return;
  const uint32_t first = __builtin_amdgcn_readfirstlane(active ? bin : 0xffffffffu);
  const uint64_t same = __ballot(active && bin == first);
  if (same == act) {
    if (lane_id() == __ffsll((unsigned long long)act) - 1) atomicAdd(&hist[first], (uint32_t)__popcll(act));
  } else if (active) {
    atomicAdd(&hist[bin], 1u);
  }
}

__global__ __launch_bounds__(kSelThreads, 8) void topk_kernel(TopkSegs S, int32_t k, float* __restrict__ top_scores,
                                                          int32_t* __restrict__ top_ids) {
  __shared__ uint64_t keys[kSelCap];
  __shared__ uint32_t hist[256];
  __shared__ uint32_t suf[257];
  __shared__ int s_cnt;
  __shared__ uint32_t s_sel, s_gt;

  for (int64_t seg = blockIdx.x; seg < S.n_segs; seg += gridDim.x) {
  __syncthreads();                                   // LDS reuse across segments
  SegAccess A;
  if (S.off) {
    const int64_t a = S.off[seg], b = S.off[seg + 1];
    A.sc = S.scores + a;
    A.ids = S.ids ? S.ids + a : nullptr;
    A.n = b - a;
  } else {
    const int64_t row = S.rows ? (int64_t)S.rows[seg] : seg;
    A.sc = S.scores + row * S.ld;
    A.ids = S.ids ? S.ids + row * S.ld : nullptr;
    A.n = S.len;
  }
  const bool may_repeat = A.ids != nullptr;
  const int tid = threadIdx.x;

  int n_keys = 0;
  if (A.n <= kSelCap) {
    // whole segment fits: take every valid entry
    if (tid == 0) s_cnt = 0;
    __syncthreads();
    for (int64_t j = tid; j < A.n; j += kSelThreads) {
      const int32_t id = A.id(j);
      if (id >= 0) keys[atomicAdd(&s_cnt, 1)] = rank_key(A.sc[j], id);
    }
    __syncthreads();
    n_keys = s_cnt;
    __syncthreads();
    n_keys = dedup_and_sort<kSelCap, kSelThreads>(keys, n_keys, may_repeat, &s_cnt);
  } else if (may_repeat) {
    // ids may repeat: stream the segment through LDS in chunks, keeping the
    // best k distinct ids seen so far (an entry dropped here is beaten by k
    // distinct ids whose kept entries can only improve later)
    const int step = kSelCap - k;
    int cur = 0;
    for (int64_t c0 = 0; c0 < A.n; c0 += step) {
      const int64_t c1 = min(A.n, c0 + (int64_t)step);
      if (tid == 0) s_cnt = cur;
      __syncthreads();
      for (int64_t j = c0 + tid; j < c1; j += kSelThreads) {
        const int32_t id = A.id(j);
        if (id >= 0) keys[atomicAdd(&s_cnt, 1)] = rank_key(A.sc[j], id);
      }
      __syncthreads();
      const int n = s_cnt;
      __syncthreads();
      cur = min(dedup_and_sort<kSelCap, kSelThreads>(keys, n, true, &s_cnt), (int)k);
    }
    n_keys = cur;
  } else {
    // positions as ids (all distinct). First a sampled threshold: the r-th
    // best of kSample evenly spaced entries, r a wide margin above the
    // sample's expected share of the top k; every entry at least as good is
    // collected in one pass, and when that is between k and kSelCap entries
    // the top k are among them (keys are distinct), so one sort finishes.
    // Otherwise (heavy ties, skewed orders) the radix select below.
    bool done = false;
    if (k <= kSelCap / 4) {
      const int64_t stride = A.n / kTopkSample;                  // >= 1: A.n > kSelCap
      for (int i = tid; i < kTopkSample; i += kSelThreads)
        keys[i] = rank_key(A.sc[i * stride], (int32_t)(i * stride));
      __syncthreads();
      block_bitonic_sort(keys, kTopkSample, true);
      const int r = (int)min<int64_t>(kTopkSample - 1, (3 * (int64_t)k * kTopkSample) / (2 * A.n) + 16);
      const uint64_t thr = keys[r];
      __syncthreads();
      if (tid == 0) s_cnt = 0;
      __syncthreads();
      auto take = [&](float x, int64_t j) {
        const uint64_t key = rank_key(x, (int32_t)j);
        if (key >= thr) {
          const int pos = atomicAdd(&s_cnt, 1);
          if (pos < kSelCap) keys[pos] = key;
        }
      };
      // 16-byte loads: the entries before the segment's first 16-byte
      // boundary and after its last whole float4 one by one
      const int64_t head = min<int64_t>(A.n, (int64_t)(((16u - ((uint32_t)reinterpret_cast<uintptr_t>(A.sc) & 15u)) & 15u) >> 2));
      const int64_t nv = (A.n - head) >> 2;
      const float4* sc4 = reinterpret_cast<const float4*>(A.sc + head);
      if (tid < head) take(A.sc[tid], tid);
      for (int64_t i0 = 0; i0 < nv; i0 += (int64_t)kSelThreads * kSelVec) {
        float4 v[kSelVec];
#pragma unroll
        for (int u = 0; u < kSelVec; ++u) {
          const int64_t i = i0 + u * kSelThreads + tid;
          v[u] = i < nv ? sc4[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < kSelVec; ++u) {
          const int64_t i = i0 + u * kSelThreads + tid;
          if (i >= nv) continue;
          const int64_t j = head + 4 * i;
          take(v[u].x, j);
          take(v[u].y, j + 1);
          take(v[u].z, j + 2);
          take(v[u].w, j + 3);
        }
      }
      const int64_t tail = head + 4 * nv;
      if (tail + tid < A.n) take(A.sc[tail + tid], tail + tid);
      __syncthreads();
      const int got = s_cnt;
      __syncthreads();
      if (got >= k && got <= kSelCap) {
        n_keys = dedup_and_sort<kSelCap, kSelThreads>(keys, got, false, &s_cnt);
        done = true;
      }
    }
    if (!done) {
      // positions as ids (all distinct): radix select of the k-th largest key,
      // 8 bits a pass, stopping as soon as the threshold bucket holds exactly
      // the entries still needed
      uint64_t prefix = 0, mask = 0;
      int need = k;
      bool exact = false, take_all = false;
      for (int shift = 56; shift >= 0; shift -= 8) {
        for (int i = tid; i < 256; i += kSelThreads) hist[i] = 0;
        __syncthreads();
        // kSelUnroll loads in flight per thread before their histogram adds
        for (int64_t j0 = 0; j0 < A.n; j0 += (int64_t)kSelThreads * kSelUnroll) {
          float v[kSelUnroll];
#pragma unroll
          for (int u = 0; u < kSelUnroll; ++u) {
            const int64_t j = j0 + u * kSelThreads + tid;
            v[u] = j < A.n ? A.sc[j] : 0.0f;
          }
#pragma unroll
          for (int u = 0; u < kSelUnroll; ++u) {
            const int64_t j = j0 + u * kSelThreads + tid;
            bool act = false;
            uint32_t bin = 0;
            if (j < A.n) {
              const uint64_t key = rank_key(v[u], (int32_t)j);
              if ((key & mask) == prefix) { act = true; bin = (uint32_t)(key >> shift) & 0xffu; }
            }
            hist_add(hist, act, bin);
          }
        }
        __syncthreads();
        if (tid < 256) suf[tid] = hist[tid];
        if (tid == 0) suf[256] = 0;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {          // suffix sums
          uint32_t v = (tid < 256 && tid + o < 256) ? suf[tid + o] : 0;
          __syncthreads();
          if (tid < 256) suf[tid] += v;
          __syncthreads();
        }
        if (shift == 56 && suf[0] <= (uint32_t)k) { take_all = true; break; }
        if (tid < 256 && suf[tid] >= (uint32_t)need && suf[tid + 1] < (uint32_t)need) { s_sel = tid; s_gt = suf[tid + 1]; }
        __syncthreads();
        const uint32_t sel = s_sel;
        need -= (int)s_gt;
        prefix |= (uint64_t)sel << shift;
        mask |= 0xffull << shift;
        const bool ex = hist[sel] == (uint32_t)need;
        __syncthreads();
        if (ex) { exact = true; break; }
      }
      // collect the keys above the threshold and the threshold's share (keys are
      // distinct, so a full-width threshold is a single key)
      if (tid == 0) s_cnt = 0;
      __syncthreads();
      for (int64_t j0 = 0; j0 < A.n; j0 += (int64_t)kSelThreads * kSelUnroll) {
        float v[kSelUnroll];
#pragma unroll
        for (int u = 0; u < kSelUnroll; ++u) {
          const int64_t j = j0 + u * kSelThreads + tid;
          v[u] = j < A.n ? A.sc[j] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kSelUnroll; ++u) {
          const int64_t j = j0 + u * kSelThreads + tid;
          if (j >= A.n) continue;
          const uint64_t key = rank_key(v[u], (int32_t)j);
          const bool take = take_all || (key & mask) > prefix || (exact && (key & mask) == prefix) ||
                            (!exact && key == prefix);
          if (take) {
            const int pos = atomicAdd(&s_cnt, 1);
            if (pos < kSelCap) keys[pos] = key;
          }
        }
      }
      __syncthreads();
      const int got = min(s_cnt, kSelCap);
      __syncthreads();
      n_keys = dedup_and_sort<kSelCap, kSelThreads>(keys, got, false, &s_cnt);
    }
  }
  for (int r = tid; r < k; r += kSelThreads) {
    const uint64_t key = r < n_keys ? keys[r] : 0ull;
    top_scores[seg * k + r] = key ? key_score(key) : neg_inf();
    top_ids[seg * k + r] = key ? key_id(key) : -1;
  }
  }
}

hipError_t launch_topk(const TopkSegs& segs, int32_t k, float* top_scores, int32_t* top_ids, hipStream_t s) {
  if (segs.n_segs == 0 || k == 0) return hipSuccess;
  hipLaunchKernelGGL(topk_kernel, dim3(capped_blocks(segs.n_segs, kSelThreads)), dim3(kSelThreads), 0, s, segs, k,
                     top_scores, top_ids);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Merge of the fused top-k's regions (one workgroup per query): the region
// keys stream through LDS; whenever the buffer is full it is sorted and cut to
// the best k (a key dropped there is beaten by k others), and the final sort
// gives the query's top-k. Keys are distinct within a query, so this is the
// top-k of the whole score row, written as topk_kernel writes it.
__global__ __launch_bounds__(kSelThreads, 8) void topk_regions_kernel(const uint64_t* __restrict__ keys,
                                                                  const int32_t* __restrict__ cnt, int64_t n_q,
                                                                  int32_t regions, int32_t cap, int32_t k,
                                                                  float* __restrict__ top_scores,
                                                                  int32_t* __restrict__ top_ids) {
  __shared__ uint64_t buf[kSelCap];
  __shared__ int s_cnt;
  const int tid = threadIdx.x;
  for (int64_t q = blockIdx.x; q < n_q; q += gridDim.x) {
    __syncthreads();                                   // LDS reuse across queries
    int fill = 0;
    for (int r = 0; r < regions; ++r) {
      const int n_r = cnt[q * regions + r];
      const uint64_t* src = keys + (q * regions + r) * (int64_t)cap;
      for (int e0 = 0; e0 < n_r;) {
        const int take = min(n_r - e0, kSelCap - fill);
        for (int i = tid; i < take; i += kSelThreads) buf[fill + i] = src[e0 + i];
        fill += take;
        e0 += take;
        if (fill == kSelCap) {
          __syncthreads();
          fill = min(dedup_and_sort<kSelCap, kSelThreads>(buf, fill, false, &s_cnt), (int)k);
        }
      }
    }
    __syncthreads();
    const int n_keys = dedup_and_sort<kSelCap, kSelThreads>(buf, fill, false, &s_cnt);
    for (int r = tid; r < k; r += kSelThreads) {
      const uint64_t key = r < n_keys ? buf[r] : 0ull;
      top_scores[q * k + r] = key ? key_score(key) : neg_inf();
      top_ids[q * k + r] = key ? key_id(key) : -1;
    }
  }
}

hipError_t launch_topk_regions(const uint64_t* keys, const int32_t* cnt, int64_t n_q, int32_t regions, int32_t cap,
                               int32_t k, float* top_scores, int32_t* top_ids, hipStream_t s) {
  if (n_q == 0 || k == 0) return hipSuccess;
  if (k > kSelCap / 2 || regions < 1 || cap < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(topk_regions_kernel, dim3(capped_blocks(n_q, kSelThreads)), dim3(kSelThreads), 0, s, keys, cnt,
                     n_q, regions, cap, k, top_scores, top_ids);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Beam update: row q of the beam becomes the best ef of (row q) U (list q's
// scored entries), ids distinct. One workgroup per query.
// Slot of an id in the merge's hash table of beam positions (Fibonacci hashing).
template <int kSlots>
__device__ __forceinline__ uint32_t beam_hash(int32_t id) {
  static_assert((kSlots & (kSlots - 1)) == 0, "power of two");
  return ((uint32_t)id * 0x9E3779B1u) >> (32 - __builtin_ctz((unsigned)kSlots));
}

// Merge of beam row `q` in its stored form (rank keys strictly descending,
// padding only at the tail, ids distinct; the form this merge and the reset
// leave) with a list of at most kCap / 2 entries, ef <= kCap / 2. Only the
// list is sorted: by id to keep the best entry of each id, then by rank. A
// listed id that the beam holds keeps the better of the two entries (the beam's
// on equal keys). Each survivor's output position is its rank in its own
// sorted run plus the count of entries of the other run ranked above it
// (keys are distinct between the runs), found by binary search. Returns false,
// with nothing written, when the row is not in the stored form; the caller then
// merges by the full sort, which gives the same result on any row.
template <int kCap, int kThreads>
__device__ bool merge_sorted_beam(uint64_t* keys, uint32_t* slots, uint32_t* drop, int* s_int,
                                  const float* __restrict__ cand_scores, const int32_t* __restrict__ cids,
                                  int nl, int ef, float* bs, int32_t* bi) {
  constexpr int kHalf = kCap / 2;
  constexpr int kSlots = kCap;                       // twice the largest beam
  constexpr uint32_t kEmpty = 0xffffffffu;
  constexpr int kPer = kHalf / kThreads;
  uint64_t* bk = keys;                               // the beam's rank keys, [0, ef)
  uint64_t* ck = keys + kHalf;                       // the list's keys, [0, nc)
  const int tid = threadIdx.x;
  const int nc = pow2_ceil(max(nl, 1));
  // s_int: [0] not in stored form, [1] valid beam entries, [2] dropped beam
  // entries, [3] surviving list entries
  if (tid < 4) s_int[tid] = 0;
  for (int r = tid; r < ef; r += kThreads) {
    const int32_t id = bi[r];
    bk[r] = id >= 0 ? rank_key(bs[r], id) : 0ull;
    drop[r] = 0;
  }
  for (int h = tid; h < kSlots; h += kThreads) slots[h] = kEmpty;
  for (int j = tid; j < nc; j += kThreads) {
    const int32_t id = j < nl ? cids[j] : -1;
    ck[j] = id >= 0 ? id_key(rank_key(cand_scores[j], id)) : ~0ull;
  }
  __syncthreads();
  int bad = 0, valid = 0;
  for (int r = tid; r < ef; r += kThreads) {
    const uint64_t k = bk[r];
    if (r + 1 < ef) {
      const uint64_t k2 = bk[r + 1];
      if (k2 != 0ull && (k == 0ull || k2 >= k)) bad = 1;
    }
    if (k == 0ull) continue;
    ++valid;
    const int32_t id = key_id(k);
    uint32_t h = beam_hash<kSlots>(id);
    for (;;) {                                       // at most ef of 2 ef slots are taken: ends
      const uint32_t prev = atomicCAS(&slots[h], kEmpty, (uint32_t)r);
      if (prev == kEmpty) break;
      if (key_id(bk[prev]) == id) { bad = 1; break; }
      h = (h + 1) & (kSlots - 1);
    }
  }
  if (bad) atomicOr(&s_int[0], 1);
  if (valid) atomicAdd(&s_int[1], valid);
  __syncthreads();
  if (s_int[0]) return false;                        // uniform: read after the barrier
  block_bitonic_sort(ck, nc, false);                 // by id, best entry of an id first
  uint64_t kept[kPer];
  int n_kept = 0, n_drop = 0;
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int j = tid + c * kThreads;
    kept[c] = 0ull;
    if (j >= nc) continue;
    const uint64_t ik = ck[j];
    if (ik == ~0ull || (j > 0 && (uint32_t)(ck[j - 1] >> 32) == (uint32_t)(ik >> 32))) continue;
    const uint64_t rk = rank_from_id_key(ik);
    const int32_t id = key_id(rk);
    bool keep = true;
    for (uint32_t h = beam_hash<kSlots>(id);; h = (h + 1) & (kSlots - 1)) {
      const uint32_t p = slots[h];
      if (p == kEmpty) break;
      if (key_id(bk[p]) == id) {                     // one list entry per id: no race on drop[p]
        if (rk > bk[p]) { drop[p] = 1; ++n_drop; } else keep = false;
        break;
      }
    }
    if (keep) { kept[c] = rk; ++n_kept; }
  }
  if (n_drop) atomicAdd(&s_int[2], n_drop);
  if (n_kept) atomicAdd(&s_int[3], n_kept);
  __syncthreads();                                   // every read of the id-sorted list is done
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int j = tid + c * kThreads;
    if (j < nc) ck[j] = kept[c];
  }
  __syncthreads();
  block_bitonic_sort(ck, nc, true);                  // survivors by rank, then the zeros
  const int nb = s_int[1], dropped = s_int[2], ns = s_int[3];
  if (dropped) {
    // inclusive count of dropped beam entries up to each position (rare:
    // a listed id scored above the beam's entry for it)
    for (int off = 1; off < nb; off <<= 1) {
      uint32_t v[kPer];
#pragma unroll
      for (int c = 0; c < kPer; ++c) {
        const int r = tid + c * kThreads;
        v[c] = r < nb ? drop[r] + (r >= off ? drop[r - off] : 0u) : 0u;
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < kPer; ++c) {
        const int r = tid + c * kThreads;
        if (r < nb) drop[r] = v[c];
      }
      __syncthreads();
    }
  }
  // beam entry i (kept): position (i - dropped before i) + (list keys above it)
  for (int i = tid; i < nb; i += kThreads) {
    const uint32_t upto = dropped ? drop[i] : 0u;
    if (dropped && upto != (i > 0 ? drop[i - 1] : 0u)) continue;
    const uint64_t k = bk[i];
    int lo = 0, hi = ns;                             // first list position ranked below k
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (ck[mid] > k) lo = mid + 1; else hi = mid;
    }
    const int pos = i - (int)upto + lo;
    if (pos < ef) { bs[pos] = key_score(k); bi[pos] = key_id(k); }
  }
  // list entry j: position j + (kept beam entries above it)
  for (int j = tid; j < ns; j += kThreads) {
    const uint64_t k = ck[j];
    int lo = 0, hi = nb;                             // first beam position ranked below k
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (bk[mid] > k) lo = mid + 1; else hi = mid;
    }
    const int pos = j + lo - (int)(dropped && lo > 0 ? drop[lo - 1] : 0u);
    if (pos < ef) { bs[pos] = key_score(k); bi[pos] = key_id(k); }
  }
  for (int r = nb - dropped + ns + tid; r < ef; r += kThreads) {
    bs[r] = neg_inf();
    bi[r] = -1;
  }
  return true;
}

// kSorted: rows in the stored form with at most kCap / 2 beam and list
// entries take merge_sorted_beam (which needs kCap * 6 more bytes of LDS).
template <int kCap, int kThreads, bool kSorted>
__global__ __launch_bounds__(kThreads) void beam_merge_kernel(const float* __restrict__ cand_scores, CandsView C,
                                                                 int64_t n_q, int32_t ef,
                                                                 float* __restrict__ beam_scores,
                                                                 int32_t* __restrict__ beam_ids) {
  __shared__ uint64_t keys[kCap];
  __shared__ uint32_t slots[kSorted ? kCap : 1];
  __shared__ uint32_t drop[kSorted ? kCap / 2 : 1];
  __shared__ int s_int[4];
  __shared__ int s_cnt;
  const int tid = threadIdx.x;
  for (int64_t q = blockIdx.x; q < n_q; q += gridDim.x) {
  __syncthreads();                                   // LDS reuse across queries
  int64_t lb, le;
  if (C.off) { lb = C.off[q]; le = C.off[q + 1]; }
  else { lb = q * (int64_t)C.stride; le = lb + C.stride; }
  float* bs = beam_scores + q * ef;
  int32_t* bi = beam_ids + q * ef;
  if (kSorted && ef <= kCap / 2 && le - lb <= kCap / 2) {
    if (merge_sorted_beam<kCap, kThreads>(keys, slots, drop, s_int, cand_scores + lb, C.ids + lb, (int)(le - lb),
                                          ef, bs, bi))
      continue;
    __syncthreads();                                 // the fast path's reads of keys are done
  }
  if (tid == 0) s_cnt = 0;
  __syncthreads();
  for (int r = tid; r < ef; r += kThreads) {
    const int32_t id = bi[r];
    if (id >= 0) {
      const int pos = atomicAdd(&s_cnt, 1);
      if (pos < kCap) keys[pos] = rank_key(bs[r], id);
    }
  }
  for (int64_t e = lb + tid; e < le; e += kThreads) {
    const int32_t id = C.ids[e];
    if (id >= 0) {
      const int pos = atomicAdd(&s_cnt, 1);
      if (pos < kCap) keys[pos] = rank_key(cand_scores[e], id);
    }
  }
  __syncthreads();
  const int n = min(s_cnt, kCap);
  __syncthreads();
  const int d = dedup_and_sort<kCap, kThreads>(keys, n, true, &s_cnt);
  for (int r = tid; r < ef; r += kThreads) {
    const uint64_t key = r < d ? keys[r] : 0ull;
    bs[r] = key ? key_score(key) : neg_inf();
    bi[r] = key ? key_id(key) : -1;
  }
  }
}

hipError_t launch_beam_merge(const float* cand_scores, const CandsView& C, int64_t n_q, int32_t ef,
                             float* beam_scores, int32_t* beam_ids, int32_t max_entries, hipStream_t s) {
  if (n_q == 0) return hipSuccess;
  // merges of at most 2048 entries (ef + the longest list, when known) run
  // in half the LDS with 256 threads: twice the workgroups per CU
  if (max_entries > 0 && max_entries <= 2048)
    hipLaunchKernelGGL((beam_merge_kernel<2048, 256, true>), dim3(capped_blocks(n_q, 256)), dim3(256), 0, s, cand_scores,
                       C, n_q, ef, beam_scores, beam_ids);
  else
    hipLaunchKernelGGL((beam_merge_kernel<kSelCap, kSelThreads, false>), dim3(capped_blocks(n_q, kSelThreads)),
                       dim3(kSelThreads), 0, s, cand_scores, C, n_q, ef, beam_scores, beam_ids);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void beam_reset_kernel(float* __restrict__ s, int32_t* __restrict__ i, int64_t n) {
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < n; j += (int64_t)gridDim.x * 256) {
    s[j] = neg_inf();
    i[j] = -1;
  }
}

hipError_t launch_beam_reset(float* beam_scores, int32_t* beam_ids, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(beam_reset_kernel, dim3(capped_blocks((n + 255) / 256, 256)), dim3(256), 0, s, beam_scores,
                     beam_ids, n);
  return hipGetLastError();
}

}  // namespace gem
