// Chamfer scoring kernels for gfx950: CH(Q, P) = sum_q max_p <q, p> (GEM, Def. 1).
//
// Both kernels run the inner products on MFMA 16x16 instructions with the
// document vectors as the A operand (rows) and the query vectors as the B
// operand (columns), so that a lane's four accumulators are four document rows
// of one query column: the max over a document's vectors is then mostly
// in-register, and only its last step crosses the four 16-lane groups.
//
// A document of m vectors is covered by ceil(m / 16) row tiles; rows past its
// end re-load its last vector, which leaves the max unchanged (max is
// idempotent), so tiles never straddle documents and need no masking.
//
// The sum over a query's vectors is taken in a fixed order (vector 0, 1, ...),
// so a (query, document) score does not depend on which other queries or
// documents share the launch: the same pair scores bitwise the same in the
// dense and the gathered kernel, alone or in any batch.
#include "device_common.hpp"
#include "gem_internal.h"

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
  static __device__ __forceinline__ f32x4 mma(const Frag& a, const Frag& b, f32x4 acc, int) {
    // OCP E4M3 for both operands (format code 0), E8M0 block scales from each
    // lane's row (A) / column (B); all four 32-wide blocks of a row share it.
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a.v, b.v, acc, 0, 0, 0, a.scale, 0, b.scale);
  }
  static constexpr int kSteps = 1;
};

// Column tiles (16 query vectors each) held in registers by one pass.
template <int DT> struct DenseCfg;
template <> struct DenseCfg<GEM_F32> { static constexpr int kNT = 8; };
template <> struct DenseCfg<GEM_BF16> { static constexpr int kNT = 16; };
template <> struct DenseCfg<GEM_FP8_E4M3> { static constexpr int kNT = 32; };

int dense_pass_rows(int dtype) {
  switch (dtype) {
    case GEM_F32: return 16 * DenseCfg<GEM_F32>::kNT;
    case GEM_BF16: return 16 * DenseCfg<GEM_BF16>::kNT;
    default: return 16 * DenseCfg<GEM_FP8_E4M3>::kNT;
  }
}

int dense_block_rows(int dtype, int max_len) {
  int r = dense_pass_rows(dtype);
  int passes = max_len <= r ? 1 : (max_len + r - 1) / r;
  return r * passes;
}

int64_t dense_blocks_upper(int64_t n_q, int64_t n_rows, int block_rows, int max_len) {
  int64_t win = block_rows - (max_len > 0 ? max_len : 1) + 1;   // >= 1
  return n_rows / win + 2 + n_q / kBlockMaxQueries + 1;
}

// --------------------------------------------------------------------------
// Query-block plan: cut the query batch into runs of whole queries so that a
// run spans at most `block_rows` vectors and at most kBlockMaxQueries queries.
// A run starts at query i when i is a multiple of kBlockMaxQueries or when the
// start row of i falls into a new window of (block_rows - max_len + 1) rows.
__global__ __launch_bounds__(1024) void plan_query_blocks_kernel(const int64_t* __restrict__ q_off, int64_t n_q,
                                                                 int64_t win, int32_t* __restrict__ qb_start,
                                                                 int64_t n_blocks_max) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n_q + 1023) / 1024;
  const int64_t a = t * per, b = min(n_q, a + per);
  const int64_t base = n_q > 0 ? q_off[0] : 0;
  auto starts = [&](int64_t i) -> bool {
    if (i == 0) return true;
    if (i % kBlockMaxQueries == 0) return true;
    return (q_off[i] - base) / win != (q_off[i - 1] - base) / win;
  };
  int64_t cnt = 0;
  for (int64_t i = a; i < b; ++i) cnt += starts(i) ? 1 : 0;
  part[t] = cnt;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {          // inclusive scan
    int64_t v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t pos = part[t] - cnt;
  for (int64_t i = a; i < b; ++i)
    if (starts(i) && pos <= n_blocks_max) qb_start[pos++] = (int32_t)i;
  const int64_t n_blocks = min(part[1023], n_blocks_max);
  for (int64_t j = n_blocks + t; j <= n_blocks_max; j += 1024) qb_start[j] = (int32_t)n_q;
}

hipError_t launch_plan_query_blocks(const int64_t* q_off, int64_t n_q, int block_rows, int max_len,
                                    int32_t* qb_start, int64_t n_blocks_max, hipStream_t s) {
  int64_t win = block_rows - (max_len > 0 ? max_len : 1) + 1;
  hipLaunchKernelGGL(plan_query_blocks_kernel, dim3(1), dim3(1024), 0, s, q_off, n_q, win, qb_start, n_blocks_max);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Dense scorer: every query block against every document of a 64-document
// chunk. A workgroup is four waves = four query blocks on the same chunk, so
// the chunk's tiles are read from HBM once and served to the waves from cache.
// Work items are laid out so that consecutive workgroups on one XCD (dispatch
// is round-robin over the 8 XCDs) share a chunk.
constexpr int kChunkDocs = 64;

struct DenseParams {
  SetsView Q, D;
  const int32_t* qb;
  int64_t n_blocks_max, n_bgroups, n_chunks;
  int block_rows;
  DenseOut out;
};

template <int DT>
__global__ __launch_bounds__(256) void score_dense_kernel(DenseParams P) {
  using O = Op<DT>;
  using Frag = typename O::Frag;
  constexpr int NT = DenseCfg<DT>::kNT;
  constexpr int PASS = 16 * NT;
  __shared__ float lds_cm[4][PASS];
  __shared__ float lds_sc[4][kBlockMaxQueries * kChunkDocs];

  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c16 = l & 15;
  const int64_t total = P.n_bgroups * P.n_chunks;
  const int64_t per = (total + 7) / 8;
  const int64_t item = (int64_t)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (item >= total) return;
  const int64_t chunk = item / P.n_bgroups;
  const int64_t b = (item % P.n_bgroups) * 4 + w;
  if (b >= P.n_blocks_max) return;
  const int q0 = P.qb[b], q1 = P.qb[b + 1];
  if (q0 >= q1) return;
  const int nq = q1 - q0;
  const int64_t p0 = chunk * kChunkDocs;
  const int64_t p1 = min(P.D.n_sets, p0 + kChunkDocs);
  const int nd = (int)(p1 - p0);

  const int64_t r0 = P.Q.off[q0];
  const int nrows = (int)(P.Q.off[q1] - r0);
  // lane j < nq: query j of the block (first column, length)
  int qcs = 0, qlen = 0;
  if (l < nq) {
    int64_t a = P.Q.off[q0 + l], e = P.Q.off[q0 + l + 1];
    qcs = (int)(a - r0);
    qlen = (int)(e - a);
  }
  // lane j <= nd: offset of document p0 + j (lane 64 does not exist: use doff_end)
  const int64_t doff_lane = (l <= nd) ? P.D.off[p0 + l] : 0;
  const int64_t doff_end = P.D.off[p1];
  auto doc_start = [&](int dd) -> int64_t {
    if (dd >= 64) return doff_end;
    uint32_t lo = __builtin_amdgcn_readlane((uint32_t)doff_lane, dd);
    uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(doff_lane >> 32), dd);
    return (int64_t)(((uint64_t)hi << 32) | lo);
  };

  float* cm = lds_cm[w];
  float* sc = lds_sc[w];
  const float ninf = neg_inf();

  for (int prow0 = 0; prow0 < nrows; prow0 += PASS) {
    const int pr = min(PASS, nrows - prow0);
    const int nct = (pr + 15) >> 4;
    const bool first = prow0 == 0;
    Frag B[NT];
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) {
      const int col = prow0 + 16 * ct + c16;
      if (ct < nct && col < nrows) O::load(B[ct], P.Q.vecs, P.Q.scales, r0 + col, g);
      else O::zero(B[ct]);
    }

    // empty documents: record their score and move on
    auto skip_empty = [&](int dd) -> int {
      while (dd < nd && doc_start(dd + 1) == doc_start(dd)) {
        if (first && l < nq) sc[l * kChunkDocs + dd] = qlen > 0 ? ninf : 0.0f;
        ++dd;
      }
      return dd;
    };

    int dd = skip_empty(0);
    int t = 0;
    int64_t dbeg = 0, dlen = 0;
    Frag A_next;
    if (dd < nd) {
      dbeg = doc_start(dd);
      dlen = doc_start(dd + 1) - dbeg;
      O::load(A_next, P.D.vecs, P.D.scales, dbeg + min((int64_t)c16, dlen - 1), g);
    }
    float rm[NT];
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) rm[ct] = ninf;

    while (dd < nd) {
      Frag A = A_next;
      // position of the next tile, and its prefetch
      int ndd = dd, nt = t + 1;
      int64_t nbeg = dbeg, nlen = dlen;
      const bool last_tile = (int64_t)nt * 16 >= dlen;
      if (last_tile) {
        ndd = skip_empty(dd + 1);
        nt = 0;
        if (ndd < nd) { nbeg = doc_start(ndd); nlen = doc_start(ndd + 1) - nbeg; }
      }
      if (ndd < nd) O::load(A_next, P.D.vecs, P.D.scales, nbeg + min((int64_t)(nt * 16 + c16), nlen - 1), g);

      f32x4 acc[NT];
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < O::kSteps; ++s) {
#pragma unroll
        for (int ct = 0; ct < NT; ++ct)
          if (ct < nct) acc[ct] = O::mma(A, B[ct], acc[ct], s);
      }
#pragma unroll
      for (int ct = 0; ct < NT; ++ct)
        if (ct < nct) rm[ct] = fmaxf(rm[ct], max4(acc[ct]));

      if (last_tile) {
        // max over the document's rows: finish across the four lane groups
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
          if (ct < nct) {
            float v = max_across_groups(rm[ct]);
            if (l < 16) cm[16 * ct + l] = v;
          }
          rm[ct] = ninf;
        }
        __builtin_amdgcn_wave_barrier();
        // sum over each query's vectors that this pass holds, in vector order
        if (l < nq) {
          float acc_s = first ? 0.0f : sc[l * kChunkDocs + dd];
          const int a0 = max(qcs - prow0, 0), a1 = min(qcs + qlen - prow0, pr);
          for (int a = a0; a < a1; ++a) acc_s += cm[a];
          sc[l * kChunkDocs + dd] = acc_s;
        }
        __builtin_amdgcn_wave_barrier();
      }
      dd = ndd; t = nt; dbeg = nbeg; dlen = nlen;
    }
  }
  if (nrows == 0) {                    // only empty queries: every score is 0
    for (int j = 0; j < nq; ++j)
      if (l < nd) sc[j * kChunkDocs + l] = 0.0f;
  }
  __builtin_amdgcn_wave_barrier();
  // write the chunk's scores, one 64-document row segment per query
  for (int j = 0; j < nq; ++j) {
    if (l < nd) {
      const int64_t row = P.out.rows ? (int64_t)P.out.rows[q0 + j] : (int64_t)(q0 + j);
      P.out.scores[row * P.out.ld + p0 + l] = sc[j * kChunkDocs + l];
    }
  }
}

hipError_t launch_score_dense(int dtype, const SetsView& Q, const SetsView& D, const int32_t* qb_start,
                              int64_t n_blocks_max, int block_rows, const DenseOut& out, hipStream_t s) {
  DenseParams P;
  P.Q = Q; P.D = D; P.qb = qb_start; P.n_blocks_max = n_blocks_max;
  P.n_bgroups = (n_blocks_max + 3) / 4;
  P.n_chunks = (D.n_sets + kChunkDocs - 1) / kChunkDocs;
  P.block_rows = block_rows;
  P.out = out;
  const int64_t total = P.n_bgroups * P.n_chunks;
  if (total == 0) return hipSuccess;
  const int64_t grid = ((total + 7) / 8) * 8;
  switch (dtype) {
    case GEM_F32: hipLaunchKernelGGL(score_dense_kernel<GEM_F32>, dim3((unsigned)grid), dim3(256), 0, s, P); break;
    case GEM_BF16: hipLaunchKernelGGL(score_dense_kernel<GEM_BF16>, dim3((unsigned)grid), dim3(256), 0, s, P); break;
    case GEM_FP8_E4M3: hipLaunchKernelGGL(score_dense_kernel<GEM_FP8_E4M3>, dim3((unsigned)grid), dim3(256), 0, s, P); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Gathered scorer: one wave scores up to kGatherEntries consecutive entries of
// one query's candidate list. The query's vectors stay in registers (64 per
// pass); each candidate document is streamed tile by tile, the next tile's
// load in flight while the current one is multiplied.
constexpr int kGatherEntries = 16;
constexpr int kGatherNT = 4;

struct GatherParams {
  SetsView Q, D;
  CandsView C;
  int64_t chunks_per_query;
  float* scores;
};

template <int DT>
__global__ __launch_bounds__(256) void score_gather_kernel(GatherParams P) {
  using O = Op<DT>;
  using Frag = typename O::Frag;
  constexpr int NT = kGatherNT;
  constexpr int PASS = 16 * NT;
  __shared__ float lds_cm[4][PASS];
  __shared__ float lds_sc[4][kGatherEntries];

  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c16 = l & 15;
  const int64_t gw = (int64_t)blockIdx.x * 4 + w;
  const int64_t q = gw / P.chunks_per_query;
  if (q >= P.C.n_lists) return;
  const int64_t ch = gw % P.chunks_per_query;
  int64_t lb, le;
  if (P.C.off) { lb = P.C.off[q]; le = P.C.off[q + 1]; }
  else { lb = q * (int64_t)P.C.stride; le = lb + P.C.stride; }
  const int64_t e0 = lb + ch * kGatherEntries;
  const int64_t e1 = min(le, e0 + kGatherEntries);
  if (e0 >= e1) return;
  const int ne = (int)(e1 - e0);
  const float ninf = neg_inf();

  // lane e < ne: the entry's document id and row range
  int32_t my_id = -1;
  int64_t my_beg = 0, my_len = 0;
  if (l < ne) {
    my_id = P.C.ids[e0 + l];
    if (my_id >= 0) { my_beg = P.D.off[my_id]; my_len = P.D.off[my_id + 1] - my_beg; }
  }
  auto rd64 = [&](int64_t v, int e) -> int64_t {
    uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, e);
    uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), e);
    return (int64_t)(((uint64_t)hi << 32) | lo);
  };

  const int64_t r0 = P.Q.off[q];
  const int m = (int)(P.Q.off[q + 1] - r0);
  float* cm = lds_cm[w];
  float* sc = lds_sc[w];

  if (m == 0) {
    if (l < ne) P.scores[e0 + l] = my_id < 0 ? ninf : 0.0f;
    return;
  }
  // entries that score without any tile: padding ids and empty documents
  if (l < ne) sc[l] = (my_id < 0 || my_len == 0) ? ninf : 0.0f;
  __builtin_amdgcn_wave_barrier();

  for (int prow0 = 0; prow0 < m; prow0 += PASS) {
    const int pr = min(PASS, m - prow0);
    const int nct = (pr + 15) >> 4;
    Frag B[NT];
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) {
      const int col = prow0 + 16 * ct + c16;
      if (ct < nct && col < m) O::load(B[ct], P.Q.vecs, P.Q.scales, r0 + col, g);
      else O::zero(B[ct]);
    }
    auto next_entry = [&](int e) -> int {          // next entry with a non-empty document
      while (e < ne && rd64(my_len, e) == 0) ++e;
      return e;
    };
    int e = next_entry(0);
    int t = 0;
    int64_t dbeg = 0, dlen = 0;
    Frag A_next;
    if (e < ne) {
      dbeg = rd64(my_beg, e);
      dlen = rd64(my_len, e);
      O::load(A_next, P.D.vecs, P.D.scales, dbeg + min((int64_t)c16, dlen - 1), g);
    }
    float rm[NT];
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) rm[ct] = ninf;
    while (e < ne) {
      Frag A = A_next;
      int ne_ = e, nt = t + 1;
      int64_t nbeg = dbeg, nlen = dlen;
      const bool last_tile = (int64_t)nt * 16 >= dlen;
      if (last_tile) {
        ne_ = next_entry(e + 1);
        nt = 0;
        if (ne_ < ne) { nbeg = rd64(my_beg, ne_); nlen = rd64(my_len, ne_); }
      }
      if (ne_ < ne) O::load(A_next, P.D.vecs, P.D.scales, nbeg + min((int64_t)(nt * 16 + c16), nlen - 1), g);
      f32x4 acc[NT];
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < O::kSteps; ++s) {
#pragma unroll
        for (int ct = 0; ct < NT; ++ct)
          if (ct < nct) acc[ct] = O::mma(A, B[ct], acc[ct], s);
      }
#pragma unroll
      for (int ct = 0; ct < NT; ++ct)
        if (ct < nct) rm[ct] = fmaxf(rm[ct], max4(acc[ct]));
      if (last_tile) {
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
          if (ct < nct) {
            float v = max_across_groups(rm[ct]);
            if (l < 16) cm[16 * ct + l] = v;
          }
          rm[ct] = ninf;
        }
        __builtin_amdgcn_wave_barrier();
        if (l == 0) {
          float s_ = sc[e];
          for (int a = 0; a < pr; ++a) s_ += cm[a];
          sc[e] = s_;
        }
        __builtin_amdgcn_wave_barrier();
      }
      e = ne_; t = nt; dbeg = nbeg; dlen = nlen;
    }
  }
  __builtin_amdgcn_wave_barrier();
  if (l < ne) P.scores[e0 + l] = sc[l];
}

hipError_t launch_score_gather(int dtype, const SetsView& Q, const SetsView& D, const CandsView& C,
                               int32_t max_list_len, int32_t, float* scores, hipStream_t s) {
  GatherParams P;
  P.Q = Q; P.D = D; P.C = C; P.scores = scores;
  P.chunks_per_query = (max_list_len + kGatherEntries - 1) / kGatherEntries;
  if (P.chunks_per_query == 0 || C.n_lists == 0) return hipSuccess;
  const int64_t waves = P.chunks_per_query * C.n_lists;
  const int64_t grid = (waves + 3) / 4;
  switch (dtype) {
    case GEM_F32: hipLaunchKernelGGL(score_gather_kernel<GEM_F32>, dim3((unsigned)grid), dim3(256), 0, s, P); break;
    case GEM_BF16: hipLaunchKernelGGL(score_gather_kernel<GEM_BF16>, dim3((unsigned)grid), dim3(256), 0, s, P); break;
    case GEM_FP8_E4M3: hipLaunchKernelGGL(score_gather_kernel<GEM_FP8_E4M3>, dim3((unsigned)grid), dim3(256), 0, s, P); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gem
