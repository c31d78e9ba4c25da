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
// The sum over a query's vectors is taken in a fixed order that depends only on
// the query itself (a fixed lane tree inside each 16-vector tile, then the tiles
// in order), so a (query, document) score does not depend on which other
// queries or documents share the launch: the same pair scores bitwise the same
// in the dense and the gathered kernel, alone or in any batch.
#include <algorithm>

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
    // OCP E4M3 for both operands (format code 0), E8M0 block scales from each
    // lane's row (A) / column (B); all four 32-wide blocks of a row share it.
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a.v, b.v, acc, 0, 0, 0, a.scale, 0, b.scale);
  }
  static constexpr int kSteps = 1;
};

// Column tiles (16 query vectors each) held in registers by one pass.
template <int DT> struct DenseCfg;
// kNT: 16-column tiles a wave holds; kGroup: document tiles per LDS group buffer.
template <> struct DenseCfg<GEM_F32> { static constexpr int kNT = 4; static constexpr int kGroup = 4; };
template <> struct DenseCfg<GEM_BF16> { static constexpr int kNT = 8; static constexpr int kGroup = 8; };
template <> struct DenseCfg<GEM_FP8_E4M3> { static constexpr int kNT = 16; static constexpr int kGroup = 8; };

int dense_pass_rows(int dtype) {
  switch (dtype) {
    case GEM_F32: return 16 * DenseCfg<GEM_F32>::kNT;
    case GEM_BF16: return 16 * DenseCfg<GEM_BF16>::kNT;
    default: return 16 * DenseCfg<GEM_FP8_E4M3>::kNT;
  }
}

static int pad16(int m) { return (m + 15) & ~15; }

int dense_block_rows(int dtype, int max_len) {
  const int r = dense_pass_rows(dtype);
  const int m = pad16(max_len);
  return m <= r ? r : ((m + r - 1) / r) * r;
}

int64_t dense_blocks_upper(int64_t n_q, int64_t n_rows, int block_rows, int max_len) {
  // within a segment every run but the last is followed by a query (at most
  // pad16(max_len) columns) that did not fit, so it spans more than
  // block_rows - pad16(max_len) columns
  const int64_t win = block_rows - pad16(max_len > 0 ? max_len : 1) + 1;   // >= 1
  const int64_t cols = n_rows + 15 * n_q;                                   // padded columns, upper bound
  const int64_t bound = cols / win + 1 + (n_q + kBlockMaxQueries - 1) / kBlockMaxQueries;
  return bound < n_q ? bound : n_q;                                         // a run holds a query
}

// --------------------------------------------------------------------------
// Per-document epilogue shared by both scorers.
//
// rm[ct] holds, per lane, the running max over a document's rows 4g..4g+3 of
// each tile for query column (16 ct + l % 16). Four tiles at a time:
// two permlane16 swaps and one permlane32 swap leave tile (4i + r)'s column
// maxima in row r (lanes 16r..16r+15) of R[i], already reduced over the four
// lane groups (for FP8 each column is then multiplied by its query vector's
// scale); four DPP adds inside each 16-lane row then leave that tile's column
// sum T in every lane of the row. Every step pairs fixed lanes, so T
// depends only on the tile's own values.
template <int NT, bool kScaled = false>
__device__ __forceinline__ void tile_sums(const float (&rm)[NT], float (&R)[NT / 4], const float* colscale = nullptr) {
#pragma unroll
  for (int i = 0; i < NT / 4; ++i) {
    auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(rm[4 * i + 0]), __float_as_uint(rm[4 * i + 1]), false, false);
    const float ab = fmaxf(__uint_as_float(p[0]), __uint_as_float(p[1]));       // rows: A01 B01 A23 B23
    auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(rm[4 * i + 2]), __float_as_uint(rm[4 * i + 3]), false, false);
    const float cd = fmaxf(__uint_as_float(q[0]), __uint_as_float(q[1]));       // rows: C01 D01 C23 D23
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(ab), __float_as_uint(cd), false, false);
    float m = fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));             // rows: A B C D
    if constexpr (kScaled) m *= colscale[i];                                    // query vector's scale
    m += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(m), 0xb1, 0xf, 0xf, false));   // lane ^ 1
    m += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(m), 0x4e, 0xf, 0xf, false));   // lane ^ 2
    m += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(m), 0x141, 0xf, 0xf, false));  // half mirror
    m += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(m), 0x140, 0xf, 0xf, false));  // row mirror
    R[i] = m;
  }
}

template <int NT>
__device__ __forceinline__ float tile_sum_at(const float (&R)[NT / 4], int ct) {
  return __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(R[ct >> 2]), 16 * (ct & 3)));
}

__device__ __forceinline__ void update_max(float& rm, f32x4 a) {
  rm = fmaxf(fmaxf(rm, a[0]), a[1]);
  rm = fmaxf(fmaxf(rm, a[2]), a[3]);
}

// --------------------------------------------------------------------------
// Query-block plan. Each query is laid out from a 16-aligned column (its
// columns past the last vector are zero vectors, whose max over any document
// is exactly 0, so they add nothing). The batch is cut into segments of
// kBlockMaxQueries consecutive queries, and each segment greedily into runs of
// whole queries spanning at most `block_cols` padded columns: a run ends when
// the next query would not fit. One thread plans one or more whole segments;
// the runs' first queries go to qb_start in order, the tail up to
// n_blocks_max is filled with n_q, and qb_start[n_blocks_max + 1] receives the
// number of runs.
__global__ __launch_bounds__(1024) void plan_query_blocks_kernel(const int64_t* __restrict__ q_off, int64_t n_q,
                                                                 int64_t block_cols, int32_t* __restrict__ qb_start,
                                                                 int64_t* __restrict__ qcol, int64_t n_blocks_max) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t n_seg = (n_q + kBlockMaxQueries - 1) / kBlockMaxQueries;
  const int64_t per = ((n_seg + 1023) / 1024) * kBlockMaxQueries;      // whole segments per thread
  const int64_t a = min(n_q, t * per), b = min(n_q, a + per);
  auto scan = [&](int64_t v) -> int64_t {         // exclusive block scan; part[t] = total afterwards
    part[t] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      int64_t u = t >= o ? part[t - o] : 0;
      __syncthreads();
      part[t] += u;
      __syncthreads();
    }
    const int64_t incl = part[t];
    const int64_t tot = part[1023];
    __syncthreads();
    part[t] = tot;
    return incl - v;
  };
  auto cols_of = [&](int64_t i) -> int64_t { return (q_off[i + 1] - q_off[i] + 15) & ~(int64_t)15; };
  int64_t cols = 0;
  for (int64_t i = a; i < b; ++i) cols += cols_of(i);
  int64_t c = scan(cols);
  const int64_t total_cols = part[t];
  // greedy runs over this thread's segments (columns are relative, so the
  // scan result is not needed for the cut)
  int64_t cnt = 0;
  {
    int64_t run_cols = 0;
    for (int64_t i = a; i < b; ++i) {
      const int64_t ci = cols_of(i);
      if (i % kBlockMaxQueries == 0 || run_cols + ci > block_cols) { ++cnt; run_cols = 0; }
      run_cols += ci;
    }
  }
  int64_t pos = scan(cnt);
  const int64_t n_blocks = min(part[t], n_blocks_max);
  {
    int64_t run_cols = 0;
    for (int64_t i = a; i < b; ++i) {
      const int64_t ci = cols_of(i);
      qcol[i] = c;
      c += ci;
      if (i % kBlockMaxQueries == 0 || run_cols + ci > block_cols) {
        if (pos < n_blocks_max) qb_start[pos] = (int32_t)i;
        ++pos;
        run_cols = 0;
      }
      run_cols += ci;
    }
  }
  if (t == 0) {
    qcol[n_q] = total_cols;
    qb_start[n_blocks_max + 1] = (int32_t)n_blocks;
  }
  for (int64_t j = n_blocks + t; j <= n_blocks_max; j += 1024) qb_start[j] = (int32_t)n_q;
}

hipError_t launch_plan_query_blocks(const int64_t* q_off, int64_t n_q, int block_rows, int,
                                    int32_t* qb_start, int64_t* qcol, int64_t n_blocks_max, hipStream_t s) {
  hipLaunchKernelGGL(plan_query_blocks_kernel, dim3(1), dim3(1024), 0, s, q_off, n_q, (int64_t)block_rows, qb_start,
                     qcol, n_blocks_max);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Dense scorer: every query block against every document of a 64-document
// chunk. A workgroup is eight waves (two per SIMD, so one wave's MFMAs cover
// the other's epilogue and waits) = eight query blocks on the same chunk.
//
// The chunk's document tiles stream through LDS and are shared by the eight
// waves. They are copied HBM -> LDS by direct-to-LDS loads (no registers), in
// groups of kGroup tiles, kBuffers group buffers deep: while one group is
// multiplied the next two are in flight. The copies rotate over the waves so
// that every wave issues the same number per group. Each wave waits for its own copies
// with an explicit vector-memory count, then one barrier per group publishes
// the group and frees the buffer the next copy overwrites. The loop holds no
// other vector-memory operation and reads LDS only through fixed sequences
// that wait for themselves, so no wait is ever widened to the copies still in
// flight. Inside a tile row the 16-byte chunks are XOR-swizzled by the row
// index, so the 16 lanes reading one chunk of 16 rows hit distinct banks.
//
// Scores stay in registers: at a document's end each finished query's score
// is written into lane (document index) of a per-tile register, and a pass
// ends with one coalesced 64-document row store per query.
// Work items are laid out so that consecutive workgroups on one XCD (dispatch
// is round-robin over the 8 XCDs) share a chunk.
constexpr int kChunkDocs = 64;
constexpr int kBuffers = 3;                    // group buffers: two groups in flight
constexpr int kDenseWaves = 8;                 // two waves per SIMD
constexpr int kDenseThreads = 64 * kDenseWaves;

typedef __attribute__((address_space(3))) void* lds_void_ptr;
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

struct DenseParams {
  SetsView Q, D;
  const int32_t* qb;
  const int64_t* qcol;
  int64_t n_blocks_max, n_bgroups, n_chunks;
  int64_t chunk0;         // first document chunk of this launch (large batches launch in slices)
  DenseOut out;
};

// LDS image of one 16-row tile: row r at r * kRowBytes, chunk c at position c ^ swz(r).
template <int DT> struct TileStage {
  using O = Op<DT>;
  static constexpr int kRowBytes = O::kRowBytes;
  static constexpr int kChunksPerRow = kRowBytes / 16;
  static constexpr int kTileBytes = 16 * kRowBytes;
  static constexpr int kSlots = kTileBytes / 16;                 // 16-byte pieces per tile
  static constexpr int kPieceWaves = kSlots / 64;                // waves copying one piece per lane
  static constexpr bool kScales = DT == GEM_FP8_E4M3;
  static constexpr int kCopyWaves = kPieceWaves + (kScales ? 1 : 0);   // waves busy copying one tile
  static constexpr int kStageBytes = kTileBytes + (kScales ? 64 : 0);
  static constexpr int kGroup = DenseCfg<DT>::kGroup;
  // tile u of a group is copied by waves kCopyWaves*u .. kCopyWaves*u + kCopyWaves-1
  // (mod 8), so over a group every wave issues the same number of copies
  static constexpr int kCopiesPerWave = kGroup * kCopyWaves / kDenseWaves;
  static_assert(kSlots % 64 == 0 && kCopyWaves <= kDenseWaves, "tile copy layout");
  static_assert((kGroup * kCopyWaves) % kDenseWaves == 0, "copies must spread evenly over the waves");

  // chunk c of row r sits at position c ^ swz(r): the 16 rows read by one
  // 16-lane group then cover all 64 banks (128-byte rows pair up first)
  static __device__ __forceinline__ int swz(int r) { return kRowBytes == 128 ? ((r >> 1) & 7) : (r & 15); }
  // global address of piece `slot` of the tile whose rows start at doc row beg
  static __device__ __forceinline__ const void* src(const void* vecs, int64_t beg, int64_t len, int t, int slot) {
    const int r = slot / kChunksPerRow, pos = slot % kChunksPerRow;
    const int c = pos ^ swz(r);
    const int64_t row = beg + min((int64_t)(16 * t + r), len - 1);
    return static_cast<const char*>(vecs) + row * kRowBytes + c * 16;
  }
  // this wave's share of copying tile u of a group into the stage at LDS address `stage`
  static __device__ __forceinline__ void copy(const void* vecs, const float* scales, int64_t beg, int64_t len,
                                              int t, char* stage, int u, int w, int l) {
    const int role = (w - kCopyWaves * u) & (kDenseWaves - 1);
    if (role < kPieceWaves) {
      __builtin_amdgcn_global_load_lds(src(vecs, beg, len, t, 64 * role + l), (lds_void_ptr)(stage + 1024 * role),
                                       16, 0, 0);
    } else if (kScales && role == kPieceWaves) {
      if (l < 16)
        __builtin_amdgcn_global_load_lds(scales + beg + min((int64_t)(16 * t + l), len - 1),
                                         (lds_void_ptr)(stage + kTileBytes), 4, 0, 0);
    }
  }
};

// s_waitcnt with only the vector-memory count set (expcnt / lgkmcnt left open)
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0f70);
}

// A operand of one tile from its LDS stage: the reads and their wait form one
// block, so the compiler never sees an LDS read it would order after the copies.
template <int DT>
__device__ __forceinline__ void frag_from_lds(typename Op<DT>::Frag& f, uint32_t stage, int c16, int g);

template <>
__device__ __forceinline__ void frag_from_lds<GEM_BF16>(Op<GEM_BF16>::Frag& f, uint32_t stage, int c16, int g) {
  const uint32_t row = stage + c16 * 256;
  const uint32_t a0 = row + (((4 * g + 0) ^ (c16 & 15)) << 4), a1 = row + (((4 * g + 1) ^ (c16 & 15)) << 4);
  const uint32_t a2 = row + (((4 * g + 2) ^ (c16 & 15)) << 4), a3 = row + (((4 * g + 3) ^ (c16 & 15)) << 4);
  u32x4 v0, v1, v2, v3;
  asm volatile("ds_read_b128 %0, %4\n\tds_read_b128 %1, %5\n\tds_read_b128 %2, %6\n\tds_read_b128 %3, %7\n\t"
               "s_waitcnt lgkmcnt(0)"
               : "=&v"(v0), "=&v"(v1), "=&v"(v2), "=&v"(v3)
               : "v"(a0), "v"(a1), "v"(a2), "v"(a3)
               : "memory");
  f.v[0] = __builtin_bit_cast(bf16x8, v0);
  f.v[1] = __builtin_bit_cast(bf16x8, v1);
  f.v[2] = __builtin_bit_cast(bf16x8, v2);
  f.v[3] = __builtin_bit_cast(bf16x8, v3);
}

template <>
__device__ __forceinline__ void frag_from_lds<GEM_FP8_E4M3>(Op<GEM_FP8_E4M3>::Frag& f, uint32_t stage, int c16, int g) {
  const uint32_t row = stage + c16 * 128;
  const uint32_t a0 = row + (((2 * g) ^ ((c16 >> 1) & 7)) << 4);
  const uint32_t a1 = row + (((2 * g + 1) ^ ((c16 >> 1) & 7)) << 4);
  const uint32_t as = stage + 16 * 128 + 4 * c16;
  u32x4 v0, v1;
  uint32_t sc;
  asm volatile("ds_read_b128 %0, %3\n\tds_read_b128 %1, %4\n\tds_read_b32 %2, %5\n\ts_waitcnt lgkmcnt(0)"
               : "=&v"(v0), "=&v"(v1), "=&v"(sc)
               : "v"(a0), "v"(a1), "v"(as)
               : "memory");
  f.v = i32x8{(int)v0.x, (int)v0.y, (int)v0.z, (int)v0.w, (int)v1.x, (int)v1.y, (int)v1.z, (int)v1.w};
  f.scale = (int)((sc >> 23) & 0xffu);
}

template <>
__device__ __forceinline__ void frag_from_lds<GEM_F32>(Op<GEM_F32>::Frag& f, uint32_t stage, int c16, int g) {
  const uint32_t row = stage + c16 * 512;
  uint32_t a[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) a[s] = row + (((8 * g + s) ^ (c16 & 15)) << 4);
  u32x4 v0, v1, v2, v3, v4, v5, v6, v7;
  asm volatile("ds_read_b128 %0, %8\n\tds_read_b128 %1, %9\n\tds_read_b128 %2, %10\n\tds_read_b128 %3, %11\n\t"
               "ds_read_b128 %4, %12\n\tds_read_b128 %5, %13\n\tds_read_b128 %6, %14\n\tds_read_b128 %7, %15\n\t"
               "s_waitcnt lgkmcnt(0)"
               : "=&v"(v0), "=&v"(v1), "=&v"(v2), "=&v"(v3), "=&v"(v4), "=&v"(v5), "=&v"(v6), "=&v"(v7)
               : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4]), "v"(a[5]), "v"(a[6]), "v"(a[7])
               : "memory");
  const u32x4 vv[8] = {v0, v1, v2, v3, v4, v5, v6, v7};
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    f.v[4 * s + 0] = __uint_as_float(vv[s].x); f.v[4 * s + 1] = __uint_as_float(vv[s].y);
    f.v[4 * s + 2] = __uint_as_float(vv[s].z); f.v[4 * s + 3] = __uint_as_float(vv[s].w);
  }
}

__device__ __forceinline__ float writelane_f(float old, float v, int lane) {
  return lane_id() == lane ? v : old;
}
__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(v), lane));
}

template <int DT>
__global__ __launch_bounds__(kDenseThreads) void score_dense_kernel(DenseParams P) {
  using O = Op<DT>;
  using Frag = typename O::Frag;
  using TS = TileStage<DT>;
  constexpr int NT = DenseCfg<DT>::kNT;
  constexpr int kGroup = TS::kGroup;
  __shared__ __attribute__((aligned(1024))) char lds_tiles[kBuffers][kGroup][TS::kStageBytes];
  __shared__ int lds_npass[kDenseWaves];

  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, g = l >> 4, c16 = l & 15;
  // the plan's real block count sets the work: items (chunk, block group) with
  // the group fastest, each XCD (workgroups go round-robin over the 8 XCDs)
  // taking one contiguous range, so that the workgroups an XCD runs at once
  // share a chunk; the grid is sized for the upper bound and the rest exit
  const int64_t n_bg = (P.qb[P.n_blocks_max + 1] + kDenseWaves - 1) / kDenseWaves;
  const int64_t total = n_bg * P.n_chunks;
  const int64_t per = (total + 7) / 8;
  const int64_t slot = blockIdx.x >> 3;
  const int64_t item = (int64_t)(blockIdx.x & 7) * per + slot;
  if (slot >= per || item >= total) return;                    // whole workgroup
  const int64_t chunk = P.chunk0 + item / n_bg;
  const int64_t b0 = (item % n_bg) * kDenseWaves;
  const int64_t b = b0 + w;
  int q0 = 0, q1 = 0;
  if (b < P.n_blocks_max) { q0 = P.qb[b]; q1 = P.qb[b + 1]; }
  const int nq = max(q1 - q0, 0);                              // 0: this wave only helps copy
  const int64_t p0 = chunk * kChunkDocs;
  const int64_t p1 = min(P.D.n_sets, p0 + kChunkDocs);
  const int nd = (int)(p1 - p0);
  const float ninf = neg_inf();

  // lane j < nq: query j of the block (first row, length, first tile, tiles)
  int64_t qrow = 0;
  int qm = 0, qt0 = 0, qnt = 0;
  int total_tiles = 0;
  if (nq > 0) {
    const int64_t col0 = P.qcol[q0];
    if (l < nq) {
      qrow = P.Q.off[q0 + l];
      qm = (int)(P.Q.off[q0 + l + 1] - qrow);
      qt0 = (int)((P.qcol[q0 + l] - col0) >> 4);
      qnt = (qm + 15) >> 4;
    }
    total_tiles = (int)((P.qcol[q1] - col0) >> 4);
  }
  total_tiles = __builtin_amdgcn_readfirstlane(total_tiles);
  // lane dd <= nd: offset of document p0 + dd; lane dd < nd: is document dd empty
  const int64_t doff_lane = (l <= nd) ? P.D.off[p0 + l] : 0;
  const int64_t doff_end = P.D.off[p1];
  if (l == 0) lds_npass[w] = (total_tiles + NT - 1) / NT;
  __builtin_amdgcn_s_waitcnt(0);                               // nothing in flight before the tile stream
  __syncthreads();
  int n_pass = 0;
#pragma unroll
  for (int i = 0; i < kDenseWaves; ++i) n_pass = max(n_pass, lds_npass[i]);
  auto rd64 = [&](int64_t v, int lane) -> int64_t {
    uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, lane);
    uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), lane);
    return (int64_t)(((uint64_t)hi << 32) | lo);
  };
  auto doc_start = [&](int dd) -> int64_t { return dd >= 64 ? doff_end : rd64(doff_lane, dd); };
  const uint32_t nx_lo = (uint32_t)__shfl_down((int)(uint32_t)doff_lane, 1);
  const uint32_t nx_hi = (uint32_t)__shfl_down((int)(uint32_t)(doff_lane >> 32), 1);
  const int64_t doff_next = (l == 63) ? doff_end : (int64_t)(((uint64_t)nx_hi << 32) | nx_lo);
  const bool doc_empty = l < nd && doff_next == doff_lane;
  auto skip_empty = [&](int dd) -> int {
    while (dd < nd && doc_start(dd + 1) == doc_start(dd)) ++dd;
    return dd;
  };
  const int dd_first = skip_empty(0);
  const int64_t beg_first = dd_first < nd ? doc_start(dd_first) : 0;
  const int64_t len_first = dd_first < nd ? doc_start(dd_first + 1) - beg_first : 1;
  const uint32_t lds0 = (uint32_t)(size_t)(lds_void_ptr)&lds_tiles[0][0][0];

  float part = 0.0f;                                            // lane dd: partial score carried to the next pass
  for (int pass = 0; pass < n_pass; ++pass) {
    const int pt0 = pass * NT;
    const int nct = __builtin_amdgcn_readfirstlane(max(0, min(NT, total_tiles - pt0)));
    // tile map of this pass: owner query, first/last flags, B operand rows
    Frag B[NT];
    float qs[NT / 4];                                           // FP8: scale of this lane's column in R[i]
#pragma unroll
    for (int i = 0; i < NT / 4; ++i) qs[i] = 1.0f;
    int tq_lane = 0;                                            // lane ct: query owning tile ct
    uint64_t first_mask = 0, last_mask = 0;
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) {
      O::zero(B[ct]);
      if (ct < nct) {
        const int t = pt0 + ct;
        const uint64_t own = __ballot(l < nq && qt0 <= t && t < qt0 + qnt);
        const int j = __ffsll((unsigned long long)own) - 1;
        const int jt0 = __builtin_amdgcn_readlane(qt0, j);
        const int jm = __builtin_amdgcn_readlane(qm, j);
        const int64_t jrow = rd64(qrow, j);
        const int k = t - jt0;                                  // tile index inside query j
        if (l == ct) tq_lane = j;
        if (k == 0) first_mask |= 1ull << ct;
        if (16 * (k + 1) >= jm) last_mask |= 1ull << ct;
        if (16 * k + c16 < jm) {
          O::load_b(B[ct], P.Q.vecs, P.Q.scales, jrow + 16 * k + c16, g);
          if constexpr (O::kColumnScale)
            if (g == (ct & 3)) qs[ct >> 2] = P.Q.scales[jrow + 16 * k + c16];
        }
      }
    }
    float rm[NT], scr[NT];
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) { rm[ct] = ninf; scr[ct] = 0.0f; }
    __builtin_amdgcn_s_waitcnt(0);                             // operands in; the stream starts from zero

    // copy cursor (l_*) runs kBuffers-1 groups ahead of the compute cursor (c_*)
    int l_dd = dd_first, l_t = 0;
    int64_t l_beg = beg_first, l_len = len_first;
    int c_dd = dd_first, c_t = 0;
    int64_t c_len = len_first;
    int issued_full = 0;                                        // groups after the current one, fully issued
    auto issue_group = [&](int buf) -> bool {                   // true if all kGroup tiles were issued
      int n = 0;
#pragma unroll
      for (int u = 0; u < kGroup; ++u) {
        if (l_dd < nd) {
          TS::copy(P.D.vecs, P.D.scales, l_beg, l_len, l_t, &lds_tiles[buf][u][0], u, w, l);
          ++n;
          if ((int64_t)(l_t + 1) * 16 < l_len) ++l_t;
          else {
            l_dd = skip_empty(l_dd + 1); l_t = 0;
            if (l_dd < nd) { l_beg = doc_start(l_dd); l_len = doc_start(l_dd + 1) - l_beg; }
          }
        }
      }
      return n == kGroup;
    };
    issue_group(0);
    issued_full = issue_group(1) ? 1 : 0;
    for (int grp = 0; c_dd < nd; ++grp) {
      const int buf = grp % kBuffers;
      // this wave's copies of group grp are done when at most one later group is in flight
      if (issued_full) wait_vm<TS::kCopiesPerWave>(); else wait_vm<0>();
      __builtin_amdgcn_s_barrier();                             // group grp landed; buffer grp-1 is free
      issued_full = issue_group((grp + kBuffers - 1) % kBuffers) ? 1 : 0;
      const uint32_t gbase = lds0 + (uint32_t)(buf * kGroup * TS::kStageBytes);
#pragma nounroll
      for (int u = 0; u < kGroup; ++u) {
        if (c_dd < nd) {
          const bool last_tile = (int64_t)(c_t + 1) * 16 >= c_len;
          if (nct > 0) {
            Frag A;
            frag_from_lds<DT>(A, gbase + u * TS::kStageBytes, c16, g);
            // column tiles in groups of 4 (a group past the last used tile is
            // skipped; unused tiles inside a group have zero B operands and
            // their maxima are never read)
#pragma unroll
            for (int g0 = 0; g0 < NT; g0 += 4) {
              if (g0 < nct) {
                f32x4 acc[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s = 0; s < O::kSteps; ++s) {
#pragma unroll
                  for (int c = 0; c < 4; ++c) acc[c] = O::mma(A, B[g0 + c], acc[c], s);
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) update_max(rm[g0 + c], acc[c]);
              }
            }
            if (last_tile) {
              float Rs[NT / 4];
              tile_sums<NT, O::kColumnScale>(rm, Rs, qs);
              // each query's score: its tile sums in tile order, parked in lane dd
              const int dd = c_dd;
              float s_run = 0.0f;
#pragma unroll
              for (int ct = 0; ct < NT; ++ct) {
                if (ct < nct) {
                  const float T = tile_sum_at<NT>(Rs, ct);
                  if ((first_mask >> ct) & 1) s_run = T;
                  else if (ct == 0) s_run = readlane_f(part, dd) + T;     // continues from the previous pass
                  else s_run += T;
                  if (((last_mask >> ct) & 1) || ct == nct - 1) scr[ct] = writelane_f(scr[ct], s_run, dd);
                }
                rm[ct] = ninf;
              }
            }
          }
          if (!last_tile) ++c_t;
          else {
            c_dd = skip_empty(c_dd + 1); c_t = 0;
            if (c_dd < nd) c_len = doc_start(c_dd + 1) - doc_start(c_dd);
          }
        }
      }
    }
    wait_vm<0>();                                               // no copy outlives the pass
    __syncthreads();                                            // buffers are reused by the next pass
    // finished queries: one 64-document row each (empty documents score -inf)
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) {
      if (ct < nct) {
        if ((last_mask >> ct) & 1) {
          const int j = __builtin_amdgcn_readlane(tq_lane, ct);
          const int64_t row = P.out.rows ? (int64_t)P.out.rows[q0 + j] : (int64_t)(q0 + j);
          if (l < nd) P.out.scores[row * P.out.ld + p0 + l] = doc_empty ? ninf : scr[ct];
        } else if (ct == nct - 1) {
          part = scr[ct];
        }
      }
    }
  }
  // empty queries score 0 against every document
  for (int j = 0; j < nq; ++j) {
    if (__builtin_amdgcn_readlane(qm, j) == 0 && l < nd) {
      const int64_t row = P.out.rows ? (int64_t)P.out.rows[q0 + j] : (int64_t)(q0 + j);
      P.out.scores[row * P.out.ld + p0 + l] = 0.0f;
    }
  }
}

hipError_t launch_score_dense(int dtype, const SetsView& Q, const SetsView& D, const int32_t* qb_start,
                              const int64_t* qcol, int64_t n_blocks_max, const DenseOut& out, hipStream_t s) {
  DenseParams P;
  P.Q = Q; P.D = D; P.qb = qb_start; P.qcol = qcol; P.n_blocks_max = n_blocks_max;
  P.n_bgroups = (n_blocks_max + kDenseWaves - 1) / kDenseWaves;
  P.out = out;
  const int64_t n_chunks = (D.n_sets + kChunkDocs - 1) / kChunkDocs;
  if (P.n_bgroups == 0 || n_chunks == 0) return hipSuccess;
  // slices of whole chunks, each launch within the dispatch's work-item limit
  const int64_t max_items = (kMaxGridThreads / kDenseThreads) & ~int64_t(7);
  const int64_t slice = std::max<int64_t>(1, max_items / P.n_bgroups);
  const dim3 blk(kDenseThreads);
  for (int64_t c0 = 0; c0 < n_chunks; c0 += slice) {
    P.chunk0 = c0;
    P.n_chunks = std::min(slice, n_chunks - c0);
    const int64_t grid = ((P.n_bgroups * P.n_chunks + 7) / 8) * 8;
    switch (dtype) {
      case GEM_F32: hipLaunchKernelGGL(score_dense_kernel<GEM_F32>, dim3((unsigned)grid), blk, 0, s, P); break;
      case GEM_BF16: hipLaunchKernelGGL(score_dense_kernel<GEM_BF16>, dim3((unsigned)grid), blk, 0, s, P); break;
      case GEM_FP8_E4M3: hipLaunchKernelGGL(score_dense_kernel<GEM_FP8_E4M3>, dim3((unsigned)grid), blk, 0, s, P); break;
      default: return hipErrorInvalidValue;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// --------------------------------------------------------------------------
// Gathered scorer: one wave scores up to kGatherEntries consecutive entries of
// one query's candidate list. The query's vectors stay in registers (64 per
// pass); each candidate document is streamed tile by tile, the next tile's
// load in flight while the current one is multiplied. A score is the same sum
// of per-tile column sums, in tile order, as in the dense scorer.
constexpr int kGatherEntries = 16;
constexpr int kGatherNT = 4;

struct GatherParams {
  SetsView Q, D;
  CandsView C;
  int64_t chunks_per_query;
  int64_t wave0;          // first wave of this launch (large batches launch in slices)
  float* scores;
};

template <int DT>
__global__ __launch_bounds__(256) void score_gather_kernel(GatherParams P) {
  using O = Op<DT>;
  using Frag = typename O::Frag;
  constexpr int NT = kGatherNT;
  constexpr int PASS = 16 * NT;
  __shared__ float lds_sc[4][kGatherEntries];
  __shared__ int64_t lds_ent[4][kGatherEntries][2];

  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c16 = l & 15;
  const int64_t gw = P.wave0 + (int64_t)blockIdx.x * 4 + w;
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

  // lane e < ne: the entry's document id and row range, kept in LDS so that
  // the per-entry bookkeeping never waits on the vector-memory counter
  int32_t my_id = -1;
  int64_t my_beg = 0, my_len = 0;
  if (l < ne) {
    my_id = P.C.ids[e0 + l];
    if (my_id >= 0) { my_beg = P.D.off[my_id]; my_len = P.D.off[my_id + 1] - my_beg; }
    lds_ent[w][l][0] = my_beg;
    lds_ent[w][l][1] = my_len;
  }
  __builtin_amdgcn_wave_barrier();
  auto ent_beg = [&](int e) -> int64_t { return lds_ent[w][e][0]; };
  auto ent_len = [&](int e) -> int64_t { return lds_ent[w][e][1]; };

  const int64_t r0 = P.Q.off[q];
  const int m = (int)(P.Q.off[q + 1] - r0);
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
    const int nct = __builtin_amdgcn_readfirstlane((pr + 15) >> 4);
    const bool first_pass = prow0 == 0;
    Frag B[NT];
    float qs[NT / 4];
#pragma unroll
    for (int i = 0; i < NT / 4; ++i) qs[i] = 1.0f;
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) {
      const int col = prow0 + 16 * ct + c16;
      if (ct < nct && col < m) {
        O::load_b(B[ct], P.Q.vecs, P.Q.scales, r0 + col, g);
        if constexpr (O::kColumnScale)
          if (g == (ct & 3)) qs[ct >> 2] = P.Q.scales[r0 + col];
      } else {
        O::zero(B[ct]);
      }
    }
    auto next_entry = [&](int e) -> int {          // next entry with a non-empty document
      while (e < ne && ent_len(e) == 0) ++e;
      return e;
    };
    int e = next_entry(0);
    int t = 0;
    int64_t dbeg = 0, dlen = 0;
    Frag A_next;
    if (e < ne) {
      dbeg = ent_beg(e);
      dlen = ent_len(e);
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
        if (ne_ < ne) { nbeg = ent_beg(ne_); nlen = ent_len(ne_); }
      }
      if (ne_ < ne) O::load(A_next, P.D.vecs, P.D.scales, nbeg + min((int64_t)(nt * 16 + c16), nlen - 1), g);
      // all NT column tiles: tiles past the query's last vector have zero B
      // operands and their maxima are never read
      f32x4 acc[NT];
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < O::kSteps; ++s) {
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) acc[ct] = O::mma(A, B[ct], acc[ct], s);
      }
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) update_max(rm[ct], acc[ct]);
      if (last_tile) {
        float R[NT / 4];
        tile_sums<NT, O::kColumnScale>(rm, R, qs);
        float s_run = first_pass ? tile_sum_at<NT>(R, 0) : sc[e] + tile_sum_at<NT>(R, 0);
#pragma unroll
        for (int ct = 1; ct < NT; ++ct)
          if (ct < nct) s_run += tile_sum_at<NT>(R, ct);
        if (l == 0) sc[e] = s_run;
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) rm[ct] = ninf;
      }
      e = ne_; t = nt; dbeg = nbeg; dlen = nlen;
    }
    __builtin_amdgcn_wave_barrier();
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
  const int64_t max_blocks = kMaxGridThreads / 256;
  for (int64_t b0 = 0; b0 < (waves + 3) / 4; b0 += max_blocks) {
    P.wave0 = b0 * 4;
    const int64_t grid = std::min(max_blocks, (waves + 3) / 4 - b0);
    switch (dtype) {
      case GEM_F32: hipLaunchKernelGGL(score_gather_kernel<GEM_F32>, dim3((unsigned)grid), dim3(256), 0, s, P); break;
      case GEM_BF16: hipLaunchKernelGGL(score_gather_kernel<GEM_BF16>, dim3((unsigned)grid), dim3(256), 0, s, P); break;
      case GEM_FP8_E4M3: hipLaunchKernelGGL(score_gather_kernel<GEM_FP8_E4M3>, dim3((unsigned)grid), dim3(256), 0, s, P); break;
      default: return hipErrorInvalidValue;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace gem
