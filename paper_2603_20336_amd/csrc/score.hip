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
#include <type_traits>

#include "device_common.hpp"
#include "gem_internal.h"
#include "mfma_ops.hpp"

namespace gem {

// Row of S's vector array that entry r stands for (code sets: its centroid).
__device__ __forceinline__ int64_t vec_row(const SetsView& S, int64_t r) {
  return S.codes ? (int64_t)S.codes[r] : r;
}

// Column tiles (16 query vectors each) held in registers by one pass.
template <int DT> struct DenseCfg;
// kNT: 16-column tiles a wave holds; kGroup: document tiles per LDS group buffer.
template <> struct DenseCfg<GEM_F32> { static constexpr int kNT = 4; static constexpr int kGroup = 4; };
template <> struct DenseCfg<GEM_BF16X3> { static constexpr int kNT = 4; static constexpr int kGroup = 4; };
template <> struct DenseCfg<GEM_BF16> { static constexpr int kNT = 8; static constexpr int kGroup = 8; };
template <> struct DenseCfg<GEM_FP8_E4M3> { static constexpr int kNT = 16; static constexpr int kGroup = 8; };
template <> struct DenseCfg<GEM_MXFP4> { static constexpr int kNT = 16; static constexpr int kGroup = 8; };
template <> struct DenseCfg<GEM_MXFP6> { static constexpr int kNT = 16; static constexpr int kGroup = 8; };

int dense_pass_rows(int dtype) {
  switch (dtype) {
    case GEM_F32: return 16 * DenseCfg<GEM_F32>::kNT;
    case GEM_BF16X3: return 16 * DenseCfg<GEM_BF16X3>::kNT;
    case GEM_BF16: return 16 * DenseCfg<GEM_BF16>::kNT;
    default: return 16 * DenseCfg<GEM_FP8_E4M3>::kNT;
  }
}

static int pad16(int m) { return (m + 15) & ~15; }
constexpr int64_t kDenseWavesPerGroup = 8;       // query blocks per block group (waves per workgroup)
constexpr int kNarrowCols = 64;                    // block width of the FP8 narrow-block variant
constexpr int64_t kNarrowGroups = 16;  // block groups a batch may fill with narrow blocks

int dense_block_rows(int dtype, int max_len) {
  const int r = dense_pass_rows(dtype);
  const int m = pad16(max_len);
  return m <= r ? r : ((m + r - 1) / r) * r;
}

// Block width for a batch of n_q queries holding n_vecs vectors: the full
// width, or for a small batch one narrow enough to give each wave of a block
// group a block of its own (a narrower block only changes the plan, never a
// score).
int dense_block_rows_for(int dtype, int max_len, int64_t n_q, int64_t n_vecs) {
  const int full = dense_block_rows(dtype, max_len);
  const int64_t cols = n_vecs + 15 * n_q;                                   // padded columns, upper bound
  const int64_t per_wave = (((cols + kDenseWavesPerGroup - 1) / kDenseWavesPerGroup) + 15) & ~(int64_t)15;
  const int64_t narrow = std::max<int64_t>(pad16(max_len > 0 ? max_len : 1), per_wave);
  // FP8: a batch of short queries that up to 16 block groups of 64-column
  // blocks hold takes such blocks (the narrow-block variant of the scorer,
  // four waves per SIMD): against 256-column blocks, whose last block group
  // a batch of this size fills only in part, 32 and 64 serving-mix queries
  // score 1.55-1.65x faster, 128 about 5 % faster, 256 the same
  if (dtype == GEM_FP8_E4M3 && narrow > kNarrowCols && max_len <= kNarrowCols &&
      cols <= kNarrowCols * kDenseWavesPerGroup * kNarrowGroups)
    return kNarrowCols;
  return narrow < full ? (int)narrow : full;
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
    // (maxima of finite or -inf values: IEEE maximum, which needs no NaN
    // quieting of the lane-swapped operands)
    auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(rm[4 * i + 0]), __float_as_uint(rm[4 * i + 1]), false, false);
    const float ab = __builtin_elementwise_maximum(__uint_as_float(p[0]), __uint_as_float(p[1]));   // rows: A01 B01 A23 B23
    auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(rm[4 * i + 2]), __float_as_uint(rm[4 * i + 3]), false, false);
    const float cd = __builtin_elementwise_maximum(__uint_as_float(q[0]), __uint_as_float(q[1]));   // rows: C01 D01 C23 D23
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(ab), __float_as_uint(cd), false, false);
    float m = __builtin_elementwise_maximum(__uint_as_float(r[0]), __uint_as_float(r[1]));         // rows: A B C D
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
constexpr int kMaxChunkDocs = 64;               // a chunk's documents map to the 64 lanes
constexpr int kBuffers = 3;                    // group buffers: two groups in flight
constexpr int kDenseWaves = 8;                 // two waves per SIMD
static_assert(kDenseWaves == kDenseWavesPerGroup, "block groups hold one block per wave");
constexpr int kDenseThreads = 64 * kDenseWaves;

typedef __attribute__((address_space(3))) void* lds_void_ptr;
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

struct DenseParams {
  SetsView Q, D;
  const int32_t* qb;
  const int64_t* qcol;
  int64_t n_blocks_max, n_bgroups, n_chunks;
  int64_t chunk0;         // first document chunk of this launch
  int32_t chunk_docs;     // documents per chunk (<= kMaxChunkDocs)
  int32_t items_per_slot; // target work items per workgroup
  DenseOut out;
};

// LDS image of one 16-row tile: row r at r * kRowBytes, 16-byte chunk c at
// position c ^ swz(r); FP8 and MX tiles are followed by their 16 row scales.
// MXFP6 rows (96 bytes in memory) are staged as 128-byte rows: chunks 6 and 7
// of a row repeat its chunk 5 and are never read.
template <int DT> struct TileStage {
  using O = Op<DT>;
  static constexpr int kRowBytes = DT == GEM_MXFP6 ? 128 : O::kRowBytes;
  static constexpr int kGlobalChunks = O::kRowBytes / 16;      // chunks of a row in memory
  static constexpr int kChunksPerRow = kRowBytes / 16;
  static constexpr int kTileBytes = 16 * kRowBytes;
  static constexpr int kSlots = kTileBytes / 16;                 // 16-byte pieces per tile
  static constexpr int kPieceWaves = kSlots / 64;                // waves copying one piece per lane
  static constexpr bool kScales = DT == GEM_FP8_E4M3 || DT == GEM_MXFP4 || DT == GEM_MXFP6;   // a scale word per row
  static constexpr int kCopyWaves = kPieceWaves + (kScales ? 1 : 0);   // waves busy copying one tile
  // FP8: the tile's 16 row scales, copied by a whole wave (lanes past 16 fill
  // the rest of the slot with repeats)
  static constexpr int kStageBytes = kTileBytes + (kScales ? 256 : 0);
  static constexpr int kGroup = DenseCfg<DT>::kGroup;
  static constexpr int kGroupVecs = kGroup * kStageBytes / 16;  // one group buffer in 16-byte units
  // a group's piece copies are slots s = u * kPieceWaves + role (tile u,
  // 1 KiB piece `role`); wave w issues the contiguous slots [w K, w K + K)
  // (K = kPieceCopiesPerWave), which lie in one tile, so that one document
  // lookup serves all of them; the scale copies of that tile are the same
  // wave's. Every wave issues the same number of copies.
  static constexpr int kPieceCopiesPerWave = kGroup * kPieceWaves / kDenseWaves;
  static constexpr int kScaleCopiesPerWave = kScales ? kGroup / kDenseWaves : 0;
  static constexpr int kCopiesPerWave = kPieceCopiesPerWave + kScaleCopiesPerWave;
  static_assert(kSlots % 64 == 0, "tile copy layout");
  static_assert((kGroup * kPieceWaves) % kDenseWaves == 0 && (!kScales || kGroup % kDenseWaves == 0),
                "copies must spread evenly over the waves");
  static_assert(kPieceCopiesPerWave <= kPieceWaves && kPieceWaves % kPieceCopiesPerWave == 0,
                "a wave's piece copies lie in one tile");
  static_assert(!kScales || (kPieceCopiesPerWave == kPieceWaves && kScaleCopiesPerWave == 1),
                "a wave copies the scales of its own tile");
  // the tile of the group that wave w copies, and the piece of its copy j
  static __device__ __forceinline__ int wave_tile(int w) { return w * kPieceCopiesPerWave / kPieceWaves; }
  static __device__ __forceinline__ int wave_piece(int w, int j) { return (w * kPieceCopiesPerWave + j) % kPieceWaves; }
  static_assert(kStageBytes % 16 == 0, "stage alignment");

  // chunk c of row r sits at position c ^ swz(r). A 16-byte LDS read serves
  // its 64 lanes in two halves of 32 lanes (16 rows x two lane groups), and a
  // half runs without bank conflicts when its 32 reads fall in 32 distinct
  // 16-byte columns of the 512-byte bank space. For 256- and 512-byte rows the
  // plain row XOR (r & 15) maps the two lane groups of a half onto the same
  // columns (measured: twice the cycles of a conflict-free read); the forms
  // below keep the two groups apart. 64-byte rows interleave four rows and
  // 128-byte rows pair up first.
  static __device__ __forceinline__ int swz(int r) {
    if constexpr (kRowBytes == 64) return (r >> 2) & 3;
    else if constexpr (kRowBytes == 128) return (r >> 1) & 7;
    else if constexpr (kRowBytes == 256) return ((r >> 1) & 3) | (r & 8) | ((r & 1) << 2);
    else return (r & 7) | ((r & 8) << 1);
  }
  // the memory chunk copied into LDS chunk c (the padding chunks of a staged
  // MXFP6 row repeat the row's last chunk)
  static __device__ __forceinline__ int mem_chunk(int c) {
    if constexpr (kGlobalChunks < kChunksPerRow) return min(c, kGlobalChunks - 1);
    else return c;
  }

  // Piece `role` (1 KiB) of tile k of the document whose rows are
  // base + [rs, re), into `stage`.
  static __device__ __forceinline__ void copy_piece(const void* vecs, int64_t base, int rs, int re, int k,
                                                    u32x4* stage, int role, int l) {
    const int slot = 64 * role + l;
    const int r = slot / kChunksPerRow, pos = slot % kChunksPerRow;
    const int c = mem_chunk(pos ^ swz(r));
    const int64_t row = base + min(rs + 16 * k + r, re - 1);
    __builtin_amdgcn_global_load_lds(static_cast<const char*>(vecs) + row * O::kRowBytes + c * 16,
                                     (lds_void_ptr)(stage + 64 * role), 16, 0, 0);
  }
  // Code sets: the same piece, when the lane's row of the vector array is
  // already known (its code).
  static __device__ __forceinline__ void copy_piece_row(const void* vecs, int64_t vrow, u32x4* stage, int role,
                                                        int l) {
    const int slot = 64 * role + l;
    const int r = slot / kChunksPerRow, pos = slot % kChunksPerRow;
    const int c = mem_chunk(pos ^ swz(r));
    __builtin_amdgcn_global_load_lds(static_cast<const char*>(vecs) + vrow * O::kRowBytes + c * 16,
                                     (lds_void_ptr)(stage + 64 * role), 16, 0, 0);
  }
  // Entry index whose row lane l copies in piece `role` of tile k.
  static __device__ __forceinline__ int64_t piece_entry(int64_t base, int rs, int re, int k, int role, int l) {
    const int r = (64 * role + l) / kChunksPerRow;
    return base + min(rs + 16 * k + r, re - 1);
  }
  // The 16 row scales of that tile (lanes past 16 repeat them).
  static __device__ __forceinline__ void copy_scales(const float* scales, int64_t base, int rs, int re, int k,
                                                     u32x4* stage, int l) {
    __builtin_amdgcn_global_load_lds(scales + base + min(rs + 16 * k + (l & 15), re - 1),
                                     (lds_void_ptr)(stage + kTileBytes / 16), 4, 0, 0);
  }
};

// s_waitcnt with only the vector-memory count set (expcnt / lgkmcnt left open)
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0f70);
}

// Keeps the compiler from moving memory operations across this point (no
// hardware wait is implied).
__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

// A operand of one tile from its LDS stage (plain loads: the compiler places
// their waits; the copies in flight target other LDS arrays).
template <int DT>
__device__ __forceinline__ void frag_from_lds(typename Op<DT>::Frag& f, const u32x4* stage, int c16, int g);

template <>
__device__ __forceinline__ void frag_from_lds<GEM_BF16>(Op<GEM_BF16>::Frag& f, const u32x4* stage, int c16, int g) {
  const u32x4* row = stage + c16 * 16;
  const int sw = TileStage<GEM_BF16>::swz(c16);
#pragma unroll
  for (int s = 0; s < 4; ++s) f.v[s] = __builtin_bit_cast(bf16x8, row[(4 * g + s) ^ sw]);
}

template <>
__device__ __forceinline__ void frag_from_lds<GEM_FP8_E4M3>(Op<GEM_FP8_E4M3>::Frag& f, const u32x4* stage, int c16,
                                                            int g) {
  const u32x4* row = stage + c16 * 8;
  const u32x4 v0 = row[(2 * g) ^ ((c16 >> 1) & 7)];
  const u32x4 v1 = row[(2 * g + 1) ^ ((c16 >> 1) & 7)];
  const uint32_t sc = reinterpret_cast<const uint32_t*>(stage + 128)[c16];
  f.v = i32x8{(int)v0.x, (int)v0.y, (int)v0.z, (int)v0.w, (int)v1.x, (int)v1.y, (int)v1.z, (int)v1.w};
  f.scale = (int)((sc >> 23) & 0xffu);
}

template <>
__device__ __forceinline__ void frag_from_lds<GEM_MXFP4>(Op<GEM_MXFP4>::Frag& f, const u32x4* stage, int c16, int g) {
  const u32x4 v = stage[c16 * 4 + (g ^ ((c16 >> 2) & 3))];
  const uint32_t sc = reinterpret_cast<const uint32_t*>(stage + 64)[c16];
  f.v = i32x4{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
  f.scale = (int)((sc >> (8 * g)) & 0xffu);
}

// MXFP6: block g (24 bytes) of the staged 128-byte row is chunk 3h (whole)
// and the low half of chunk 3h + 1 for g = 2h, the high half of chunk 3h + 1
// and chunk 3h + 2 (whole) for g = 2h + 1.
template <>
__device__ __forceinline__ void frag_from_lds<GEM_MXFP6>(Op<GEM_MXFP6>::Frag& f, const u32x4* stage, int c16, int g) {
  const u32x4* row = stage + c16 * 8;
  const int sw = (c16 >> 1) & 7, h = g >> 1, odd = g & 1;
  const u32x4 w = row[(3 * h + 2 * odd) ^ sw];
  const uint2 m = reinterpret_cast<const uint2*>(row + ((3 * h + 1) ^ sw))[odd];
  const uint32_t sc = reinterpret_cast<const uint32_t*>(stage + 128)[c16];
  f.v = odd ? i32x8{(int)m.x, (int)m.y, (int)w.x, (int)w.y, (int)w.z, (int)w.w, 0, 0}
            : i32x8{(int)w.x, (int)w.y, (int)w.z, (int)w.w, (int)m.x, (int)m.y, 0, 0};
  f.scale = (int)((sc >> (8 * g)) & 0xffu);
}

template <>
__device__ __forceinline__ void frag_from_lds<GEM_F32>(Op<GEM_F32>::Frag& f, const u32x4* stage, int c16, int g) {
  const u32x4* row = stage + c16 * 32;
  const int sw = TileStage<GEM_F32>::swz(c16);
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const u32x4 v = row[(8 * g + s) ^ sw];
    f.v[4 * s + 0] = __uint_as_float(v.x); f.v[4 * s + 1] = __uint_as_float(v.y);
    f.v[4 * s + 2] = __uint_as_float(v.z); f.v[4 * s + 3] = __uint_as_float(v.w);
  }
}

// GEM_BF16X3: block g of the staged 512-byte row is chunks 8g .. 8g + 7 (hi
// in the first four, lo in the last four).
template <>
__device__ __forceinline__ void frag_from_lds<GEM_BF16X3>(Op<GEM_BF16X3>::Frag& f, const u32x4* stage, int c16,
                                                          int g) {
  const u32x4* row = stage + c16 * 32;
  const int sw = TileStage<GEM_BF16X3>::swz(c16);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    f.h[i] = __builtin_bit_cast(bf16x8, row[(8 * g + i) ^ sw]);
    f.l[i] = __builtin_bit_cast(bf16x8, row[(8 * g + 4 + i) ^ sw]);
  }
}

__device__ __forceinline__ float writelane_f(float old, float v, int lane) {
  return lane_id() == lane ? v : old;
}
__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __uint_as_float(__builtin_amdgcn_readlane(__float_as_uint(v), lane));
}

// --------------------------------------------------------------------------
// Fused top-k: one wave's region of candidate keys for one query and piece.
// A key holds the score's order-preserving bits above the complemented
// document id, so a larger key is a higher score or, on equal scores, a
// smaller id; the keys of one query's documents are distinct.
__device__ __forceinline__ uint64_t tk_rank_key(float s, int32_t id) {
  return ((uint64_t)float_order_key(s) << 32) | (uint64_t)(~(uint32_t)id);
}

// Region reads take the entries other lanes of the wave stored: they wait for
// those stores and read past the vector L1.
__device__ __forceinline__ uint64_t tk_load(uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum over the wave of v (every lane receives it).
__device__ __forceinline__ uint32_t tk_wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Histogram add from the whole wave: one LDS atomic per lane group that hits
// the same bin as the first active lane when all active lanes agree.
__device__ __forceinline__ void tk_hist_add(uint32_t* hist, bool active, uint32_t bin) {
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

// Keys a region holds at most (k <= 1024 plus 1024 free slots).
constexpr int kTkMaxCap = 2048;
// Keys a lane reads per batch in a selection (loads in flight).
constexpr int kTkBatch = 16;

// The k best of the n (k < n <= kTkMaxCap) distinct keys R[0..n) move to
// R[0..k); returns the k-th best. Radix select over the wave, eight bits a
// round from the top, with a 256-bin histogram in `hist` (this wave's own
// LDS); each round reads the keys in batches of kTkBatch per lane, and the
// select stops early once the selected bin holds exactly the keys still
// needed (the threshold is then the least key kept). It runs rarely (when a
// region is full) and out of line, so that its registers stay out of the
// scorer's. Wave-uniform arguments; all lanes call it.
__device__ __attribute__((noinline)) uint64_t tk_select_k(uint64_t* R, int n, int k, uint32_t* hist) {
  const int l = lane_id();
  __builtin_amdgcn_s_waitcnt(0);                        // this wave's stores into R are done
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  uint64_t prefix = 0, mask = 0;
  uint32_t need = (uint32_t)k;
  bool whole_bin = false;                               // keep every key of the selected bin
  for (int shift = 56; shift >= 0; shift -= 8) {
#pragma unroll
    for (int b = 0; b < 4; ++b) hist[4 * l + b] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int i0 = 0; i0 < n; i0 += 64 * kTkBatch) {
      uint64_t kv[kTkBatch];
#pragma unroll
      for (int u = 0; u < kTkBatch; ++u) {
        const int i = i0 + 64 * u + l;
        kv[u] = i < n ? tk_load(R + i) : 0ull;
      }
#pragma unroll
      for (int u = 0; u < kTkBatch; ++u) {
        const int i = i0 + 64 * u + l;
        tk_hist_add(hist, i < n && (kv[u] & mask) == prefix, (uint32_t)(kv[u] >> shift) & 0xffu);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // lane l holds bins 4l..4l+3; `above` counts the keys in higher bins
    const uint32_t h0 = hist[4 * l], h1 = hist[4 * l + 1], h2 = hist[4 * l + 2], h3 = hist[4 * l + 3];
    const uint32_t own = h0 + h1 + h2 + h3;
    uint32_t incl = own;                                // sum over lanes >= l
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t v = __shfl_down(incl, o);
      if (l + o < 64) incl += v;
    }
    uint32_t gt = incl - own;
    int digit = -1;
    uint32_t gt_sel = 0, h_sel = 0;
    const uint32_t hb[4] = {h0, h1, h2, h3};
#pragma unroll
    for (int b = 3; b >= 0; --b) {
      if (digit < 0 && gt < need && need <= gt + hb[b]) { digit = 4 * l + b; gt_sel = gt; h_sel = hb[b]; }
      gt += hb[b];
    }
    const uint64_t who = __ballot(digit >= 0);
    const int src = __ffsll((unsigned long long)who) - 1;
    const uint32_t d = (uint32_t)__builtin_amdgcn_readlane(digit, src);
    const uint32_t g_above = (uint32_t)__builtin_amdgcn_readlane(gt_sel, src);
    const uint32_t in_bin = (uint32_t)__builtin_amdgcn_readlane(h_sel, src);
    need -= g_above;
    prefix |= (uint64_t)d << shift;
    mask |= 0xffull << shift;
    if (in_bin == need) { whole_bin = true; break; }
  }
  // keep the keys above the selected bin and (all of, or the one key of) it,
  // in their order; every key kept moves left, so a batch's stores only hit
  // entries this batch or earlier ones read
  uint64_t kmin = ~0ull;
  int pos = 0;
  for (int i0 = 0; i0 < n; i0 += 64 * kTkBatch) {
    uint64_t kv[kTkBatch];
#pragma unroll
    for (int u = 0; u < kTkBatch; ++u) {
      const int i = i0 + 64 * u + l;
      kv[u] = i < n ? tk_load(R + i) : 0ull;
    }
#pragma unroll
    for (int u = 0; u < kTkBatch; ++u) {
      const int i = i0 + 64 * u + l;
      const uint64_t key = kv[u];
      const bool keep = i < n && ((key & mask) > prefix || (whole_bin ? (key & mask) == prefix : key == prefix));
      const uint64_t b = __ballot(keep);
      if (keep) {
        R[pos + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u))] = key;
        kmin = key < kmin ? key : kmin;
      }
      pos += __popcll(b);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t v = __shfl_xor(kmin, o);
    kmin = v < kmin ? v : kmin;
  }
  return kmin;
}

// State of one wave over one pass of the dense scorer.
template <int DT, int NTO = 0> struct DensePass {
  using O = Op<DT>;
  using Frag = typename O::Frag;
  static constexpr int NT = NTO ? NTO : DenseCfg<DT>::kNT;
  Frag B[NT];                   // query columns of this pass
  float qs[NT / 4];             // FP8: scale of this lane's column in the tile sums
  float rm[NT];                 // running max over the current document, per column tile
  float* tsum;                  // this wave's [NT][64] LDS array: tile ct's column sum for document dd
  int nct, tq_lane;
  uint64_t first_mask, last_mask;

  // one document tile against the pass's column tiles (all of them when
  // kFull; a group past the last used tile is skipped, and unused tiles
  // inside a group have zero B operands and are never summed), then the next
  // tile's A operand, read into A once the last product has taken it. At a
  // document's last tile its tile sums are parked in column dd of the wave's
  // LDS array (the first lane of each 16-lane row stores that row's sum).
  template <bool kFull>
  __device__ __forceinline__ void tile(Frag& A, const u32x4* next, int c16, int g, uint64_t end_mask) {
#pragma unroll
    for (int g0 = 0; g0 < NT; g0 += 4) {
      if (kFull || g0 < nct) {
        f32x4 acc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < O::kSteps; ++s) {
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[c] = O::mma(A, B[g0 + c], acc[c], s);
        }
        if (kFull && g0 + 4 == NT) frag_from_lds<DT>(A, next, c16, g);
#pragma unroll
        for (int c = 0; c < 4; ++c) update_max(rm[g0 + c], acc[c]);
      }
    }
    if (!kFull) frag_from_lds<DT>(A, next, c16, g);
    if (end_mask) {
      const int dd = __builtin_ctzll(end_mask);
      float Rs[NT / 4];
      tile_sums<NT, O::kColumnScale>(rm, Rs, qs);
      const int l = lane_id();
      if ((l & 15) == 0) {
#pragma unroll
        for (int i = 0; i < NT / 4; ++i) tsum[(4 * i + (l >> 4)) * 64 + dd] = Rs[i];
      }
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) rm[ct] = neg_inf();
    }
  }
};

// kCodes: the documents are a code set. Each tile copy then needs the code of
// the row it copies; every wave fetches the codes of its own copies into its
// slots of one of three LDS code arrays (one per group buffer) two groups
// ahead, with the copies of the group two before, so that a copy never waits
// on a dependent load and the wait counts stay static.
// kTopk: the fused top-k (P.out.tk) takes the finished scores instead of the
// score matrix.
template <int DT, bool kCodes, int NTO, bool kTopk>
__device__ __forceinline__ void dense_body(const DenseParams& P) {
  using O = Op<DT>;
  using Frag = typename O::Frag;
  using TS = TileStage<DT>;
  constexpr int NT = NTO ? NTO : DenseCfg<DT>::kNT;
  constexpr int kGroup = TS::kGroup;
  constexpr int kCodeCopies = TS::kCopiesPerWave;               // one code per copy
  constexpr int kIssueOps = TS::kCopiesPerWave + (kCodes ? kCodeCopies : 0);
  constexpr int kCodeWords = kCodes ? kDenseWaves * kCodeCopies * 64 : 1;
  __shared__ int32_t lds_code0[kCodeWords];
  __shared__ int32_t lds_code1[kCodeWords];
  __shared__ int32_t lds_code2[kCodeWords];
  // three group buffers as separate arrays: the compiler then knows that the
  // copies in flight (into one buffer) never alias the reads (of another)
  __shared__ u32x4 lds_buf0[TS::kGroupVecs];
  __shared__ u32x4 lds_buf1[TS::kGroupVecs];
  __shared__ u32x4 lds_buf2[TS::kGroupVecs];
  __shared__ int lds_npass[kDenseWaves];
  __shared__ float lds_tsum[kDenseWaves][NT * 64];              // parked tile sums, per wave
  // fused top-k: the wave's selection histogram
  __shared__ uint32_t lds_tk_hist[kTopk ? kDenseWaves * 256 : 1];

  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63, g = l >> 4, c16 = l & 15;
  const float ninf = neg_inf();
  // Persistent workgroups. Workgroups go round-robin over the 8 XCDs; XCD x
  // owns a contiguous range of document chunks, cut into pieces, and its
  // workgroups take items (piece, block group), the group fastest, in
  // strides of the workgroup count. The workgroups an XCD runs at once then
  // walk the same chunks together (one L2 fetch serves all block groups),
  // and a workgroup whose block group does not change keeps its query
  // operands in registers from one item to the next.
  const int64_t n_bg = (P.qb[P.n_blocks_max + 1] + kDenseWaves - 1) / kDenseWaves;
  const int xcd = blockIdx.x & 7;
  const int64_t slot = blockIdx.x >> 3, n_slots = gridDim.x >> 3;
  const int64_t c_lo = P.chunk0 + (P.n_chunks * xcd) / 8;
  const int64_t c_hi = P.chunk0 + (P.n_chunks * (xcd + 1)) / 8;
  // about items_per_slot items per workgroup, the piece count rounded so
  // that the items divide evenly over the workgroups; piece p is chunks
  // [c_lo + p C / np, c_lo + (p + 1) C / np)
  const int64_t C = c_hi - c_lo;
  int64_t ga = n_slots, gb = n_bg;
  while (gb != 0) { const int64_t t = ga % gb; ga = gb; gb = t; }
  const int64_t even = n_slots / ga;                           // piece counts that divide evenly: multiples of this
  int64_t np = ((int64_t)P.items_per_slot * n_slots + n_bg - 1) / n_bg;
  np = min(((np + even - 1) / even) * even, C);
  if constexpr (kTopk) np = min((int64_t)P.out.tk.np, C);       // the caller's pieces (its regions)
  const int64_t n_items = np * n_bg;
  const int64_t tk_regions = kTopk ? 8 * (int64_t)P.out.tk.np : 0;

  DensePass<DT, NT> S;
  S.tsum = lds_tsum[w];
  int64_t cur_bg = -1;
  // fused top-k: lane j holds query j's running threshold and its region's
  // entry count (query j of the wave's current block)
  uint64_t tk_thr = 0;
  int tk_cnt = 0;
  int q0 = 0, nq = 0, n_pass = 0, total_tiles = 0;
  int64_t qrow = 0;
  int qm = 0, qt0 = 0, qnt = 0;
  bool b_loaded = false;                                       // S holds pass 0 of the current block group

  for (int64_t it = slot; it < n_items; it += n_slots) {
    const int64_t bgi = it % n_bg;
    if (bgi != cur_bg) {
      cur_bg = bgi;
      b_loaded = false;
      const int64_t b = bgi * kDenseWaves + w;
      int q1 = 0;
      q0 = 0;
      if (b < P.n_blocks_max) { q0 = P.qb[b]; q1 = P.qb[b + 1]; }
      nq = max(q1 - q0, 0);                                    // 0: this wave only helps copy
      // lane j < nq: query j of the block (first row, length, first tile, tiles)
      qrow = 0; qm = 0; qt0 = 0; qnt = 0;
      total_tiles = 0;
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
      __syncthreads();                                         // lds_npass of the previous group is read
      if (l == 0) lds_npass[w] = (total_tiles + NT - 1) / NT;
      __syncthreads();
      n_pass = 0;
#pragma unroll
      for (int i = 0; i < kDenseWaves; ++i) n_pass = max(n_pass, lds_npass[i]);
    }
    const int64_t pidx = it / n_bg;
    const int64_t pc0 = c_lo + (pidx * C) / np;
    const int64_t pc1 = c_lo + ((pidx + 1) * C) / np;
    const int64_t tk_piece = xcd * (int64_t)(kTopk ? P.out.tk.np : 0) + pidx;
    if constexpr (kTopk) {
      // this piece's regions start empty, behind the query's shared bound
      tk_thr = l < nq ? tk_load(reinterpret_cast<uint64_t*>(P.out.tk.gthr + q0 + l)) : 0ull;
      tk_cnt = 0;
    }
    for (int64_t chunk = pc0; chunk < pc1; ++chunk) {
      const int64_t p0 = chunk * P.chunk_docs;
      const int64_t p1 = min(P.D.n_sets, p0 + P.chunk_docs);
      const int nd = (int)(p1 - p0);

      // the chunk's document tiles, in order: lane dd < nd holds document
      // p0 + dd's rows (relative to the chunk's first row), its first tile in
      // the chunk's tile sequence and its last tile (-1 when it is empty)
      const int64_t base = P.D.off[p0];
      int d_rs = 0, d_re = 0;
      if (l < nd) {
        d_rs = (int)(P.D.off[p0 + l] - base);
        d_re = (int)(P.D.off[p0 + l + 1] - base);
      }
      const int d_nt = (d_re - d_rs + 15) >> 4;
      int d_incl = d_nt;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(d_incl, o);
        if (l >= o) d_incl += v;
      }
      const int d_t0 = d_incl - d_nt;
      const int d_tl = d_nt > 0 ? d_incl - 1 : -1;
      const int n_tiles = __builtin_amdgcn_readlane(d_incl, 63);
      const bool doc_empty = l < nd && d_nt == 0;
      const int n_groups = (n_tiles + kGroup - 1) / kGroup;

      // copies of group G into buffer Y. Every wave issues exactly
      // kCopiesPerWave copies per group, also past the last tile (those
      // repeat the last tile into slots that are never read), so that the
      // copies of later groups alone fill the wait count: the compiler can
      // then prove that the buffer being read has landed without waiting for
      // every copy.
      // tile T belongs to the last non-empty document whose first tile is <= T
      auto locate = [&](int T, int& k, int& rs, int& re) {
        const uint64_t m = __ballot(d_nt > 0 && d_t0 <= T);
        const int dd = 63 - __builtin_clzll(m);
        k = T - __builtin_amdgcn_readlane(d_t0, dd);
        rs = __builtin_amdgcn_readlane(d_rs, dd);
        re = __builtin_amdgcn_readlane(d_re, dd);
      };
      // code sets: the codes of this wave's copies of group G into array Z
      // (slot j of the wave: copy j's rows, one per lane)
      auto fetch_codes = [&](auto zbuf, int G) {
        constexpr int Z = decltype(zbuf)::value;
        int32_t* cb = (Z == 0 ? lds_code0 : (Z == 1 ? lds_code1 : lds_code2)) + w * kCodeCopies * 64;
        int k, rs, re;
        locate(min(G * kGroup + TS::wave_tile(w), n_tiles - 1), k, rs, re);
#pragma unroll
        for (int j = 0; j < TS::kPieceCopiesPerWave; ++j)
          __builtin_amdgcn_global_load_lds(P.D.codes + TS::piece_entry(base, rs, re, k, TS::wave_piece(w, j), l),
                                           (lds_void_ptr)(cb + 64 * j), 4, 0, 0);
#pragma unroll
        for (int j = 0; j < TS::kScaleCopiesPerWave; ++j)
          __builtin_amdgcn_global_load_lds(P.D.codes + base + min(rs + 16 * k + (l & 15), re - 1),
                                           (lds_void_ptr)(cb + 64 * (TS::kPieceCopiesPerWave + j)), 4, 0, 0);
      };
      auto issue = [&](auto ybuf, int G) {
        constexpr int Y = decltype(ybuf)::value;
        u32x4* buf = Y == 0 ? lds_buf0 : (Y == 1 ? lds_buf1 : lds_buf2);
        u32x4* stage = buf + TS::wave_tile(w) * (TS::kStageBytes / 16);
        if constexpr (kCodes) {
          // this group's codes (array Y, fetched two groups ago), then the
          // codes of group G + 2 into the array whose group is already issued
          const int32_t* cb = (Y == 0 ? lds_code0 : (Y == 1 ? lds_code1 : lds_code2)) + w * kCodeCopies * 64;
#pragma unroll
          for (int j = 0; j < TS::kPieceCopiesPerWave; ++j)
            TS::copy_piece_row(P.D.vecs, (int64_t)cb[64 * j + l], stage, TS::wave_piece(w, j), l);
#pragma unroll
          for (int j = 0; j < TS::kScaleCopiesPerWave; ++j)
            __builtin_amdgcn_global_load_lds(P.D.scales + cb[64 * (TS::kPieceCopiesPerWave + j) + l],
                                             (lds_void_ptr)(stage + TS::kTileBytes / 16), 4, 0, 0);
          fetch_codes(std::integral_constant<int, (Y + 2) % 3>{}, G + 2);
        } else {
          int k, rs, re;
          locate(min(G * kGroup + TS::wave_tile(w), n_tiles - 1), k, rs, re);
#pragma unroll
          for (int j = 0; j < TS::kPieceCopiesPerWave; ++j)
            TS::copy_piece(P.D.vecs, base, rs, re, k, stage, TS::wave_piece(w, j), l);
#pragma unroll
          for (int j = 0; j < TS::kScaleCopiesPerWave; ++j) TS::copy_scales(P.D.scales, base, rs, re, k, stage, l);
        }
      };

      // fused top-k: lane l's score (document p0 + l) for query j of the
      // block joins the query's region if its key beats the threshold; a full
      // region keeps its k best first and raises the threshold to the k-th
      auto tk_append = [&](int j, float sc) {
        uint64_t thr = readlane_u64(tk_thr, j);
        int cnt = __builtin_amdgcn_readlane(tk_cnt, j);
        const uint64_t key = tk_rank_key(sc, (int32_t)(p0 + l));
        bool v = l < nd && key > thr;
        uint64_t b = __ballot(v);
        if (b == 0) return;
        int nb = __popcll(b);
        const int cap = P.out.tk.cap;
        uint64_t* R = P.out.tk.keys + ((int64_t)(q0 + j) * tk_regions + tk_piece) * cap;
        if (cnt + nb > cap && cnt > P.out.tk.k) {
          const uint64_t kth = tk_select_k(R, cnt, P.out.tk.k, lds_tk_hist + w * 256);
          unsigned long long old = 0;
          if (l == 0) old = atomicMax(P.out.tk.gthr + q0 + j, (unsigned long long)kth);
          old = readfirstlane_u64(old);
          thr = kth > old ? kth : (uint64_t)old;
          tk_thr = l == j ? thr : tk_thr;
          cnt = P.out.tk.k;
          v = v && key > thr;
          b = __ballot(v);
          nb = __popcll(b);
        }
        const int pos = cnt + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
        if (v && pos < cap) R[pos] = key;                       // (cap bounds every piece by construction)
        cnt = min(cnt + nb, cap);
        tk_cnt = l == j ? cnt : tk_cnt;
      };

      float part = 0.0f;                                        // lane dd: partial score carried to the next pass
      for (int pass = 0; pass < n_pass; ++pass) {
        if (!(b_loaded && n_pass == 1)) {
          // query columns of this pass: owner query, first/last flags, B operand rows
          const int pt0 = pass * NT;
          S.nct = __builtin_amdgcn_readfirstlane(max(0, min(NT, total_tiles - pt0)));
#pragma unroll
          for (int i = 0; i < NT / 4; ++i) S.qs[i] = 1.0f;
          S.tq_lane = 0;
          S.first_mask = 0;
          S.last_mask = 0;
#pragma unroll
          for (int ct = 0; ct < NT; ++ct) {
            O::zero(S.B[ct]);
            if (ct < S.nct) {
              const int t = pt0 + ct;
              const uint64_t own = __ballot(l < nq && qt0 <= t && t < qt0 + qnt);
              const int j = __ffsll((unsigned long long)own) - 1;
              const int jt0 = __builtin_amdgcn_readlane(qt0, j);
              const int jm = __builtin_amdgcn_readlane(qm, j);
              const int64_t jrow = (int64_t)readlane_u64((uint64_t)qrow, j);
              const int k = t - jt0;                            // tile index inside query j
              if (l == ct) S.tq_lane = j;
              if (k == 0) S.first_mask |= 1ull << ct;
              if (16 * (k + 1) >= jm) S.last_mask |= 1ull << ct;
              if (16 * k + c16 < jm) {
                const int64_t vr = vec_row(P.Q, jrow + 16 * k + c16);
                O::load_b(S.B[ct], P.Q.vecs, P.Q.scales, vr, g);
                if constexpr (O::kColumnScale)
                  if (g == (ct & 3)) S.qs[ct >> 2] = P.Q.scales[vr];
              }
            }
          }
          b_loaded = true;
        }
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) S.rm[ct] = ninf;
        __builtin_amdgcn_s_waitcnt(0);                         // operands in; the stream starts from zero

        // group G (in buffer X): wait for this wave's copies of G, publish G
        // with one barrier (which also frees the buffer G - 1 used), start the
        // copies of G + 2 into that buffer, then multiply G's tiles
        auto group = [&](auto xbuf, int G) {
          constexpr int X = decltype(xbuf)::value;
          const u32x4* buf = X == 0 ? lds_buf0 : (X == 1 ? lds_buf1 : lds_buf2);
          wait_vm<kIssueOps>();                                 // only group G + 1's copies may be in flight
          compiler_fence();
          __builtin_amdgcn_s_barrier();
          compiler_fence();
          issue(std::integral_constant<int, (X + 2) % 3>{}, G + 2);
          const int nt = min(kGroup, n_tiles - G * kGroup);       // <= 0 past the end
          const int T0 = G * kGroup;
          // (full passes take the unbranched body)
          auto tiles = [&](auto full) {
            Frag A;
            frag_from_lds<DT>(A, buf, c16, g);
#pragma nounroll
            for (int u = 0; u < nt; ++u)
              S.template tile<decltype(full)::value>(A, buf + min(u + 1, nt - 1) * (TS::kStageBytes / 16), c16, g,
                                                     __ballot(d_tl == T0 + u));
          };
          if (nt > 0) {
            if (S.nct == NT) tiles(std::true_type{});
            else if (S.nct > 0) tiles(std::false_type{});
          }
        };
        if (n_tiles > 0) {
          if constexpr (kCodes) {
            fetch_codes(std::integral_constant<int, 0>{}, 0);
            fetch_codes(std::integral_constant<int, 1>{}, 1);
            wait_vm<0>();                                       // (each wave reads only its own codes)
          }
          issue(std::integral_constant<int, 0>{}, 0);
          issue(std::integral_constant<int, 1>{}, 1);
        }
        // whole triples of groups (the ones past the end hold no tiles), so
        // that every path through the loop issues the same copies
        for (int G = 0; G < n_groups; G += 3) {
          group(std::integral_constant<int, 0>{}, G);
          group(std::integral_constant<int, 1>{}, G + 1);
          group(std::integral_constant<int, 2>{}, G + 2);
        }
        wait_vm<0>();                                           // no copy outlives the pass
        __syncthreads();                                        // buffers are reused by the next pass
        // each query's score: its tile sums in tile order (continuing the
        // partial score of a query that began in the previous pass); finished
        // queries store one row of the chunk's documents each (empty
        // documents score -inf)
        float s_run = part;
        uint64_t fin = 0;                                       // fused top-k: column tiles whose query has news
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
          if (ct < S.nct) {
            const float tv = S.tsum[ct * 64 + l];
            s_run = ((S.first_mask >> ct) & 1) ? tv : s_run + tv;
            if ((S.last_mask >> ct) & 1) {
              if constexpr (kTopk) {
                // the documents that beat the query's threshold join its
                // region; when the region is full, the query is taken below
                // (its region selected first; the score waits in the
                // parked-sum slot, read above)
                const int j = __builtin_amdgcn_readlane(S.tq_lane, ct);
                const float sc = doc_empty ? ninf : s_run;
                const uint64_t key = tk_rank_key(sc, (int32_t)(p0 + l));
                const bool v = l < nd && key > readlane_u64(tk_thr, j);
                const uint64_t b = __ballot(v);
                if (b) {
                  const int cnt = __builtin_amdgcn_readlane(tk_cnt, j);
                  const int nb = __popcll(b);
                  if (cnt + nb <= P.out.tk.cap) {
                    uint64_t* R = P.out.tk.keys + ((int64_t)(q0 + j) * tk_regions + tk_piece) * P.out.tk.cap;
                    if (v) R[cnt + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u))] = key;
                    tk_cnt = l == j ? cnt + nb : tk_cnt;
                  } else {
                    S.tsum[ct * 64 + l] = sc;
                    fin |= 1ull << ct;
                  }
                }
              } else {
                const int j = __builtin_amdgcn_readlane(S.tq_lane, ct);
                const int64_t row = P.out.rows ? (int64_t)P.out.rows[q0 + j] : (int64_t)(q0 + j);
                if (l < nd) P.out.scores[row * P.out.ld + p0 + l] = doc_empty ? ninf : s_run;
              }
            }
          }
        }
        if constexpr (kTopk) {
          // queries whose regions are full: select, then append
          while (fin) {
            const int ct = __builtin_ctzll(fin);
            fin &= fin - 1;
            tk_append(__builtin_amdgcn_readlane(S.tq_lane, ct), S.tsum[ct * 64 + l]);
          }
        }
        part = s_run;
      }
      // empty queries score 0 against every document
      for (int j = 0; j < nq; ++j) {
        if constexpr (kTopk) {
          if (__builtin_amdgcn_readlane(qm, j) == 0) tk_append(j, 0.0f);
        } else if (__builtin_amdgcn_readlane(qm, j) == 0 && l < nd) {
          const int64_t row = P.out.rows ? (int64_t)P.out.rows[q0 + j] : (int64_t)(q0 + j);
          P.out.scores[row * P.out.ld + p0 + l] = 0.0f;
        }
      }
    }
    if constexpr (kTopk) {
      // the piece's entry counts, for the merge
      if (l < nq) P.out.tk.cnt[(int64_t)(q0 + l) * tk_regions + tk_piece] = tk_cnt;
    }
  }
}

// The persistent scorer, and its variant for plans of narrow query blocks
// (small batches): four column tiles a wave, a quarter of the parked-sum LDS
// and of the query registers, compiled for four waves per SIMD (two resident
// workgroups per CU).
template <int DT, bool kCodes, bool kTopk>
__global__ __launch_bounds__(kDenseThreads) void score_dense_kernel(DenseParams P) {
  dense_body<DT, kCodes, 0, kTopk>(P);
}
template <int DT, bool kTopk>
__global__ __launch_bounds__(kDenseThreads, 4) void score_dense_narrow_kernel(DenseParams P) {
  dense_body<DT, false, 4, kTopk>(P);
}

DenseSchedule default_dense_schedule(int dtype, int64_t q_rows, int64_t n_docs, int cus_per_xcd) {
  (void)dtype; (void)q_rows; (void)n_docs;
  DenseSchedule d;
  d.chunk_docs = kMaxChunkDocs;
  d.items_per_slot = 8;
  d.slots_per_xcd = cus_per_xcd;        // one resident workgroup per CU (LDS-bound)
  return d;
}

void topk_fuse_shape(int32_t k, int64_t n_docs, int64_t n_bg_min, int slots_per_xcd, int32_t* np_out,
                     int32_t* cap_out) {
  // enough pieces per XCD that every workgroup of the XCD gets an item
  const int64_t bg = std::max<int64_t>(1, n_bg_min);
  const int64_t np = std::min<int64_t>(64, std::max<int64_t>(1, (slots_per_xcd + bg - 1) / bg));
  // a region holds the k best of its piece plus room for new entries (a
  // selection frees at least 1024 slots, or k when k is larger), unless the
  // piece's documents fit in less: then no selection ever runs
  const int64_t kr = (k + 63) & ~(int64_t)63;
  const int64_t cap_k = kr + std::max<int64_t>(1024, kr);
  int64_t piece_docs = 0;
  for (int64_t cd : {(int64_t)32, (int64_t)kMaxChunkDocs}) {
    const int64_t chunks_xcd = ((n_docs + cd - 1) / cd + 7) / 8;
    piece_docs = std::max(piece_docs, ((chunks_xcd + np - 1) / np) * cd);
  }
  const int64_t cap_p = std::max<int64_t>(64, (piece_docs + 63) & ~(int64_t)63);
  *np_out = (int32_t)np;
  *cap_out = (int32_t)std::min(cap_k, cap_p);
}

bool dense_schedule_valid(const DenseSchedule& d, int cus_per_xcd) {
  return (d.chunk_docs == 32 || d.chunk_docs == 64) && d.items_per_slot >= 1 && d.items_per_slot <= 64 &&
         d.slots_per_xcd >= 1 && d.slots_per_xcd <= cus_per_xcd;
}

template <bool kTopk>
static void launch_dense_variant(int dtype, bool codes, int32_t block_rows, dim3 grid, dim3 blk, const DenseParams& P,
                                 hipStream_t s) {
  switch (dtype) {
    case GEM_F32:
      if (codes) hipLaunchKernelGGL((score_dense_kernel<GEM_F32, true, kTopk>), grid, blk, 0, s, P);
      else hipLaunchKernelGGL((score_dense_kernel<GEM_F32, false, kTopk>), grid, blk, 0, s, P);
      break;
    case GEM_BF16:
      if (codes) hipLaunchKernelGGL((score_dense_kernel<GEM_BF16, true, kTopk>), grid, blk, 0, s, P);
      else hipLaunchKernelGGL((score_dense_kernel<GEM_BF16, false, kTopk>), grid, blk, 0, s, P);
      break;
    case GEM_BF16X3:
      if (codes) hipLaunchKernelGGL((score_dense_kernel<GEM_BF16X3, true, kTopk>), grid, blk, 0, s, P);
      else hipLaunchKernelGGL((score_dense_kernel<GEM_BF16X3, false, kTopk>), grid, blk, 0, s, P);
      break;
    case GEM_FP8_E4M3:
      if (codes) hipLaunchKernelGGL((score_dense_kernel<GEM_FP8_E4M3, true, kTopk>), grid, blk, 0, s, P);
      else if (block_rows <= 64)                             // two workgroups per CU
        hipLaunchKernelGGL((score_dense_narrow_kernel<GEM_FP8_E4M3, kTopk>), dim3(2 * grid.x), blk, 0, s, P);
      else hipLaunchKernelGGL((score_dense_kernel<GEM_FP8_E4M3, false, kTopk>), grid, blk, 0, s, P);
      break;
    case GEM_MXFP4:
      if (codes) hipLaunchKernelGGL((score_dense_kernel<GEM_MXFP4, true, kTopk>), grid, blk, 0, s, P);
      else hipLaunchKernelGGL((score_dense_kernel<GEM_MXFP4, false, kTopk>), grid, blk, 0, s, P);
      break;
    case GEM_MXFP6:
      if (codes) hipLaunchKernelGGL((score_dense_kernel<GEM_MXFP6, true, kTopk>), grid, blk, 0, s, P);
      else hipLaunchKernelGGL((score_dense_kernel<GEM_MXFP6, false, kTopk>), grid, blk, 0, s, P);
      break;
    default: break;
  }
}

hipError_t launch_score_dense(int dtype, const SetsView& Q, const SetsView& D, const int32_t* qb_start,
                              const int64_t* qcol, int64_t n_blocks_max, const DenseOut& out,
                              const DenseSchedule& sched, int32_t block_rows, hipStream_t s) {
  DenseParams P;
  P.Q = Q; P.D = D; P.qb = qb_start; P.qcol = qcol; P.n_blocks_max = n_blocks_max;
  P.n_bgroups = (n_blocks_max + kDenseWaves - 1) / kDenseWaves;
  P.out = out;
  P.chunk0 = 0;
  P.chunk_docs = sched.chunk_docs;
  P.items_per_slot = sched.items_per_slot;
  P.n_chunks = (D.n_sets + sched.chunk_docs - 1) / sched.chunk_docs;
  if (P.n_bgroups == 0 || P.n_chunks == 0) return hipSuccess;
  if (sched.chunk_docs < 1 || sched.chunk_docs > kMaxChunkDocs || sched.items_per_slot < 1 || sched.slots_per_xcd < 1)
    return hipErrorInvalidValue;
  if (dtype != GEM_F32 && dtype != GEM_BF16 && dtype != GEM_BF16X3 && dtype != GEM_FP8_E4M3 && dtype != GEM_MXFP4 &&
      dtype != GEM_MXFP6)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)(8 * sched.slots_per_xcd)), blk(kDenseThreads);
  const bool codes = D.codes != nullptr;
  if (out.tk.k > 0) {
    if (out.tk.np < 1 || out.tk.cap < 64 || (out.tk.cap & 63) || out.tk.cap > kTkMaxCap || 2 * out.tk.k > kTkMaxCap ||
        !out.tk.keys || !out.tk.cnt || !out.tk.gthr)
      return hipErrorInvalidValue;
    launch_dense_variant<true>(dtype, codes, block_rows, grid, blk, P, s);
  } else {
    launch_dense_variant<false>(dtype, codes, block_rows, grid, blk, P, s);
  }
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Gathered scorer: one wave scores up to kGatherEntries consecutive entries of
// one query's candidate list (fewer when a call has too few entries to give
// every CU several waves: an entry's score does not depend on its wave). The query's vectors stay in registers (64 per
// pass). The entries' documents form one sequence of tiles, which the wave
// streams from memory several tiles ahead of the one being multiplied
// (enough loads in flight to cover the memory latency). A score is the same
// sum of per-tile column sums, in tile order, as in the dense scorer.
constexpr int kGatherEntries = 16;
constexpr int kGatherNT = 4;
// Tiles in flight per wave: the choices of each format (registers: a float32
// tile fragment takes 32 VGPRs, a split-bf16 one 32, bf16 16, FP8 9, MXFP6 7,
// MXFP4 5); the middle one is the default.
template <int DT> struct GatherDepths;
template <> struct GatherDepths<GEM_F32> { static constexpr int d[3] = {1, 2, 3}; };
template <> struct GatherDepths<GEM_BF16X3> { static constexpr int d[3] = {1, 2, 3}; };
template <> struct GatherDepths<GEM_BF16> { static constexpr int d[3] = {2, 4, 6}; };
template <> struct GatherDepths<GEM_FP8_E4M3> { static constexpr int d[3] = {4, 6, 8}; };
template <> struct GatherDepths<GEM_MXFP4> { static constexpr int d[3] = {6, 8, 12}; };
template <> struct GatherDepths<GEM_MXFP6> { static constexpr int d[3] = {4, 6, 8}; };

int gather_depth_choice(int dtype, int i) {
  switch (dtype) {
    case GEM_F32: return GatherDepths<GEM_F32>::d[i];
    case GEM_BF16X3: return GatherDepths<GEM_BF16X3>::d[i];
    case GEM_BF16: return GatherDepths<GEM_BF16>::d[i];
    case GEM_FP8_E4M3: return GatherDepths<GEM_FP8_E4M3>::d[i];
    case GEM_MXFP6: return GatherDepths<GEM_MXFP6>::d[i];
    default: return GatherDepths<GEM_MXFP4>::d[i];
  }
}

struct GatherParams {
  SetsView Q, D;
  CandsView C;
  int64_t chunks_per_query;
  int64_t wave0;          // first wave of this launch (large batches launch in slices)
  int32_t entries_per_wave;
  float* scores;
  // range mode: list q is every document of D, in order (no ids), and entry
  // e's score goes to scores[(out_rows ? out_rows[q] : q) * out_ld + e]
  int32_t range;
  const int32_t* out_rows;
  int64_t out_ld;
  // entries of documents with work items in the document-major scorer
  // (skip_items: its item scan) are left to it
  const int32_t* skip_items;
  // reordered lists: each entry's index in the caller's entry array
  const int32_t* out_pos;
  int32_t chunk_major;
};

// kCodes: the documents are a code set. Each lane then loads the code of the
// row it will load PF tiles before that row's load is issued (a second ring of
// PF codes), so tile loads never wait on a dependent load.
template <int DT, bool kCodes, int PF>
__global__ __launch_bounds__(256) void score_gather_kernel(GatherParams P) {
  using O = Op<DT>;
  using Frag = typename O::Frag;
  constexpr int NT = kGatherNT;
  constexpr int PASS = 16 * NT;

  const int l = threadIdx.x & 63, g = l >> 4, c16 = l & 15;
  const int64_t gw = P.wave0 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  int64_t q, ch;
  if (P.chunk_major) {
    q = gw % P.C.n_lists;
    ch = gw / P.C.n_lists;
    if (ch >= P.chunks_per_query) return;
  } else {
    q = gw / P.chunks_per_query;
    if (q >= P.C.n_lists) return;
    ch = gw % P.chunks_per_query;
  }
  int64_t lb, le;
  if (P.range) { lb = 0; le = P.D.n_sets; }
  else if (P.C.off) { lb = P.C.off[q]; le = P.C.off[q + 1]; }
  else { lb = q * (int64_t)P.C.stride; le = lb + P.C.stride; }
  const int64_t e0 = lb + ch * P.entries_per_wave;
  const int64_t e1 = min(le, e0 + P.entries_per_wave);
  if (e0 >= e1) return;
  const int ne = (int)(e1 - e0);
  const float ninf = neg_inf();

  // lane e < ne: the entry's document (first row, length), its first tile in
  // the wave's tile sequence and its last tile (-1 for a padding id or an
  // empty document)
  int32_t my_id = -1;
  int64_t d_beg = 0;
  int d_len = 0;
  bool skip = false;                                   // scored by the document-major scorer
  if (l < ne) {
    my_id = P.range ? (int32_t)(e0 + l) : P.C.ids[e0 + l];
    if (my_id >= 0) {
      // (the skip test's loads go out with the offsets', not before them)
      d_beg = P.D.off[my_id];
      d_len = (int)(P.D.off[my_id + 1] - d_beg);
      if (P.skip_items) skip = P.skip_items[my_id + 1] > P.skip_items[my_id];
      if (skip) d_len = 0;
    }
  }
  const int d_nt = (d_len + 15) >> 4;
  int d_incl = d_nt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(d_incl, o);
    if (l >= o) d_incl += v;
  }
  const int d_t0 = d_incl - d_nt;
  const int d_tl = d_nt > 0 ? d_incl - 1 : -1;
  const int n_tiles = __builtin_amdgcn_readlane(d_incl, 63);

  const int64_t r0 = P.Q.off[q];
  const int m = (int)(P.Q.off[q + 1] - r0);
  // lane e: the entry's score (padding ids and empty documents: -inf; an
  // empty query: 0)
  float res = (my_id < 0 || (d_len == 0 && m > 0)) ? ninf : 0.0f;

  // row of tile T that lane row c16 loads: tile T belongs to the last entry
  // with tiles whose first tile is <= T (T is clamped into the sequence)
  auto tile_row = [&](int T) -> int64_t {
    T = min(T, n_tiles - 1);
    const uint64_t msk = __ballot(d_nt > 0 && d_t0 <= T);
    const int e = 63 - __builtin_clzll(msk);
    const int k = T - __builtin_amdgcn_readlane(d_t0, e);
    const int len = __builtin_amdgcn_readlane(d_len, e);
    const int64_t beg = (int64_t)readlane_u64((uint64_t)d_beg, e);
    return beg + min(16 * k + c16, len - 1);
  };

  if (m > 0 && n_tiles > 0) {
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
          const int64_t vr = vec_row(P.Q, r0 + col);
          O::load_b(B[ct], P.Q.vecs, P.Q.scales, vr, g);
          if constexpr (O::kColumnScale)
            if (g == (ct & 3)) qs[ct >> 2] = P.Q.scales[vr];
        } else {
          O::zero(B[ct]);
        }
      }
      float rm[NT];
#pragma unroll
      for (int ct = 0; ct < NT; ++ct) rm[ct] = ninf;
      // the first PF tiles in flight; then every step multiplies one tile and
      // starts the load PF tiles ahead (past the end: the last tile again,
      // never used, so that every step issues the same loads)
      Frag A[PF];
      int code[PF];                                           // code sets: rows of the tiles PF ahead of A
      if constexpr (kCodes) {
#pragma unroll
        for (int j = 0; j < PF; ++j) code[j] = P.D.codes[tile_row(j)];
#pragma unroll
        for (int j = 0; j < PF; ++j) {
          O::load(A[j], P.D.vecs, P.D.scales, code[j], g);
          code[j] = P.D.codes[tile_row(PF + j)];
          __builtin_amdgcn_sched_barrier(0);                  // keep the loads in tile order
        }
      } else {
#pragma unroll
        for (int j = 0; j < PF; ++j) {
          O::load(A[j], P.D.vecs, P.D.scales, tile_row(j), g);
          __builtin_amdgcn_sched_barrier(0);                  // keep the loads in tile order
        }
      }
      for (int T0 = 0; T0 < n_tiles; T0 += PF) {
#pragma unroll
        for (int j = 0; j < PF; ++j) {
          const int T = T0 + j;
          f32x4 acc[NT];
#pragma unroll
          for (int ct = 0; ct < NT; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
          if (T < n_tiles) {
            // column tiles in pairs, a pair only if the query reaches it (a
            // tile past the query's last vector has zero B operands and its
            // maxima are never summed)
#pragma unroll
            for (int c0 = 0; c0 < NT; c0 += 2) {
              if (c0 < nct) {
#pragma unroll
                for (int s = 0; s < O::kSteps; ++s) {
                  acc[c0] = O::mma(A[j], B[c0], acc[c0], s);
                  acc[c0 + 1] = O::mma(A[j], B[c0 + 1], acc[c0 + 1], s);
                }
              }
            }
          }
          // A[j] is free once its products are issued: load the tile PF ahead
          if constexpr (kCodes) {
            O::load(A[j], P.D.vecs, P.D.scales, code[j], g);
            code[j] = P.D.codes[tile_row(T + 2 * PF)];
          } else {
            O::load(A[j], P.D.vecs, P.D.scales, tile_row(T + PF), g);
          }
          if (T < n_tiles) {
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) update_max(rm[ct], acc[ct]);
            const uint64_t end = __ballot(d_tl == T);
            if (end) {
              const int e = __builtin_ctzll(end);
              float R[NT / 4];
              tile_sums<NT, O::kColumnScale>(rm, R, qs);
              float s_run = first_pass ? tile_sum_at<NT>(R, 0) : readlane_f(res, e) + tile_sum_at<NT>(R, 0);
#pragma unroll
              for (int ct = 1; ct < NT; ++ct)
                if (ct < nct) s_run += tile_sum_at<NT>(R, ct);
              res = writelane_f(res, s_run, e);
#pragma unroll
              for (int ct = 0; ct < NT; ++ct) rm[ct] = ninf;
            }
          }
        }
      }
    }
  }
  if (l < ne && !skip) {
    if (P.range) P.scores[(P.out_rows ? (int64_t)P.out_rows[q] : q) * P.out_ld + e0 + l] = res;
    else P.scores[P.out_pos ? (int64_t)P.out_pos[e0 + l] : e0 + l] = res;
  }
}

template <int DT, int PF>
static void launch_gather_pf(bool codes, dim3 gr, dim3 blk, const GatherParams& P, hipStream_t s) {
  if (codes) hipLaunchKernelGGL((score_gather_kernel<DT, true, PF>), gr, blk, 0, s, P);
  else hipLaunchKernelGGL((score_gather_kernel<DT, false, PF>), gr, blk, 0, s, P);
}

template <int DT>
static bool launch_gather_depth(int depth, bool codes, dim3 gr, dim3 blk, const GatherParams& P, hipStream_t s) {
  using G = GatherDepths<DT>;
  if (depth == G::d[0]) launch_gather_pf<DT, G::d[0]>(codes, gr, blk, P, s);
  else if (depth == G::d[1]) launch_gather_pf<DT, G::d[1]>(codes, gr, blk, P, s);
  else if (depth == G::d[2]) launch_gather_pf<DT, G::d[2]>(codes, gr, blk, P, s);
  else return false;
  return true;
}

bool gather_schedule_valid(int dtype, const GatherSchedule& g) {
  if (g.entries_per_wave != 0 && (g.entries_per_wave < 1 || g.entries_per_wave > 64)) return false;
  if (g.depth == 0) return true;
  for (int i = 0; i < 3; ++i)
    if (g.depth == gather_depth_choice(dtype, i)) return true;
  return false;
}

// Launches the gathered scorer over C.n_lists lists of at most max_list_len
// entries (in slices of at most kMaxGridThreads threads).
static hipError_t run_gather(int dtype, GatherParams P, int64_t max_list_len, const GatherSchedule& g, hipStream_t s) {
  // entries per wave: the schedule's, else kGatherEntries, or as few as one
  // when the call holds fewer than kGatherWaves full waves (a single
  // request's rerank of 1000 candidates then runs on 1000 waves rather than 63)
  constexpr int64_t kGatherWaves = 4096;
  const int64_t cap = P.C.n_lists * std::max<int64_t>(max_list_len, 0);
  if (g.entries_per_wave > 0) P.entries_per_wave = g.entries_per_wave;
  else P.entries_per_wave = cap >= kGatherEntries * kGatherWaves
                                ? kGatherEntries
                                : (int32_t)std::max<int64_t>(1, (cap + kGatherWaves - 1) / kGatherWaves);
  const int depth = g.depth > 0 ? g.depth : gather_depth_choice(dtype, 1);
  P.chunks_per_query = (max_list_len + P.entries_per_wave - 1) / P.entries_per_wave;
  if (P.chunks_per_query == 0 || P.C.n_lists == 0) return hipSuccess;
  const int64_t waves = P.chunks_per_query * P.C.n_lists;
  const int64_t max_blocks = kMaxGridThreads / 256;
  for (int64_t b0 = 0; b0 < (waves + 3) / 4; b0 += max_blocks) {
    P.wave0 = b0 * 4;
    const int64_t grid = std::min(max_blocks, (waves + 3) / 4 - b0);
    const dim3 gr((unsigned)grid), blk(256);
    const bool codes = P.D.codes != nullptr;
    bool ok = false;
    switch (dtype) {
      case GEM_F32: ok = launch_gather_depth<GEM_F32>(depth, codes, gr, blk, P, s); break;
      case GEM_BF16X3: ok = launch_gather_depth<GEM_BF16X3>(depth, codes, gr, blk, P, s); break;
      case GEM_BF16: ok = launch_gather_depth<GEM_BF16>(depth, codes, gr, blk, P, s); break;
      case GEM_FP8_E4M3: ok = launch_gather_depth<GEM_FP8_E4M3>(depth, codes, gr, blk, P, s); break;
      case GEM_MXFP4: ok = launch_gather_depth<GEM_MXFP4>(depth, codes, gr, blk, P, s); break;
      case GEM_MXFP6: ok = launch_gather_depth<GEM_MXFP6>(depth, codes, gr, blk, P, s); break;
      default: break;
    }
    if (!ok) return hipErrorInvalidValue;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_score_gather(int dtype, const SetsView& Q, const SetsView& D, const CandsView& C,
                               int32_t max_list_len, int32_t, float* scores, const GatherSchedule& g, hipStream_t s,
                               const GatherOpts& opts) {
  GatherParams P{};
  P.Q = Q; P.D = D; P.C = C; P.scores = scores;
  P.range = 0;
  P.skip_items = opts.item_start;
  P.out_pos = opts.out_pos;
  P.chunk_major = opts.chunk_major ? 1 : 0;
  return run_gather(dtype, P, max_list_len, g, s);
}

hipError_t launch_score_range(int dtype, const SetsView& Q, const SetsView& D, const DenseOut& out, hipStream_t s) {
  if (D.n_sets > INT32_MAX) return hipErrorInvalidValue;
  GatherParams P{};
  P.Q = Q; P.D = D;
  P.C.off = nullptr; P.C.ids = nullptr; P.C.n_lists = Q.n_sets; P.C.stride = 0;
  P.scores = out.scores; P.out_rows = out.rows; P.out_ld = out.ld;
  P.range = 1;
  return run_gather(dtype, P, D.n_sets, GatherSchedule{}, s);
}

// --------------------------------------------------------------------------
// Candidate lists sorted by document id, one workgroup per list: a bitonic
// sort of (id, position) keys in LDS, padding ids (negative) last.
__global__ __launch_bounds__(256) void sort_lists_kernel(CandsView C, int32_t* __restrict__ sorted_ids,
                                                         int32_t* __restrict__ pos) {
  __shared__ uint64_t key[kSortMaxList];
  const int t = threadIdx.x;
  for (int64_t i = blockIdx.x; i < C.n_lists; i += gridDim.x) {
    const int64_t lb = C.off ? C.off[i] : i * (int64_t)C.stride;
    const int64_t len64 = (C.off ? C.off[i + 1] : lb + C.stride) - lb;
    if (len64 > kSortMaxList) {
      // longer than the stated bound: kept in its order
      for (int64_t j = t; j < len64; j += 256) {
        sorted_ids[lb + j] = C.ids[lb + j];
        pos[lb + j] = (int32_t)(lb + j);
      }
      continue;
    }
    const int len = (int)len64;
    int n = 2;
    while (n < len) n <<= 1;
    for (int j = t; j < n; j += 256)
      key[j] = j < len ? ((uint64_t)(uint32_t)C.ids[lb + j] << 32) | (uint32_t)j : ~0ull;
    __syncthreads();
    for (int k = 2; k <= n; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int x = t; x < (n >> 1); x += 256) {
          const int a = 2 * j * (x / j) + (x % j), b = a + j;
          const uint64_t ka = key[a], kb = key[b];
          if (((a & k) == 0) == (ka > kb)) { key[a] = kb; key[b] = ka; }
        }
        __syncthreads();
      }
    }
    for (int j = t; j < len; j += 256) {
      sorted_ids[lb + j] = (int32_t)(key[j] >> 32);
      pos[lb + j] = (int32_t)(lb + (uint32_t)key[j]);
    }
    __syncthreads();
  }
}

hipError_t launch_sort_lists(const CandsView& C, int32_t max_list_len, int32_t* sorted_ids, int32_t* pos,
                             hipStream_t s) {
  if (C.n_lists == 0 || max_list_len == 0) return hipSuccess;
  if (max_list_len > kSortMaxList || max_list_len < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sort_lists_kernel, dim3(capped_blocks(C.n_lists, 256)), dim3(256), 0, s, C, sorted_ids, pos);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Gathered scoring by document. A batch of shortlists drawn from one corpus
// lists the same documents many times (a rerank of 1000 queries' top-1000
// holds about 26k distinct documents, each about 39 times), and the per-query
// gathered scorer reads a document once per listing. Here the entries are
// grouped by document first:
//   1. count the listings of every document (negative ids are padding: their
//      entries get -inf now and take no further part);
//   2. exclusive scan of the counts (each document's first slot) and of the
//      work items per document (ceil(count / kByDocListings));
//   3. scatter every entry to its document's slots (entry index and query);
//   4. one workgroup per work item stages its document's tiles in LDS once
//      and its waves score the document against the item's listings, each
//      listing query's operands loaded from memory (queries are few and stay
//      in the caches).
// The order of the entries inside a document's slots depends on the atomics,
// but every entry's score is computed on its own, in the gathered scorer's
// arithmetic: the same products, the running max over the document's tiles
// in tile order, the column sums in tile order. So every score is bitwise the
// per-query scorer's.

namespace {
constexpr int kScanBlock = 1024;

// Query of entry e of list i: lists are walked by one wave each.
__global__ __launch_bounds__(256) void bydoc_count_kernel(CandsView C, int64_t n_docs, int32_t* __restrict__ cnt,
                                                          float* __restrict__ scores) {
  const int l = threadIdx.x & 63;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < C.n_lists; i += (int64_t)gridDim.x * 4) {
    const int64_t lb = C.off ? C.off[i] : i * (int64_t)C.stride;
    const int64_t le = C.off ? C.off[i + 1] : lb + C.stride;
    for (int64_t e = lb + l; e < le; e += 64) {
      const int32_t id = C.ids[e];
      if (id < 0 || id >= n_docs) scores[e] = neg_inf();
      else atomicAdd(cnt + id, 1);
    }
  }
}

__global__ __launch_bounds__(256) void bydoc_scatter_kernel(CandsView C, int64_t n_docs,
                                                            const int32_t* __restrict__ item_start,
                                                            const int32_t* __restrict__ start,
                                                            int32_t* __restrict__ cursor,
                                                            int32_t* __restrict__ slot_entry,
                                                            int32_t* __restrict__ slot_query) {
  const int l = threadIdx.x & 63;
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < C.n_lists; i += (int64_t)gridDim.x * 4) {
    const int64_t lb = C.off ? C.off[i] : i * (int64_t)C.stride;
    const int64_t le = C.off ? C.off[i + 1] : lb + C.stride;
    for (int64_t e = lb + l; e < le; e += 64) {
      const int32_t id = C.ids[e];
      if (id < 0 || id >= n_docs || item_start[id + 1] == item_start[id]) continue;
      const int32_t pos = start[id] + atomicAdd(cursor + id, 1);
      slot_entry[pos] = (int32_t)e;
      slot_query[pos] = (int32_t)i;
    }
  }
}

// Work items of each document: ceil(count / kByDocListings), none when its
// listings times its 16-row tiles fall below min_work (min_work <= 1: every
// listed document).
__global__ __launch_bounds__(256) void bydoc_items_kernel(const int32_t* __restrict__ cnt,
                                                          const int64_t* __restrict__ d_off, int64_t n,
                                                          int32_t min_work, int32_t* __restrict__ items) {
  for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < n; d += (int64_t)gridDim.x * 256) {
    const int32_t c = cnt[d];
    const int64_t tiles = (d_off[d + 1] - d_off[d] + 15) >> 4;
    const bool take = c > 0 && (min_work <= 1 || (int64_t)c * tiles >= min_work);
    items[d] = take ? (c + kByDocListings - 1) / kByDocListings : 0;
  }
}

// Document of every work item: items item_start[d] .. item_start[d + 1] - 1
// belong to document d.
__global__ __launch_bounds__(256) void bydoc_item_doc_kernel(const int32_t* __restrict__ item_start, int64_t n,
                                                             int32_t* __restrict__ item_doc) {
  for (int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x; d < n; d += (int64_t)gridDim.x * 256)
    for (int32_t it = item_start[d]; it < item_start[d + 1]; ++it) item_doc[it] = (int32_t)d;
}

// Exclusive scan of blocks of kScanBlock values: out[i] = sum of the block's
// values before i; sums[b] = the block's total.
__global__ __launch_bounds__(kScanBlock) void scan_blocks_kernel(const int32_t* __restrict__ in, int64_t n,
                                                                 int32_t* __restrict__ out,
                                                                 int32_t* __restrict__ sums) {
  __shared__ int32_t buf[kScanBlock];
  const int t = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * kScanBlock + t;
  const int32_t v = i < n ? in[i] : 0;
  buf[t] = v;
  __syncthreads();
  for (int o = 1; o < kScanBlock; o <<= 1) {
    const int32_t a = t >= o ? buf[t - o] : 0;
    __syncthreads();
    buf[t] += a;
    __syncthreads();
  }
  if (i < n) out[i] = buf[t] - v;
  if (t == kScanBlock - 1) sums[blockIdx.x] = buf[t];
}

// Exclusive scan of the block totals in one workgroup (chunks of kScanBlock
// with a running carry); sums[n_blocks] receives the grand total.
__global__ __launch_bounds__(kScanBlock) void scan_sums_kernel(int32_t* __restrict__ sums, int64_t n_blocks) {
  __shared__ int32_t buf[kScanBlock];
  const int t = threadIdx.x;
  int32_t carry = 0;
  for (int64_t c0 = 0; c0 < n_blocks; c0 += kScanBlock) {
    const int64_t i = c0 + t;
    const int32_t v = i < n_blocks ? sums[i] : 0;
    buf[t] = v;
    __syncthreads();
    for (int o = 1; o < kScanBlock; o <<= 1) {
      const int32_t a = t >= o ? buf[t - o] : 0;
      __syncthreads();
      buf[t] += a;
      __syncthreads();
    }
    if (i < n_blocks) sums[i] = carry + buf[t] - v;
    const int32_t tot = buf[kScanBlock - 1];
    __syncthreads();
    carry += tot;
  }
  if (t == 0) sums[n_blocks] = carry;
}

__global__ __launch_bounds__(256) void scan_add_kernel(int32_t* __restrict__ out, int64_t n,
                                                       const int32_t* __restrict__ sums) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[i] += sums[i / kScanBlock];
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = sums[(n + kScanBlock - 1) / kScanBlock];
}

// out[0..n] = exclusive scan of in[0..n) with out[n] the total (sums: scratch
// of n / kScanBlock + 2 values).
hipError_t exclusive_scan(const int32_t* in, int64_t n, int32_t* out, int32_t* sums, hipStream_t s) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb > 0) hipLaunchKernelGGL(scan_blocks_kernel, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, n, out, sums);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kScanBlock), 0, s, sums, nb);
  hipLaunchKernelGGL(scan_add_kernel, dim3(capped_blocks((n + 255) / 256 + 1, 256)), dim3(256), 0, s, out, n,
                     sums);
  return hipGetLastError();
}

constexpr int kByDocWaves = 8;
constexpr int kByDocMaxTiles = kByDocMaxRows / 16;

struct ByDocParams {
  SetsView Q, D;
  const int32_t* start;       // [n_docs + 1] first slot of each document
  const int32_t* item_start;  // [n_docs + 1] first work item of each document
  const int32_t* item_doc;    // document of each work item
  const int32_t* slot_entry;  // entry index of each slot
  const int32_t* slot_query;  // list (query) of each slot
  int64_t n_docs;
  float* scores;
};
}  // namespace

// The running maxima of one pass of the document-major scorer over the staged
// tiles 0..n_tiles-1: the products of each used column tile's query columns
// with every document tile, in the gathered scorer's order (each column
// tile's accumulator takes the K steps in order). With more than two column
// tiles in use the four accumulators advance together, so that consecutive
// products never wait on one another; the next tile's A operand is read while
// the last products finish.
template <int DT, int NB>
__device__ __forceinline__ void bydoc_tiles(typename Op<DT>::Frag A, const typename Op<DT>::Frag (&B)[NB],
                                            float (&rm)[kGatherNT], const u32x4* stage, int n_tiles, int nct,
                                            int c16, int g) {
  using O = Op<DT>;
  using TS = TileStage<DT>;
  static_assert(kGatherNT == 4 && (NB == 2 || NB == 4), "column tiles of a pass");
  for (int T = 0; T < n_tiles; ++T) {
    f32x4 acc[NB];
#pragma unroll
    for (int ct = 0; ct < NB; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (NB > 2 && nct > 2) {
#pragma unroll
      for (int s = 0; s < O::kSteps; ++s) {
#pragma unroll
        for (int ct = 0; ct < NB; ++ct) acc[ct] = O::mma(A, B[ct], acc[ct], s);
      }
    } else {
#pragma unroll
      for (int s = 0; s < O::kSteps; ++s) {
        acc[0] = O::mma(A, B[0], acc[0], s);
        acc[1] = O::mma(A, B[1], acc[1], s);
      }
    }
    if (T + 1 < n_tiles) frag_from_lds<DT>(A, stage + (T + 1) * (TS::kStageBytes / 16), c16, g);
#pragma unroll
    for (int ct = 0; ct < NB; ++ct) update_max(rm[ct], acc[ct]);
  }
}

template <int DT>
__device__ __forceinline__ typename Op<DT>::Frag A_first(const u32x4* stage, int c16, int g) {
  typename Op<DT>::Frag A;
  frag_from_lds<DT>(A, stage, c16, g);
  return A;
}

// NB: column tiles of query operands a wave holds (4, or 2 for the float32
// operands, which then leave room for three waves per SIMD); WAVES: waves of
// a workgroup. The column sums stay in the layout of four column tiles, and a
// listing's sums are added in column-tile order across passes, so every
// variant gives the gathered scorer's scores bitwise.
template <int DT, int NB, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void score_bydoc_kernel(ByDocParams P) {
  using O = Op<DT>;
  using TS = TileStage<DT>;
  using Frag = typename O::Frag;
  constexpr int NT = kGatherNT;
  constexpr int PASS = 16 * NB;
  __shared__ u32x4 stage[kByDocMaxTiles * TS::kStageBytes / 16];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, c16 = l & 15;
  const float ninf = neg_inf();

  // work item -> document and its listings
  const int32_t item = (int32_t)blockIdx.x;
  if (item >= P.item_start[P.n_docs]) return;
  const int64_t d = P.item_doc[item];
  const int32_t s0 = P.start[d] + (item - P.item_start[d]) * kByDocListings;
  const int32_t s1 = min(P.start[d + 1], s0 + kByDocListings);

  // the document's tiles into LDS (rows past its end repeat its last row)
  const int64_t base = P.D.off[d];
  const int d_len = (int)(P.D.off[d + 1] - base);
  const int n_tiles = (d_len + 15) >> 4;
  if (n_tiles > kByDocMaxTiles) {
    // longer than the documents this path takes (the caller's bound was
    // wrong): NaN scores, nothing staged
    for (int32_t sl = s0 + w; sl < s1; sl += WAVES)
      if (l == 0) P.scores[P.slot_entry[sl]] = __int_as_float(0x7fc00000);
    return;
  }
  // the wave's listings s0 + w + WAVES * i (at most 8): lane i holds
  // listing i's entry, query's first row and length, loaded while the
  // document's tiles are in flight
  const int n_mine = s1 > s0 + w ? (s1 - s0 - w + WAVES - 1) / WAVES : 0;
  int32_t my_e = 0, my_q = 0, my_m = 0;
  int64_t my_r0 = 0;
  if (l < n_mine) {
    const int32_t sl = s0 + w + WAVES * l;
    my_e = P.slot_entry[sl];
    my_q = P.slot_query[sl];
  }
  for (int p = w; p < n_tiles * TS::kPieceWaves; p += WAVES) {
    const int k = p / TS::kPieceWaves, role = p % TS::kPieceWaves;
    TS::copy_piece(P.D.vecs, base, 0, d_len, k, stage + k * (TS::kStageBytes / 16), role, l);
  }
  if constexpr (TS::kScales) {
    for (int k = w; k < n_tiles; k += WAVES)
      TS::copy_scales(P.D.scales, base, 0, d_len, k, stage + k * (TS::kStageBytes / 16), l);
  }
  if (l < n_mine) {
    my_r0 = P.Q.off[my_q];
    my_m = (int)(P.Q.off[my_q + 1] - my_r0);
  }
  wait_vm<0>();
  __syncthreads();

  // The wave takes the item's listings s0 + w, s0 + w + WAVES, ...
  // Consecutive ones whose queries fit one pass of PASS columns together
  // share it: listing j takes the column tiles [qc_j, qc_j + qn_j) (qn_j = its
  // query's 16-column tiles), NT in all. A column tile's maxima and sum depend
  // only on that tile's own column values, so a listing's score does not
  // depend on the listings it shares a pass with. A query of more than PASS
  // vectors takes passes of its own.
  int i = 0;
  while (i < n_mine) {
    int32_t ent[NT], qn[NT], qc[NT], qm[NT];
    int64_t qr[NT];
    int nl = 0, ctot = 0;
    bool open = true, alone = false;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      ent[j] = 0; qn[j] = 0; qc[j] = 0; qm[j] = 0; qr[j] = 0;
    }
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      if (open && i < n_mine) {
        const int32_t e = __builtin_amdgcn_readlane(my_e, i);
        const int64_t r0 = (int64_t)readlane_u64((uint64_t)my_r0, i);
        const int m = __builtin_amdgcn_readlane(my_m, i);
        const int n = (m + 15) >> 4;
        if (m > PASS) {
          if (j == 0) {
            ent[0] = e; qr[0] = r0; qm[0] = m; nl = 1; alone = true;
            ++i;
          }
          open = false;
        } else if (ctot + n > NB) {
          open = false;
        } else {
          ent[j] = e; qr[j] = r0; qm[j] = m; qn[j] = n; qc[j] = ctot;
          ctot += n; nl = j + 1;
          ++i;
        }
      }
    }

    if (alone) {
      // one listing in passes of PASS columns
      const int m = qm[0];
      float res = d_len == 0 ? ninf : 0.0f;
      for (int prow0 = 0; prow0 < m && n_tiles > 0; prow0 += PASS) {
        const int pr = min(PASS, m - prow0);
        const int nct = __builtin_amdgcn_readfirstlane((pr + 15) >> 4);
        const bool first_pass = prow0 == 0;
        Frag B[NB];
        float qs[NT / 4];
#pragma unroll
        for (int i = 0; i < NT / 4; ++i) qs[i] = 1.0f;
#pragma unroll
        for (int ct = 0; ct < NB; ++ct) {
          const int col = prow0 + 16 * ct + c16;
          if (ct < nct && col < m) {
            const int64_t vr = vec_row(P.Q, qr[0] + col);
            O::load_b(B[ct], P.Q.vecs, P.Q.scales, vr, g);
            if constexpr (O::kColumnScale)
              if (g == (ct & 3)) qs[ct >> 2] = P.Q.scales[vr];
          } else {
            O::zero(B[ct]);
          }
        }
        float rm[NT];
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) rm[ct] = ninf;
        bydoc_tiles<DT, NB>(A_first<DT>(stage, c16, g), B, rm, stage, n_tiles, nct, c16, g);
        float R[NT / 4];
        tile_sums<NT, O::kColumnScale>(rm, R, qs);
        float s_run = first_pass ? tile_sum_at<NT>(R, 0) : res + tile_sum_at<NT>(R, 0);
#pragma unroll
        for (int ct = 1; ct < NB; ++ct)
          if (ct < nct) s_run += tile_sum_at<NT>(R, ct);
        res = s_run;
      }
      if (l == 0) P.scores[ent[0]] = res;
      continue;
    }

    if (n_tiles == 0 || ctot == 0) {
      // an empty document (-inf, or 0 for an empty query) or empty queries (0)
#pragma unroll
      for (int j = 0; j < NT; ++j)
        if (j < nl && l == 0) P.scores[ent[j]] = (d_len == 0 && qm[j] > 0) ? ninf : 0.0f;
      continue;
    }

    // the group's shared pass
    const int nct = __builtin_amdgcn_readfirstlane(ctot);
    Frag B[NB];
    float qs[NT / 4];
#pragma unroll
    for (int i = 0; i < NT / 4; ++i) qs[i] = 1.0f;
#pragma unroll
    for (int ct = 0; ct < NB; ++ct) {
      int64_t vr = -1;
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        if (j < nl && ct >= qc[j] && ct < qc[j] + qn[j]) {
          const int col = 16 * (ct - qc[j]) + c16;
          if (col < qm[j]) vr = vec_row(P.Q, qr[j] + col);
        }
      }
      if (vr >= 0) {
        O::load_b(B[ct], P.Q.vecs, P.Q.scales, vr, g);
        if constexpr (O::kColumnScale)
          if (g == (ct & 3)) qs[ct >> 2] = P.Q.scales[vr];
      } else {
        O::zero(B[ct]);
      }
    }
    float rm[NT];
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) rm[ct] = ninf;
    bydoc_tiles<DT, NB>(A_first<DT>(stage, c16, g), B, rm, stage, n_tiles, nct, c16, g);
    float R[NT / 4];
    tile_sums<NT, O::kColumnScale>(rm, R, qs);
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      if (j < nl) {
        // the listing's column tiles in order, as a pass of its own sums them
        float res = 0.0f;
        if (qn[j] > 0) {
          res = tile_sum_at<NT>(R, qc[j]);
#pragma unroll
          for (int t = 1; t < NB; ++t)
            if (t < qn[j]) res += tile_sum_at<NT>(R, qc[j] + t);
        }
        if (l == 0) P.scores[ent[j]] = res;
      }
    }
  }
}

// Work items of a call: at most one per kByDocListings listed entries plus
// one per listed document.
static int64_t bydoc_items_bound(int64_t n_docs, int64_t n_entries) {
  return n_entries / kByDocListings + std::min<int64_t>(n_docs, n_entries) + 1;
}

size_t bydoc_ws_bytes(int64_t n_docs, int64_t n_entries) {
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t nd1 = (size_t)n_docs + 1;
  const size_t nb = (size_t)(n_docs + kScanBlock - 1) / kScanBlock + 2;
  return 4 * up(nd1 * 4) + up(nb * 4) + 2 * up((size_t)n_entries * 4) +
         up((size_t)bydoc_items_bound(n_docs, n_entries) * 4);
}

// Listing-tiles from which a document is scored by document in the mixed
// order. Measured on reranks of FP8 top-200 to top-2000 shortlists of 1000
// queries over 100k documents and of 4096 beams of 1000 over 1M documents,
// thresholds 48 to 768: float32 best at 192-384 (below that the short,
// rarely listed beam documents lose to streaming), split bf16 flat from 48 to
// 192, FP8 best at 32-64.
int32_t bydoc_min_work(int dtype) {
  switch (dtype) {
    case GEM_F32: return 192;
    case GEM_BF16X3: return 96;
    default: return 64;
  }
}

hipError_t launch_score_bydoc(int dtype, const SetsView& Q, const SetsView& D, const CandsView& C, int64_t n_entries,
                              float* scores, void* ws, int32_t min_work, GatherOpts* skip, hipStream_t s) {
  if (C.n_lists == 0 || n_entries == 0) return hipSuccess;
  if (D.n_sets <= 0 || D.codes || Q.codes || n_entries > INT32_MAX || D.n_sets > INT32_MAX - 1)
    return hipErrorInvalidValue;
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const int64_t n_docs = D.n_sets;
  const size_t nd1 = (size_t)n_docs + 1;
  char* p = static_cast<char*>(ws);
  int32_t* cnt = reinterpret_cast<int32_t*>(p);        p += up(nd1 * 4);
  int32_t* start = reinterpret_cast<int32_t*>(p);      p += up(nd1 * 4);
  int32_t* items = reinterpret_cast<int32_t*>(p);      p += up(nd1 * 4);
  int32_t* item_start = reinterpret_cast<int32_t*>(p); p += up(nd1 * 4);
  int32_t* sums = reinterpret_cast<int32_t*>(p);       p += up(((size_t)(n_docs + kScanBlock - 1) / kScanBlock + 2) * 4);
  int32_t* slot_entry = reinterpret_cast<int32_t*>(p); p += up((size_t)n_entries * 4);
  int32_t* slot_query = reinterpret_cast<int32_t*>(p); p += up((size_t)n_entries * 4);
  int32_t* item_doc = reinterpret_cast<int32_t*>(p);
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(cnt), n_docs, 0u, s);
  if (e != hipSuccess) return e;
  const unsigned lgrid = capped_blocks((C.n_lists + 3) / 4, 256);
  hipLaunchKernelGGL(bydoc_count_kernel, dim3(lgrid), dim3(256), 0, s, C, n_docs, cnt, scores);
  if ((e = exclusive_scan(cnt, n_docs, start, sums, s)) != hipSuccess) return e;
  if (skip) skip->item_start = item_start;
  hipLaunchKernelGGL(bydoc_items_kernel, dim3(capped_blocks((n_docs + 255) / 256, 256)), dim3(256), 0, s, cnt,
                     D.off, n_docs, min_work, items);
  if ((e = exclusive_scan(items, n_docs, item_start, sums, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(bydoc_item_doc_kernel, dim3(capped_blocks((n_docs + 255) / 256, 256)), dim3(256), 0, s,
                     item_start, n_docs, item_doc);
  if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(cnt), n_docs, 0u, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(bydoc_scatter_kernel, dim3(lgrid), dim3(256), 0, s, C, n_docs, item_start, start, cnt,
                     slot_entry, slot_query);
  ByDocParams P;
  P.Q = Q; P.D = D; P.start = start; P.item_start = item_start; P.item_doc = item_doc; P.slot_entry = slot_entry;
  P.slot_query = slot_query; P.n_docs = n_docs; P.scores = scores;
  // workgroups past the item count exit at once
  const int64_t grid = bydoc_items_bound(n_docs, n_entries);
  if (grid > INT32_MAX) return hipErrorInvalidValue;
  const dim3 gr((unsigned)grid), blk(64 * kByDocWaves), blk12(64 * 12);
  switch (dtype) {
    case GEM_F32: hipLaunchKernelGGL((score_bydoc_kernel<GEM_F32, 2, 12>), gr, blk12, 0, s, P); break;
    case GEM_BF16X3: hipLaunchKernelGGL((score_bydoc_kernel<GEM_BF16X3, 2, 12>), gr, blk12, 0, s, P); break;
    case GEM_BF16: hipLaunchKernelGGL((score_bydoc_kernel<GEM_BF16, 4, kByDocWaves>), gr, blk, 0, s, P); break;
    case GEM_FP8_E4M3: hipLaunchKernelGGL((score_bydoc_kernel<GEM_FP8_E4M3, 4, kByDocWaves>), gr, blk, 0, s, P); break;
    case GEM_MXFP4: hipLaunchKernelGGL((score_bydoc_kernel<GEM_MXFP4, 4, kByDocWaves>), gr, blk, 0, s, P); break;
    case GEM_MXFP6: hipLaunchKernelGGL((score_bydoc_kernel<GEM_MXFP6, 4, kByDocWaves>), gr, blk, 0, s, P); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gem
