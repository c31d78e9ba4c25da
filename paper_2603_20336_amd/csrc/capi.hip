// C ABI of the scoring library (declared in include/gem.h): argument checks,
// workspace layout and the kernel sequence of each entry point.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gem_internal.h"

using namespace gem;

struct gem_ctx_s {
  int device;
  int n_cu;
  char arch[64];
  // dense-scorer schedules installed by gem_set_dense_schedule / gem_autotune_dense,
  // keyed by (dtype, shape class)
  std::mutex mu;
  std::map<uint64_t, gem::DenseSchedule> dense;
  // gathered-scorer schedules (gem_set_gather_schedule / gem_autotune_gather),
  // keyed by (dtype, class of the list count, class of the longest list)
  std::map<uint64_t, gem::GatherSchedule> gather;
  int32_t topk_mode = GEM_TOPK_AUTO;     // GEM_OPT_TOPK_FUSION
  int32_t gather_order = GEM_GATHER_AUTO;  // GEM_OPT_GATHER_ORDER
  void* scratch = nullptr;               // this device's copy of `scratch` (gem_score_quant_static)
  bool check = false;                    // GEM_OPT_CHECK: validate device inputs before computing
  unsigned long long check_bad = 0;      // violations since the last gem_check_status (under mu)
};

// Device memory that gem_score_quant_static uses as its workspace, for callers
// that cannot allocate. Each device the library runs on holds its own copy
// until the process ends; every call on a device shares it.
static __device__ __align__(256) unsigned char scratch[GEM_STATIC_SCRATCH_BYTES];

namespace {

thread_local std::string g_last_error;

gem_status fail(gem_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
gem_status fail(gem_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

gem_status hip_fail(hipError_t e, const char* what) {
  return fail(GEM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

int row_bytes(int dtype) {
  switch (dtype) {
    case GEM_F32: return 4 * GEM_DIM;
    case GEM_BF16X3: return 4 * GEM_DIM;
    case GEM_BF16: return 2 * GEM_DIM;
    case GEM_FP8_E4M3: return GEM_DIM;
    case GEM_MXFP4: return GEM_DIM / 2;
    case GEM_MXFP6: return GEM_DIM * 3 / 4;
    default: return 0;
  }
}

bool mx_dtype(int32_t d) { return d == GEM_MXFP4 || d == GEM_MXFP6; }
bool valid_dtype(int32_t d) {
  return d == GEM_F32 || d == GEM_BF16 || d == GEM_BF16X3 || d == GEM_FP8_E4M3 || mx_dtype(d);
}
// Formats that carry a 32-bit scale word per row.
bool scaled_dtype(int32_t d) { return d == GEM_FP8_E4M3 || mx_dtype(d); }
bool quant_dtype(int32_t d) { return d == GEM_FP8_E4M3 || mx_dtype(d); }

gem_status check_sets(const gem_sets* S, const char* name, bool need_max_len) {
  if (!S) return fail(GEM_ERR_INVALID, "%s is NULL", name);
  if (!valid_dtype(S->dtype)) return fail(GEM_ERR_INVALID, "%s: unknown dtype %d", name, S->dtype);
  if (S->dim != GEM_DIM) return fail(GEM_ERR_UNSUPPORTED, "%s: dim %d (only %d is supported)", name, S->dim, GEM_DIM);
  if (S->n_sets < 0 || S->n_vecs < 0) return fail(GEM_ERR_INVALID, "%s: negative size", name);
  if (S->n_sets > INT32_MAX - 1) return fail(GEM_ERR_UNSUPPORTED, "%s: more than 2^31-2 sets", name);
  if (S->n_sets > 0 && !S->offsets) return fail(GEM_ERR_INVALID, "%s: offsets is NULL", name);
  if (S->n_vecs > 0 && !S->vecs) return fail(GEM_ERR_INVALID, "%s: vecs is NULL", name);
  if (scaled_dtype(S->dtype) && S->n_vecs > 0 && !S->scales)
    return fail(GEM_ERR_INVALID, "%s: FP8 and MX sets need scales", name);
  if (S->max_set_len < 0) return fail(GEM_ERR_INVALID, "%s: negative max_set_len", name);
  if (need_max_len && S->max_set_len > GEM_MAX_QUERY_LEN)
    return fail(GEM_ERR_UNSUPPORTED, "%s: max_set_len %d exceeds %d", name, S->max_set_len, GEM_MAX_QUERY_LEN);
  if (need_max_len && S->n_vecs > 0 && S->max_set_len == 0 && S->n_sets > 0)
    return fail(GEM_ERR_INVALID, "%s: max_set_len must bound the set lengths", name);
  if (S->codes) {
    if (S->codebook_rows <= 0 && S->n_vecs > 0) return fail(GEM_ERR_INVALID, "%s: code set with an empty codebook", name);
    if (S->codebook_rows > INT32_MAX) return fail(GEM_ERR_UNSUPPORTED, "%s: codebook of more than 2^31-1 rows", name);
    if (S->codebook_rows > 0 && !S->vecs) return fail(GEM_ERR_INVALID, "%s: codebook (vecs) is NULL", name);
    if (scaled_dtype(S->dtype) && S->codebook_rows > 0 && !S->scales)
      return fail(GEM_ERR_INVALID, "%s: FP8 and MX codebooks need scales", name);
  } else if (S->codebook_rows != 0) {
    return fail(GEM_ERR_INVALID, "%s: codebook_rows set without codes", name);
  }
  return GEM_OK;
}

// Rows of S's vector array: the codebook of a code set, else one per entry.
int64_t vec_rows(const gem_sets* S) { return S->codes ? S->codebook_rows : S->n_vecs; }

gem_status check_cands(const gem_cands* C, int64_t n_q) {
  if (C->n_lists != n_q) return fail(GEM_ERR_INVALID, "cands: n_lists %lld != number of query sets %lld",
                                     (long long)C->n_lists, (long long)n_q);
  if (C->n_entries < 0) return fail(GEM_ERR_INVALID, "cands: negative n_entries");
  if (C->n_entries > 0 && !C->ids) return fail(GEM_ERR_INVALID, "cands: ids is NULL");
  if (C->offsets) {
    if (C->n_entries > 0 && C->max_list_len <= 0)
      return fail(GEM_ERR_INVALID, "cands: max_list_len must bound the list lengths");
  } else {
    if (C->stride < 0) return fail(GEM_ERR_INVALID, "cands: negative stride");
    if ((int64_t)C->stride * n_q > C->n_entries)
      return fail(GEM_ERR_INVALID, "cands: n_lists * stride exceeds n_entries");
  }
  return GEM_OK;
}

int32_t list_len_bound(const gem_cands* C) { return C->offsets ? C->max_list_len : C->stride; }

SetsView view(const gem_sets* S) {
  SetsView v;
  v.off = S->offsets; v.vecs = S->vecs; v.scales = S->scales; v.codes = S->codes; v.n_sets = S->n_sets;
  return v;
}

CandsView cview(const gem_cands* C) {
  CandsView v;
  v.off = C->offsets; v.ids = C->ids; v.n_lists = C->n_lists; v.stride = C->stride;
  return v;
}

// Query batches up to this size take the streamed (gathered) path of a dense
// call: at most this many passes over the corpus, each at memory speed. FP8
// batches of two or more queries do better on the dense scorer's narrow-block
// variant (two workgroups per CU), other formats only from four queries on.
constexpr int64_t kRangeMaxQueries = 3;
constexpr int64_t kRangeMaxQueriesFp8 = 1;

// Largest k of the top-k fused into the dense scorer (a region holds the k best
// plus as many free entries).
constexpr int32_t kTopkFusedMaxK = 1024;

bool range_call(const gem_sets* Q, int32_t compute) {
  return Q->n_sets <= (compute == GEM_FP8_E4M3 ? kRangeMaxQueriesFp8 : kRangeMaxQueries);
}

// How a gathered call walks its entries: 0, by query; 1, every listed
// document by document (the caller's choice); else the mixed order of auto,
// in which documents with at least that many listing-tiles (listings x 16-row
// tiles) are scored by document and the rest by query. Auto mixes when the
// lists hold at least two entries per corpus document in float32 and split
// bf16, four in the cheaper formats (below that few documents can reach the
// threshold, and the counting sort costs more than it can save: on 2.1M
// random FP8 entries over 1M documents it took the call from 3.6 to 5.3 ms).
// Documents must be bounded by kByDocMaxRows (D->max_set_len), without code
// sets.
int64_t bydoc_min_entries_per_doc(int32_t compute) {
  return compute == GEM_F32 || compute == GEM_BF16X3 ? 2 : 4;
}

int32_t bydoc_min_work_of(const gem_sets* Q, const gem_sets* D, const gem_cands* C, int32_t gather_order,
                          int32_t compute) {
  if (!C || gather_order == GEM_GATHER_BY_QUERY) return 0;
  const bool ok = !D->codes && !Q->codes && D->n_sets > 0 && D->n_sets < INT32_MAX && D->max_set_len >= 1 &&
                  D->max_set_len <= kByDocMaxRows && C->n_entries > 0 && C->n_entries <= INT32_MAX &&
                  C->n_lists <= INT32_MAX;
  if (!ok) return 0;
  if (gather_order == GEM_GATHER_BY_DOCUMENT) return 1;
  return C->n_entries >= bydoc_min_entries_per_doc(compute) * D->n_sets ? bydoc_min_work(compute) : 0;
}

// A gathered call large enough for the gathered scorer's full split (16
// entries a wave), with lists that fit the sort and documents that are rows
// (not code sets), scores its lists sorted by document id and walks them
// chunk-major: the listings of a document then run close together and find
// its rows in the Infinity Cache. An expansion step of 4096 lists of 512
// random ids over 1M documents: the FP8 gather 3.33 -> 3.06 ms, MXFP4 1.73 ->
// 1.58, MXFP6 2.55 -> 2.27 (the sort 0.05 ms); the float32 rerank of the FP8
// top-1000 in the query order 18.1 -> 16.1 ms; code sets gain nothing.
constexpr int64_t kSortMinEntries = 65536;

bool sorted_walk(const gem_sets* D, const gem_cands* C) {
  const int64_t len = list_len_bound(C);
  return !D->codes && len >= 1 && len <= kSortMaxList && C->n_lists * len >= kSortMinEntries &&
         C->n_entries <= INT32_MAX;
}

// Workspace layout of a scoring call.
struct ScoreLayout {
  size_t q_conv = 0, q_scales = 0, qb = 0, qcol = 0, staged = 0, total = 0;
  int32_t bydoc_work = 0;       // see bydoc_min_work_of
  size_t bydoc_ws = 0;
  // candidate lists sorted by document id and walked chunk-major (sorted_walk)
  bool sorted = false;
  size_t sort_ids = 0, sort_pos = 0;
  int64_t n_blocks_max = 0;
  int block_rows = 0;
  // fused top-k of a dense call (k > 0 without a score matrix): regions,
  // their entry counts and the per-query bounds
  bool fused = false;
  int32_t tk_np = 0, tk_cap = 0;
  size_t tk_keys = 0, tk_cnt = 0, tk_gthr = 0;
};

ScoreLayout score_layout(const gem_sets* Q, const gem_sets* D, const gem_cands* C, int32_t compute, int32_t k,
                         bool scores_given, int slots_per_xcd, int32_t topk_mode = GEM_TOPK_AUTO,
                         int32_t gather_order = GEM_GATHER_BY_QUERY) {
  ScoreLayout L;
  size_t off = 0;
  if (Q->dtype != compute) {
    L.q_conv = off;
    off = align_up(off + (size_t)vec_rows(Q) * row_bytes(compute));
    if (scaled_dtype(compute)) {
      L.q_scales = off;
      off = align_up(off + (size_t)vec_rows(Q) * 4);
    }
  }
  if (!C) {
    L.block_rows = dense_block_rows_for(compute, Q->max_set_len, Q->n_sets, Q->n_vecs);
    L.n_blocks_max = dense_blocks_upper(Q->n_sets, Q->n_vecs, L.block_rows, Q->max_set_len);
    L.qb = off;
    off = align_up(off + (size_t)(L.n_blocks_max + 2) * 4);     // starts, end, run count
    L.qcol = off;
    off = align_up(off + (size_t)(Q->n_sets + 1) * 8);
    if (k > 0 && !scores_given) {
      // the top-k fused into the dense scorer, unless staging the score rows
      // takes less memory (small batches; the streamed path always stages)
      const size_t staged = (size_t)Q->n_sets * (size_t)D->n_sets * 4;
      if (topk_mode != GEM_TOPK_STAGED && D->n_sets > 0 && k <= kTopkFusedMaxK &&
          (topk_mode == GEM_TOPK_FUSED || !range_call(Q, compute))) {
        const bool narrow = compute == GEM_FP8_E4M3 && L.block_rows <= 64 && !D->codes;
        const int64_t bg_min = std::max<int64_t>(1, (Q->n_vecs + 8LL * L.block_rows - 1) / (8LL * L.block_rows));
        topk_fuse_shape(k, D->n_sets, bg_min, (narrow ? 2 : 1) * slots_per_xcd, &L.tk_np, &L.tk_cap);
        const size_t regions = (size_t)Q->n_sets * 8 * (size_t)L.tk_np;
        const size_t fused = regions * (size_t)L.tk_cap * 8 + regions * 4 + (size_t)Q->n_sets * 8 + 3 * 256;
        L.fused = topk_mode == GEM_TOPK_FUSED || fused < staged;
      }
      if (L.fused) {
        const size_t regions = (size_t)Q->n_sets * 8 * (size_t)L.tk_np;
        L.tk_keys = off;
        off = align_up(off + regions * (size_t)L.tk_cap * 8);
        L.tk_cnt = off;
        off = align_up(off + regions * 4);
        L.tk_gthr = off;
        off = align_up(off + (size_t)Q->n_sets * 8);
      } else {
        L.staged = off;
        off = align_up(off + staged);
      }
    }
  } else {
    if (k > 0 && !scores_given) {
      L.staged = off;
      off = align_up(off + (size_t)C->n_entries * 4);
    }
    L.bydoc_work = bydoc_min_work_of(Q, D, C, gather_order, compute);
    if (L.bydoc_work > 0) {
      L.bydoc_ws = off;
      off = align_up(off + bydoc_ws_bytes(D->n_sets, C->n_entries));
    }
    // (not in the mixed order: its per-query entries are the rarely listed
    // documents, which the sort cannot bring together, while the chunk-major
    // walk loses the reuse of each query's operands: the float32 rerank of
    // the FP8 top-1000 took 16.4 ms sorted against 15.7)
    L.sorted = L.bydoc_work == 0 && sorted_walk(D, C);
    if (L.sorted) {
      L.sort_ids = off;
      off = align_up(off + (size_t)C->n_entries * 4);
      L.sort_pos = off;
      off = align_up(off + (size_t)C->n_entries * 4);
    }
  }
  L.total = off;
  return L;
}

char* at(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

// The sorted walk of a gathered call (L.sorted): the lists sorted into the
// workspace, *cv reading them and *opts writing each score back to its
// entry's position in the caller's list.
hipError_t sort_for_walk(const ScoreLayout& L, void* ws, int32_t max_list_len, CandsView* cv, GatherOpts* opts,
                         hipStream_t stream) {
  if (!L.sorted) return hipSuccess;
  int32_t* sid = reinterpret_cast<int32_t*>(at(ws, L.sort_ids));
  int32_t* spos = reinterpret_cast<int32_t*>(at(ws, L.sort_pos));
  hipError_t e = launch_sort_lists(*cv, max_list_len, sid, spos, stream);
  if (e != hipSuccess) return e;
  cv->ids = sid;
  opts->out_pos = spos;
  opts->chunk_major = true;
  return hipSuccess;
}



gem_status convert_query(const gem_sets* Q, int32_t compute, void* ws, const ScoreLayout& L, gem_sets* Qc,
                         hipStream_t stream) {
  *Qc = *Q;
  if (Q->dtype == compute) return GEM_OK;
  if (Q->dtype != GEM_F32) return fail(GEM_ERR_INVALID, "Q: dtype must be F32 or the compute dtype");
  hipError_t e;
  // (a code set converts its codebook; the codes stay as they are)
  if (compute == GEM_BF16) {
    e = launch_convert_bf16(static_cast<const float*>(Q->vecs), vec_rows(Q) * GEM_DIM,
                            reinterpret_cast<uint16_t*>(at(ws, L.q_conv)), stream);
  } else if (compute == GEM_BF16X3) {
    e = launch_split_bf16x3(static_cast<const float*>(Q->vecs), vec_rows(Q),
                            reinterpret_cast<uint16_t*>(at(ws, L.q_conv)), stream);
  } else if (mx_dtype(compute)) {
    e = (compute == GEM_MXFP4 ? launch_quantize_mxfp4 : launch_quantize_mxfp6)(
        static_cast<const float*>(Q->vecs), vec_rows(Q), reinterpret_cast<uint8_t*>(at(ws, L.q_conv)),
        reinterpret_cast<uint8_t*>(at(ws, L.q_scales)), stream);
    Qc->scales = reinterpret_cast<const float*>(at(ws, L.q_scales));
  } else {
    e = launch_quantize_fp8(static_cast<const float*>(Q->vecs), vec_rows(Q), reinterpret_cast<uint8_t*>(at(ws, L.q_conv)),
                            reinterpret_cast<float*>(at(ws, L.q_scales)), stream);
    Qc->scales = reinterpret_cast<const float*>(at(ws, L.q_scales));
  }
  if (e != hipSuccess) return hip_fail(e, "query conversion");
  Qc->dtype = compute;
  Qc->vecs = at(ws, L.q_conv);
  return GEM_OK;
}

int log2_class(int64_t v) {
  int c = 0;
  while (v > 1 && c < 62) { v >>= 1; ++c; }
  return c;
}

// Shape class of a dense call: dtype, and the power-of-two classes of the
// query batch's rows and of the document count.
uint64_t dense_key(int32_t dtype, int64_t q_rows, int64_t n_docs) {
  return ((uint64_t)(uint32_t)dtype << 16) | ((uint64_t)log2_class(q_rows + 1) << 8) |
         (uint64_t)log2_class(n_docs + 1);
}

uint64_t gather_key(int32_t dtype, int64_t n_lists, int64_t max_list_len) {
  return ((uint64_t)(uint32_t)dtype << 16) | ((uint64_t)log2_class(n_lists + 1) << 8) |
         (uint64_t)log2_class(max_list_len + 1);
}

GatherSchedule lookup_gather(gem_ctx ctx, int32_t dtype, int64_t n_lists, int64_t max_list_len) {
  std::lock_guard<std::mutex> g(ctx->mu);
  auto it = ctx->gather.find(gather_key(dtype, n_lists, max_list_len));
  return it != ctx->gather.end() ? it->second : GatherSchedule{};
}

DenseSchedule lookup_dense(gem_ctx ctx, int32_t dtype, int64_t q_rows, int64_t n_docs) {
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    auto it = ctx->dense.find(dense_key(dtype, q_rows, n_docs));
    if (it != ctx->dense.end()) return it->second;
  }
  return default_dense_schedule(dtype, q_rows, n_docs, ctx->n_cu / 8);
}

// GEM_CHECK mode: validates the call's device inputs (offsets, scales, codes,
// ids, finite float32 values) before anything is computed; returns
// GEM_ERR_DEVICE_CHECK (and counts the violations for gem_check_status) when
// they are bad. Synchronizes the stream; does nothing when the mode is off.
gem_status device_check(gem_ctx ctx, const gem_sets* A, const gem_sets* B, const gem_cands* C, int64_t cand_sets,
                        hipStream_t stream, const char* what);

gem_status score_common(gem_ctx ctx, const gem_sets* Q, const gem_sets* D, const gem_cands* C, int32_t compute,
                        int32_t k, float* scores, int64_t ld_scores, const int32_t* score_rows, float* top_scores,
                        int32_t* top_ids, void* ws, size_t ws_bytes, hipStream_t stream,
                        const DenseSchedule* sched = nullptr, const GatherSchedule* gsched = nullptr) {
  gem_status st;
  if ((st = check_sets(Q, "Q", true)) != GEM_OK) return st;
  if ((st = check_sets(D, "D", false)) != GEM_OK) return st;
  if (D->dtype != compute) return fail(GEM_ERR_INVALID, "D: dtype %d does not match the compute dtype %d", D->dtype, compute);
  if (Q->dtype != compute && Q->dtype != GEM_F32)
    return fail(GEM_ERR_INVALID, "Q: dtype must be F32 or the compute dtype");
  if (k < 0 || k > GEM_MAX_K) return fail(GEM_ERR_INVALID, "k = %d outside [0, %d]", k, GEM_MAX_K);
  if (k > 0 && (!top_scores || !top_ids)) return fail(GEM_ERR_INVALID, "k > 0 needs top_scores and top_ids");
  if (k == 0 && !scores) return fail(GEM_ERR_INVALID, "k == 0 needs a scores buffer");
  if (C && (st = check_cands(C, Q->n_sets)) != GEM_OK) return st;
  if (!C) {
    if (ld_scores == 0) ld_scores = D->n_sets;
    if (ld_scores < D->n_sets) return fail(GEM_ERR_INVALID, "ld_scores %lld < number of documents",
                                           (long long)ld_scores);
  }
  const ScoreLayout L = score_layout(Q, D, C, compute, k, scores != nullptr, ctx->n_cu / 8, ctx->topk_mode,
                                     gsched ? (int32_t)GEM_GATHER_BY_QUERY : ctx->gather_order);
  if (ws_bytes < L.total) return fail(GEM_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, L.total);
  if (L.total > 0 && !ws) return fail(GEM_ERR_INVALID, "workspace is NULL");
  if (Q->n_sets == 0) return GEM_OK;
  if ((st = device_check(ctx, Q, D, C, D->n_sets, stream, "scoring")) != GEM_OK) return st;

  gem_sets Qc;
  if ((st = convert_query(Q, compute, ws, L, &Qc, stream)) != GEM_OK) return st;
  hipError_t e;
  if (!C) {
    if (D->n_sets == 0) {
      if (k > 0) {
        e = launch_beam_reset(top_scores, top_ids, Q->n_sets * (int64_t)k, stream);
        if (e != hipSuccess) return hip_fail(e, "top-k padding");
      }
      return GEM_OK;
    }
    DenseOut out{};
    if (L.fused) {
      // top-k fused into the scorer: cleared region counts and bounds
      const int64_t regions = Q->n_sets * 8 * (int64_t)L.tk_np;
      out.tk.k = k; out.tk.cap = L.tk_cap; out.tk.np = L.tk_np;
      out.tk.keys = reinterpret_cast<uint64_t*>(at(ws, L.tk_keys));
      out.tk.cnt = reinterpret_cast<int32_t*>(at(ws, L.tk_cnt));
      out.tk.gthr = reinterpret_cast<unsigned long long*>(at(ws, L.tk_gthr));
      e = launch_fill_u32(reinterpret_cast<uint32_t*>(out.tk.cnt), regions, 0u, stream);
      if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<uint32_t*>(out.tk.gthr), 2 * Q->n_sets, 0u, stream);
      if (e != hipSuccess) return hip_fail(e, "top-k regions");
    } else {
      out.scores = scores ? scores : reinterpret_cast<float*>(at(ws, L.staged));
      out.ld = scores ? ld_scores : D->n_sets;
      out.rows = scores ? score_rows : nullptr;
    }
    if (range_call(Q, compute) && !sched && !L.fused) {
      // a few queries: every document streamed by the gathered scorer (the
      // same scores; the dense scorer would run one lightly loaded block group)
      e = launch_score_range(compute, view(&Qc), view(D), out, stream);
      if (e != hipSuccess) return hip_fail(e, "dense scoring (streamed)");
    } else {
      int32_t* qb = reinterpret_cast<int32_t*>(at(ws, L.qb));
      int64_t* qcol = reinterpret_cast<int64_t*>(at(ws, L.qcol));
      e = launch_plan_query_blocks(Q->offsets, Q->n_sets, L.block_rows, Q->max_set_len, qb, qcol, L.n_blocks_max,
                                   stream);
      if (e != hipSuccess) return hip_fail(e, "query-block plan");
      const DenseSchedule ds = sched ? *sched : lookup_dense(ctx, compute, Q->n_vecs, D->n_sets);
      e = launch_score_dense(compute, view(&Qc), view(D), qb, qcol, L.n_blocks_max, out, ds, L.block_rows, stream);
      if (e != hipSuccess) return hip_fail(e, "dense scoring");
    }
    if (L.fused) {
      e = launch_topk_regions(out.tk.keys, out.tk.cnt, Q->n_sets, 8 * L.tk_np, L.tk_cap, k, top_scores, top_ids,
                              stream);
      if (e != hipSuccess) return hip_fail(e, "top-k merge");
    } else if (k > 0) {
      TopkSegs S;
      S.scores = out.scores; S.off = nullptr; S.ids = nullptr; S.rows = out.rows;
      S.n_segs = Q->n_sets; S.len = D->n_sets; S.ld = out.ld;
      e = launch_topk(S, k, top_scores, top_ids, stream);
      if (e != hipSuccess) return hip_fail(e, "top-k");
    }
  } else {
    float* es = scores ? scores : reinterpret_cast<float*>(at(ws, L.staged));
    GatherOpts skip;
    if (L.bydoc_work > 0) {
      e = launch_score_bydoc(compute, view(&Qc), view(D), cview(C), C->n_entries, es, at(ws, L.bydoc_ws),
                             L.bydoc_work, &skip, stream);
      if (e != hipSuccess) return hip_fail(e, "gathered scoring by document");
    }
    if (L.bydoc_work != 1) {
      // the query order, or in the mixed order the entries of the documents
      // with fewer listings
      CandsView cv = cview(C);
      if ((e = sort_for_walk(L, ws, list_len_bound(C), &cv, &skip, stream)) != hipSuccess)
        return hip_fail(e, "candidate sort");
      const GatherSchedule gs = gsched ? *gsched : lookup_gather(ctx, compute, C->n_lists, list_len_bound(C));
      e = launch_score_gather(compute, view(&Qc), view(D), cv, list_len_bound(C), Q->max_set_len, es, gs, stream,
                              skip);
      if (e != hipSuccess) return hip_fail(e, "gathered scoring");
    }
    if (k > 0) {
      TopkSegs S;
      S.scores = es; S.off = C->offsets; S.ids = C->ids; S.rows = nullptr;
      S.n_segs = Q->n_sets; S.len = C->stride; S.ld = C->stride;
      e = launch_topk(S, k, top_scores, top_ids, stream);
      if (e != hipSuccess) return hip_fail(e, "top-k");
    }
  }
  return GEM_OK;
}

__device__ unsigned long long g_validate_bad;

__global__ void validate_offsets_kernel(const int64_t* off, int64_t n, int64_t hi) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i <= n; i += (int64_t)gridDim.x * 256) {
    const int64_t v = off[i];
    bool bad = v < 0 || v > hi;
    if (i > 0 && off[i - 1] > v) bad = true;
    if (bad) atomicAdd(&g_validate_bad, 1ull);
  }
}

__global__ void validate_scales_kernel(const float* s, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const uint32_t u = __float_as_uint(s[i]);
    const uint32_t ex = (u >> 23) & 0xffu;
    if ((u >> 31) || (u & 0x7fffffu) || ex == 0 || ex == 0xffu) atomicAdd(&g_validate_bad, 1ull);
  }
}

__global__ void validate_ids_kernel(const int32_t* ids, int64_t n, int64_t n_sets) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    if (ids[i] >= n_sets) atomicAdd(&g_validate_bad, 1ull);
}

// Indices that must lie in [0, hi).
__global__ void validate_index_kernel(const int32_t* ids, int64_t n, int64_t hi) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    if (ids[i] < 0 || ids[i] >= hi) atomicAdd(&g_validate_bad, 1ull);
}

__global__ void validate_finite_kernel(const float* x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const uint32_t u = __float_as_uint(x[i]);
    if ((u & 0x7f800000u) == 0x7f800000u) atomicAdd(&g_validate_bad, 1ull);
  }
}

// E8M0 byte 0xFF is NaN: no block scale may use it.
__global__ void validate_mx_exps_kernel(const uint32_t* w, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const uint32_t v = w[i];
    bool bad = false;
    for (int b = 0; b < 4; ++b) bad |= ((v >> (8 * b)) & 0xffu) == 0xffu;
    if (bad) atomicAdd(&g_validate_bad, 1ull);
  }
}

__global__ void validate_codes_kernel(const int32_t* codes, int64_t n, int64_t n_rows) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    if (codes[i] < 0 || codes[i] >= n_rows) atomicAdd(&g_validate_bad, 1ull);
}

gem_status run_validation(hipStream_t stream, const char* what) {
  unsigned long long bad = 0;
  hipError_t e = hipMemcpyFromSymbolAsync(&bad, HIP_SYMBOL(g_validate_bad), sizeof(bad), 0, hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return hip_fail(e, "validation read-back");
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "validation sync");
  if (bad) return fail(GEM_ERR_DEVICE_CHECK, "%s: %llu violations", what, bad);
  return GEM_OK;
}

unsigned blocks_for(int64_t n) { return capped_blocks(std::min<int64_t>((n + 255) / 256, 1 << 16), 256); }

// The checks of a set batch, enqueued (the caller resets and reads the word).
hipError_t launch_set_validation(const gem_sets* S, hipStream_t stream) {
  if (S->n_sets > 0)
    hipLaunchKernelGGL(validate_offsets_kernel, dim3(blocks_for(S->n_sets + 1)), dim3(256), 0, stream, S->offsets,
                       S->n_sets, S->n_vecs);
  const int64_t rows = vec_rows(S);
  if (mx_dtype(S->dtype) && rows > 0)
    hipLaunchKernelGGL(validate_mx_exps_kernel, dim3(blocks_for(rows)), dim3(256), 0, stream,
                       reinterpret_cast<const uint32_t*>(S->scales), rows);
  if (S->dtype == GEM_FP8_E4M3 && rows > 0)
    hipLaunchKernelGGL(validate_scales_kernel, dim3(blocks_for(rows)), dim3(256), 0, stream, S->scales, rows);
  if (S->dtype == GEM_F32 && rows > 0)
    hipLaunchKernelGGL(validate_finite_kernel, dim3(blocks_for(rows * GEM_DIM)), dim3(256), 0, stream,
                       static_cast<const float*>(S->vecs), rows * GEM_DIM);
  if (S->codes && S->n_vecs > 0)
    hipLaunchKernelGGL(validate_codes_kernel, dim3(blocks_for(S->n_vecs)), dim3(256), 0, stream, S->codes, S->n_vecs,
                       S->codebook_rows);
  return hipGetLastError();
}

hipError_t launch_cand_validation(const gem_cands* C, int64_t n_sets, hipStream_t stream) {
  if (C->offsets && C->n_lists > 0)
    hipLaunchKernelGGL(validate_offsets_kernel, dim3(blocks_for(C->n_lists + 1)), dim3(256), 0, stream, C->offsets,
                       C->n_lists, C->n_entries);
  if (C->n_entries > 0)
    hipLaunchKernelGGL(validate_ids_kernel, dim3(blocks_for(C->n_entries)), dim3(256), 0, stream, C->ids,
                       C->n_entries, n_sets);
  return hipGetLastError();
}

gem_status reset_validation(hipStream_t stream) {
  const unsigned long long zero = 0;
  hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(g_validate_bad), &zero, sizeof(zero), 0, hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return hip_fail(e, "validation reset");
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "validation reset sync");
  return GEM_OK;
}

// Timing of schedule candidates: each candidate runs once untimed, then
// kRounds rounds of `reps` calls between two events on the caller's stream;
// its time is the median round. A candidate replaces the best so far only
// when it is faster by more than 0.5 %, so the first candidate (the
// incumbent) keeps near ties and timing noise does not flip the choice from
// run to run.
struct Timer {
  static constexpr int kRounds = 3;
  hipStream_t stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  explicit Timer(hipStream_t s) : stream(s) {}
  ~Timer() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
  gem_status init() {
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    return he == hipSuccess ? GEM_OK : hip_fail(he, "hipEventCreate");
  }
  template <class S, class F>
  gem_status pick(const std::vector<S>& cand, F&& run, int reps, S* best, float* best_ms) {
    for (const S& c : cand) {
      gem_status st = run(c);
      if (st != GEM_OK) return st;
      float t[kRounds];
      for (int r = 0; r < kRounds; ++r) {
        hipError_t he = hipEventRecord(e0, stream);
        if (he != hipSuccess) return hip_fail(he, "hipEventRecord");
        for (int i = 0; i < reps; ++i)
          if ((st = run(c)) != GEM_OK) return st;
        if ((he = hipEventRecord(e1, stream)) != hipSuccess) return hip_fail(he, "hipEventRecord");
        if ((he = hipEventSynchronize(e1)) != hipSuccess) return hip_fail(he, "hipEventSynchronize");
        if ((he = hipEventElapsedTime(&t[r], e0, e1)) != hipSuccess) return hip_fail(he, "hipEventElapsedTime");
        t[r] /= (float)reps;
      }
      std::sort(t, t + kRounds);
      const float ms = t[kRounds / 2];
      if (*best_ms < 0.0f || ms < *best_ms * 0.995f) {
        *best_ms = ms;
        *best = c;
      }
    }
    return GEM_OK;
  }
};

// Tune cache: a small JSON document of installed schedules, e.g.
//   {"format": "gem-tune-cache", "version": 1, "entries": [
//     {"arch": "gfx950", "kind": "dense", "dtype": 1, "q_rows_class": 15,
//      "n_docs_class": 16, "chunk_docs": 32, "items_per_slot": 8, "slots_per_xcd": 32},
//     {"arch": "gfx950", "kind": "gather", "dtype": 2, "lists_class": 12,
//      "list_len_class": 9, "entries_per_wave": 16, "depth": 6}]}
// Classes are floor(log2(x + 1)) of the shape numbers the schedule keys use.

std::string arch_base(const char* arch) {
  std::string a(arch);
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

std::string tune_cache_json(gem_ctx ctx) {
  const std::string arch = arch_base(ctx->arch);
  std::string o = "{\"format\": \"gem-tune-cache\", \"version\": 1, \"entries\": [";
  bool first = true;
  char buf[384];
  for (const auto& kv : ctx->dense) {
    std::snprintf(buf, sizeof(buf),
                  "%s\n  {\"arch\": \"%s\", \"kind\": \"dense\", \"dtype\": %u, \"q_rows_class\": %u, "
                  "\"n_docs_class\": %u, \"chunk_docs\": %d, \"items_per_slot\": %d, \"slots_per_xcd\": %d}",
                  first ? "" : ",", arch.c_str(), (unsigned)(kv.first >> 16), (unsigned)((kv.first >> 8) & 0xff),
                  (unsigned)(kv.first & 0xff), kv.second.chunk_docs, kv.second.items_per_slot,
                  kv.second.slots_per_xcd);
    o += buf;
    first = false;
  }
  for (const auto& kv : ctx->gather) {
    std::snprintf(buf, sizeof(buf),
                  "%s\n  {\"arch\": \"%s\", \"kind\": \"gather\", \"dtype\": %u, \"lists_class\": %u, "
                  "\"list_len_class\": %u, \"entries_per_wave\": %d, \"depth\": %d}",
                  first ? "" : ",", arch.c_str(), (unsigned)(kv.first >> 16), (unsigned)((kv.first >> 8) & 0xff),
                  (unsigned)(kv.first & 0xff), kv.second.entries_per_wave, kv.second.depth);
    o += buf;
    first = false;
  }
  o += "\n]}\n";
  return o;
}

// A minimal reader for that document: objects, arrays, strings without
// escapes, integers, true / false / null.
struct JVal {
  enum Kind { NUL, NUM, STR, ARR, OBJ } kind = NUL;
  long long num = 0;
  std::string str;
  std::vector<JVal> arr;
  std::vector<std::pair<std::string, JVal>> obj;
  const JVal* get(const char* k) const {
    for (const auto& kv : obj)
      if (kv.first == k) return &kv.second;
    return nullptr;
  }
};

struct JParser {
  const char* p;
  const char* end;
  int depth = 0;
  void ws() {
    while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
  }
  bool lit(const char* w) {
    const size_t n = std::strlen(w);
    if ((size_t)(end - p) < n || std::strncmp(p, w, n) != 0) return false;
    p += n;
    return true;
  }
  bool str(std::string& out) {
    if (p >= end || *p != '"') return false;
    const char* b = ++p;
    while (p < end && *p != '"') {
      if (*p == '\\') return false;
      ++p;
    }
    if (p >= end) return false;
    out.assign(b, p);
    ++p;
    return true;
  }
  bool val(JVal& v) {
    if (++depth > 16) return false;
    ws();
    bool ok = false;
    if (p < end && *p == '{') {
      ++p;
      v.kind = JVal::OBJ;
      ws();
      if (p < end && *p == '}') { ++p; ok = true; }
      while (!ok) {
        ws();
        std::string k;
        JVal x;
        if (!str(k)) break;
        ws();
        if (p >= end || *p != ':') break;
        ++p;
        if (!val(x)) break;
        v.obj.emplace_back(k, std::move(x));
        ws();
        if (p < end && *p == ',') { ++p; continue; }
        if (p < end && *p == '}') { ++p; ok = true; }
        break;
      }
    } else if (p < end && *p == '[') {
      ++p;
      v.kind = JVal::ARR;
      ws();
      if (p < end && *p == ']') { ++p; ok = true; }
      while (!ok) {
        JVal x;
        if (!val(x)) break;
        v.arr.push_back(std::move(x));
        ws();
        if (p < end && *p == ',') { ++p; continue; }
        if (p < end && *p == ']') { ++p; ok = true; }
        break;
      }
    } else if (p < end && *p == '"') {
      v.kind = JVal::STR;
      ok = str(v.str);
    } else if (p < end && (*p == '-' || (*p >= '0' && *p <= '9'))) {
      v.kind = JVal::NUM;
      std::string digits;
      while (p < end && (digits.empty() ? (*p == '-' || (*p >= '0' && *p <= '9')) : (*p >= '0' && *p <= '9')) &&
             digits.size() < 20)
        digits.push_back(*p++);
      char* q = nullptr;
      v.num = std::strtoll(digits.c_str(), &q, 10);
      ok = q && *q == '\0' && digits != "-";
    } else {
      v.kind = JVal::NUL;
      ok = lit("null") || lit("true") || lit("false");
    }
    --depth;
    return ok;
  }
};

gem_status load_tune_cache(gem_ctx ctx, const char* path, bool missing_ok) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return missing_ok ? GEM_OK : fail(GEM_ERR_INVALID, "cannot read %s", path);
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0 && text.size() < (1u << 24)) text.append(buf, n);
  std::fclose(f);
  JParser P{text.data(), text.data() + text.size()};
  JVal root;
  if (!P.val(root) || root.kind != JVal::OBJ) return fail(GEM_ERR_INVALID, "%s is not a JSON object", path);
  const JVal* fmt = root.get("format");
  const JVal* ent = root.get("entries");
  if (!fmt || fmt->kind != JVal::STR || fmt->str != "gem-tune-cache" || !ent || ent->kind != JVal::ARR)
    return fail(GEM_ERR_INVALID, "%s is not a gem tune cache", path);
  const std::string arch = arch_base(ctx->arch);
  std::map<uint64_t, DenseSchedule> dense;
  std::map<uint64_t, GatherSchedule> gather;
  auto num = [](const JVal& o, const char* k, long long lo, long long hi, long long* out) {
    const JVal* v = o.get(k);
    if (!v || v->kind != JVal::NUM || v->num < lo || v->num > hi) return false;
    *out = v->num;
    return true;
  };
  for (const JVal& e : ent->arr) {
    if (e.kind != JVal::OBJ) return fail(GEM_ERR_INVALID, "%s: an entry is not an object", path);
    const JVal* a = e.get("arch");
    const JVal* kind = e.get("kind");
    if (!a || a->kind != JVal::STR || !kind || kind->kind != JVal::STR)
      return fail(GEM_ERR_INVALID, "%s: an entry lacks arch or kind", path);
    if (a->str != arch) continue;                            // another GPU's schedules
    long long dt = 0, c1 = 0, c2 = 0, x = 0, y = 0, z = 0;
    if (kind->str == "dense") {
      if (!num(e, "dtype", 0, 3, &dt) || !num(e, "q_rows_class", 0, 62, &c1) || !num(e, "n_docs_class", 0, 62, &c2) ||
          !num(e, "chunk_docs", 0, 1 << 20, &x) || !num(e, "items_per_slot", 0, 1 << 20, &y) ||
          !num(e, "slots_per_xcd", 0, 1 << 20, &z))
        return fail(GEM_ERR_INVALID, "%s: malformed dense entry", path);
      const DenseSchedule d{(int32_t)x, (int32_t)y, (int32_t)z};
      if (!dense_schedule_valid(d, ctx->n_cu / 8)) return fail(GEM_ERR_INVALID, "%s: invalid dense schedule", path);
      dense[((uint64_t)dt << 16) | ((uint64_t)c1 << 8) | (uint64_t)c2] = d;
    } else if (kind->str == "gather") {
      if (!num(e, "dtype", 0, 3, &dt) || !num(e, "lists_class", 0, 62, &c1) || !num(e, "list_len_class", 0, 62, &c2) ||
          !num(e, "entries_per_wave", 0, 64, &x) || !num(e, "depth", 0, 64, &y))
        return fail(GEM_ERR_INVALID, "%s: malformed gather entry", path);
      const GatherSchedule g{(int32_t)x, (int32_t)y};
      if (!gather_schedule_valid((int)dt, g)) return fail(GEM_ERR_INVALID, "%s: invalid gather schedule", path);
      gather[((uint64_t)dt << 16) | ((uint64_t)c1 << 8) | (uint64_t)c2] = g;
    } else {
      return fail(GEM_ERR_INVALID, "%s: unknown entry kind %s", path, kind->str.c_str());
    }
  }
  std::lock_guard<std::mutex> g(ctx->mu);
  for (const auto& kv : dense) ctx->dense[kv.first] = kv.second;
  for (const auto& kv : gather) ctx->gather[kv.first] = kv.second;
  return GEM_OK;
}

// Reads back the violation count of the checks enqueued since the reset.
gem_status read_validation(hipStream_t stream, unsigned long long* bad) {
  hipError_t e = hipMemcpyFromSymbolAsync(bad, HIP_SYMBOL(g_validate_bad), sizeof(*bad), 0, hipMemcpyDeviceToHost,
                                          stream);
  if (e != hipSuccess) return hip_fail(e, "validation read-back");
  e = hipStreamSynchronize(stream);
  return e == hipSuccess ? GEM_OK : hip_fail(e, "validation sync");
}

gem_status device_check_extra(gem_ctx ctx, const gem_sets* A, const gem_sets* B, const gem_cands* C,
                              int64_t cand_sets, const int32_t* idx, int64_t n_idx, int64_t idx_hi,
                              const int32_t* idx2, int64_t n_idx2, int64_t idx2_hi, hipStream_t stream,
                              const char* what) {
  if (!ctx->check) return GEM_OK;
  gem_status st = reset_validation(stream);
  if (st != GEM_OK) return st;
  hipError_t e = hipSuccess;
  if (A) e = launch_set_validation(A, stream);
  if (e == hipSuccess && B) e = launch_set_validation(B, stream);
  if (e == hipSuccess && C) e = launch_cand_validation(C, cand_sets, stream);
  if (e == hipSuccess && idx && n_idx > 0) {
    hipLaunchKernelGGL(validate_index_kernel, dim3(blocks_for(n_idx)), dim3(256), 0, stream, idx, n_idx, idx_hi);
    e = hipGetLastError();
  }
  if (e == hipSuccess && idx2 && n_idx2 > 0) {
    hipLaunchKernelGGL(validate_index_kernel, dim3(blocks_for(n_idx2)), dim3(256), 0, stream, idx2, n_idx2, idx2_hi);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return hip_fail(e, "validation launch");
  unsigned long long bad = 0;
  if ((st = read_validation(stream, &bad)) != GEM_OK) return st;
  if (bad) {
    {
      std::lock_guard<std::mutex> g(ctx->mu);
      ctx->check_bad += bad;
    }
    return fail(GEM_ERR_DEVICE_CHECK, "%s: %llu invalid device values (GEM_OPT_CHECK); nothing was computed", what,
                bad);
  }
  return GEM_OK;
}

gem_status device_check(gem_ctx ctx, const gem_sets* A, const gem_sets* B, const gem_cands* C, int64_t cand_sets,
                        hipStream_t stream, const char* what) {
  return device_check_extra(ctx, A, B, C, cand_sets, nullptr, 0, 0, nullptr, 0, 0, stream, what);
}

}  // namespace

extern "C" {

gem_status gem_create(gem_ctx* out, int device, const char* tune_cache_json) {
  if (!out) return fail(GEM_ERR_INVALID, "out is NULL");
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= n) return fail(GEM_ERR_INVALID, "device %d of %d", device, n);
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(GEM_ERR_UNSUPPORTED, "device %d is %s; this library is built for gfx950", device, prop.gcnArchName);
  gem_ctx c = new (std::nothrow) gem_ctx_s;
  if (!c) return fail(GEM_ERR_INVALID, "out of host memory");
  c->device = device;
  c->n_cu = prop.multiProcessorCount;
  // the device address of this device's scratch array (the name itself is a
  // host-side stand-in), taken with the device current
  {
    int prev = 0;
    e = hipGetDevice(&prev);
    if (e == hipSuccess) e = hipSetDevice(device);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    const hipError_t e2 = hipSetDevice(prev);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) {
      delete c;
      return hip_fail(e, "static scratch address");
    }
    c->scratch = p;
  }
  std::snprintf(c->arch, sizeof(c->arch), "%s", prop.gcnArchName);
  if (tune_cache_json) {
    const gem_status st = load_tune_cache(c, tune_cache_json, true);
    if (st != GEM_OK) {
      delete c;
      return st;
    }
  }
  *out = c;
  return GEM_OK;
}

gem_status gem_destroy(gem_ctx ctx) {
  delete ctx;
  return GEM_OK;
}

const char* gem_status_string(gem_status s) {
  switch (s) {
    case GEM_OK: return "GEM_OK";
    case GEM_ERR_INVALID: return "GEM_ERR_INVALID";
    case GEM_ERR_WORKSPACE: return "GEM_ERR_WORKSPACE";
    case GEM_ERR_UNSUPPORTED: return "GEM_ERR_UNSUPPORTED";
    case GEM_ERR_HIP: return "GEM_ERR_HIP";
    case GEM_ERR_DEVICE_CHECK: return "GEM_ERR_DEVICE_CHECK";
    default: return "GEM_ERR_UNKNOWN";
  }
}

const char* gem_last_error(void) { return g_last_error.c_str(); }

const char* gem_version(void) { return "gem-mi355x 0.2 (gfx950)"; }

gem_status gem_set_option(gem_ctx ctx, int32_t option, int64_t value) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  switch (option) {
    case GEM_OPT_TOPK_FUSION:
      if (value != GEM_TOPK_AUTO && value != GEM_TOPK_FUSED && value != GEM_TOPK_STAGED)
        return fail(GEM_ERR_INVALID, "top-k fusion mode %lld", (long long)value);
      ctx->topk_mode = (int32_t)value;
      return GEM_OK;
    case GEM_OPT_GATHER_ORDER:
      if (value != GEM_GATHER_AUTO && value != GEM_GATHER_BY_QUERY && value != GEM_GATHER_BY_DOCUMENT)
        return fail(GEM_ERR_INVALID, "gather order %lld", (long long)value);
      ctx->gather_order = (int32_t)value;
      return GEM_OK;
    case GEM_OPT_CHECK:
      if (value != 0 && value != 1) return fail(GEM_ERR_INVALID, "check mode %lld", (long long)value);
      ctx->check = value != 0;
      return GEM_OK;
    default:
      return fail(GEM_ERR_INVALID, "unknown option %d", option);
  }
}

gem_status gem_check_status(gem_ctx ctx, hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  const hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "stream");
  unsigned long long bad;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    bad = ctx->check_bad;
    ctx->check_bad = 0;
  }
  if (bad) return fail(GEM_ERR_DEVICE_CHECK, "%llu invalid device values in checked calls since the last check", bad);
  return GEM_OK;
}

gem_status gem_get_option(gem_ctx ctx, int32_t option, int64_t* value) {
  if (!ctx || !value) return fail(GEM_ERR_INVALID, "NULL argument");
  switch (option) {
    case GEM_OPT_TOPK_FUSION: *value = ctx->topk_mode; return GEM_OK;
    case GEM_OPT_GATHER_ORDER: *value = ctx->gather_order; return GEM_OK;
    case GEM_OPT_CHECK: *value = ctx->check ? 1 : 0; return GEM_OK;
    default: return fail(GEM_ERR_INVALID, "unknown option %d", option);
  }
}

size_t gem_workspace_bytes(gem_ctx ctx, int32_t op, const gem_sets* Q, const gem_sets* D, const gem_cands* C,
                           int32_t compute, int32_t k, int32_t scores_given) {
  if (!Q || !ctx) return 0;
  switch (op) {
    case GEM_OP_SCORE_EXACT:
    case GEM_OP_SCORE_QUANT: {
      if (!D) return 0;
      const int32_t cd = op == GEM_OP_SCORE_QUANT ? (mx_dtype(D->dtype) ? D->dtype : (int32_t)GEM_FP8_E4M3) : compute;
      return score_layout(Q, D, C, cd, k, scores_given != 0, ctx->n_cu / 8, ctx->topk_mode, ctx->gather_order).total;
    }
    case GEM_OP_EXPAND: {
      if (!D || !C) return 0;
      return score_layout(Q, D, C, mx_dtype(D->dtype) ? D->dtype : (int32_t)GEM_FP8_E4M3, 1, scores_given != 0,
                          ctx->n_cu / 8).total;
    }
    default:
      return 0;
  }
}

gem_status gem_convert_bf16(gem_ctx ctx, const float* x, int64_t n_rows, int32_t dim, uint16_t* out,
                            hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  if (dim != GEM_DIM) return fail(GEM_ERR_UNSUPPORTED, "dim %d (only %d is supported)", dim, GEM_DIM);
  if (n_rows < 0) return fail(GEM_ERR_INVALID, "negative n_rows");
  if (n_rows > 0 && (!x || !out)) return fail(GEM_ERR_INVALID, "NULL buffer");
  hipError_t e = launch_convert_bf16(x, n_rows * GEM_DIM, out, stream);
  return e == hipSuccess ? GEM_OK : hip_fail(e, "bf16 conversion");
}

gem_status gem_split_bf16x3(gem_ctx ctx, const float* x, int64_t n_rows, int32_t dim, uint16_t* out,
                            hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  if (dim != GEM_DIM) return fail(GEM_ERR_UNSUPPORTED, "dim %d (only %d is supported)", dim, GEM_DIM);
  if (n_rows < 0) return fail(GEM_ERR_INVALID, "negative n_rows");
  if (n_rows > 0 && (!x || !out)) return fail(GEM_ERR_INVALID, "NULL buffer");
  hipError_t e = launch_split_bf16x3(x, n_rows, out, stream);
  return e == hipSuccess ? GEM_OK : hip_fail(e, "bf16 split");
}

gem_status gem_quantize_fp8(gem_ctx ctx, const float* x, int64_t n_rows, int32_t dim, uint8_t* out, float* scales,
                            hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  if (dim != GEM_DIM) return fail(GEM_ERR_UNSUPPORTED, "dim %d (only %d is supported)", dim, GEM_DIM);
  if (n_rows < 0) return fail(GEM_ERR_INVALID, "negative n_rows");
  if (n_rows > 0 && (!x || !out || !scales)) return fail(GEM_ERR_INVALID, "NULL buffer");
  hipError_t e = launch_quantize_fp8(x, n_rows, out, scales, stream);
  return e == hipSuccess ? GEM_OK : hip_fail(e, "fp8 quantization");
}

gem_status gem_quantize_mxfp4(gem_ctx ctx, const float* x, int64_t n_rows, int32_t dim, uint8_t* out, uint8_t* exps,
                              hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  if (dim != GEM_DIM) return fail(GEM_ERR_UNSUPPORTED, "dim %d (only %d is supported)", dim, GEM_DIM);
  if (n_rows < 0) return fail(GEM_ERR_INVALID, "negative n_rows");
  if (n_rows > 0 && (!x || !out || !exps)) return fail(GEM_ERR_INVALID, "NULL buffer");
  hipError_t e = launch_quantize_mxfp4(x, n_rows, out, exps, stream);
  return e == hipSuccess ? GEM_OK : hip_fail(e, "mxfp4 quantization");
}

gem_status gem_quantize_mxfp6(gem_ctx ctx, const float* x, int64_t n_rows, int32_t dim, uint8_t* out, uint8_t* exps,
                              hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  if (dim != GEM_DIM) return fail(GEM_ERR_UNSUPPORTED, "dim %d (only %d is supported)", dim, GEM_DIM);
  if (n_rows < 0) return fail(GEM_ERR_INVALID, "negative n_rows");
  if (n_rows > 0 && (!x || !out || !exps)) return fail(GEM_ERR_INVALID, "NULL buffer");
  hipError_t e = launch_quantize_mxfp6(x, n_rows, out, exps, stream);
  return e == hipSuccess ? GEM_OK : hip_fail(e, "mxfp6 quantization");
}

size_t gem_codebook_workspace_bytes(int32_t op, int64_t n_rows, int64_t n_centroids) {
  if (n_rows < 0 || n_centroids < 0) return 0;
  switch (op) {
    case GEM_OP_NEAREST_CENTROID: return nearest_centroid_ws_bytes(n_rows, n_centroids);
    case GEM_OP_CENTROID_UPDATE: return centroid_update_ws_bytes(n_rows, n_centroids);
    default: return 0;
  }
}

gem_status gem_nearest_centroid(gem_ctx ctx, const void* x, int64_t n_rows, const void* centroids, int64_t n_centroids,
                                int32_t dim, int32_t dtype, int32_t* codes, void* ws, size_t ws_bytes,
                                hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  if (dim != GEM_DIM) return fail(GEM_ERR_UNSUPPORTED, "dim %d (only %d is supported)", dim, GEM_DIM);
  if (dtype != GEM_F32 && dtype != GEM_BF16)
    return fail(GEM_ERR_UNSUPPORTED, "nearest centroid runs in F32 or BF16, not dtype %d", dtype);
  if (n_rows < 0 || n_centroids < 0) return fail(GEM_ERR_INVALID, "negative size");
  if (n_centroids > INT32_MAX - 16) return fail(GEM_ERR_UNSUPPORTED, "more than 2^31-17 centroids");
  if (n_rows == 0) return GEM_OK;
  if (n_centroids == 0) return fail(GEM_ERR_INVALID, "no centroids");
  if (!x || !centroids || !codes) return fail(GEM_ERR_INVALID, "NULL buffer");
  const size_t need = nearest_centroid_ws_bytes(n_rows, n_centroids);
  if (ws_bytes < need) return fail(GEM_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
  if (!ws) return fail(GEM_ERR_INVALID, "workspace is NULL");
  hipError_t e = launch_nearest_centroid(dtype, x, n_rows, centroids, n_centroids, codes, ws, ctx->n_cu, stream);
  return e == hipSuccess ? GEM_OK : hip_fail(e, "nearest centroid");
}

gem_status gem_centroid_update(gem_ctx ctx, const float* x, int64_t n_rows, int32_t dim, const int32_t* codes,
                               const float* centroids, int64_t n_centroids, float* new_centroids, int32_t* counts,
                               void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  if (dim != GEM_DIM) return fail(GEM_ERR_UNSUPPORTED, "dim %d (only %d is supported)", dim, GEM_DIM);
  if (n_rows < 0 || n_centroids < 0) return fail(GEM_ERR_INVALID, "negative size");
  if (n_centroids == 0) return n_rows == 0 ? GEM_OK : fail(GEM_ERR_INVALID, "rows without centroids");
  if (!centroids || !new_centroids || (n_rows > 0 && (!x || !codes))) return fail(GEM_ERR_INVALID, "NULL buffer");
  const size_t need = centroid_update_ws_bytes(n_rows, n_centroids);
  if (ws_bytes < need) return fail(GEM_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
  if (!ws) return fail(GEM_ERR_INVALID, "workspace is NULL");
  hipError_t e = launch_centroid_update(x, n_rows, codes, centroids, n_centroids, new_centroids, counts, ws, stream);
  return e == hipSuccess ? GEM_OK : hip_fail(e, "centroid update");
}

gem_status gem_copy_rows(gem_ctx ctx, const void* src, const int64_t* src_idx, void* dst, const int64_t* dst_idx,
                         int64_t n, int64_t row_bytes, hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  if (n < 0 || row_bytes < 0) return fail(GEM_ERR_INVALID, "negative size");
  if (row_bytes % 4 != 0) return fail(GEM_ERR_INVALID, "row_bytes %lld is not a multiple of 4", (long long)row_bytes);
  if (n > 0 && row_bytes > 0 && (!src || !dst)) return fail(GEM_ERR_INVALID, "NULL buffer");
  if (((uintptr_t)src % 4) != 0 || ((uintptr_t)dst % 4) != 0) return fail(GEM_ERR_INVALID, "buffers must be 4-byte aligned");
  hipError_t e = launch_copy_rows(src, src_idx, dst, dst_idx, n, row_bytes, stream);
  return e == hipSuccess ? GEM_OK : hip_fail(e, "row copy");
}

gem_status gem_score_exact(gem_ctx ctx, const gem_sets* Q, const gem_sets* D, const gem_cands* C, int32_t compute,
                           int32_t k, float* scores, int64_t ld_scores, const int32_t* score_rows, float* top_scores,
                           int32_t* top_ids, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  if (compute != GEM_F32 && compute != GEM_BF16 && compute != GEM_BF16X3)
    return fail(GEM_ERR_INVALID, "exact scoring computes in F32, BF16 or BF16X3, not dtype %d", compute);
  return score_common(ctx, Q, D, C, compute, k, scores, ld_scores, score_rows, top_scores, top_ids, ws, ws_bytes,
                      stream);
}

gem_status gem_score_quant(gem_ctx ctx, const gem_sets* Q, const gem_sets* D, const gem_cands* C, int32_t k,
                           float* scores, int64_t ld_scores, const int32_t* score_rows, float* top_scores,
                           int32_t* top_ids, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  if (!D) return fail(GEM_ERR_INVALID, "D is NULL");
  if (!quant_dtype(D->dtype)) return fail(GEM_ERR_INVALID, "D: dtype %d is not a quantized format", D->dtype);
  return score_common(ctx, Q, D, C, D->dtype, k, scores, ld_scores, score_rows, top_scores, top_ids, ws, ws_bytes,
                      stream);
}

gem_status gem_score_quant_static(gem_ctx ctx, const gem_sets* Q, const gem_sets* D, const gem_cands* C, int32_t k,
                                  float* scores, int64_t ld_scores, const int32_t* score_rows, float* top_scores,
                                  int32_t* top_ids, hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  if (!Q || !D) return fail(GEM_ERR_INVALID, "NULL sets");
  if (!quant_dtype(D->dtype)) return fail(GEM_ERR_INVALID, "D: dtype %d is not a quantized format", D->dtype);
  if (!ctx->scratch) return fail(GEM_ERR_HIP, "no static scratch on device %d", ctx->device);
  gem_status st;
  if ((st = check_sets(Q, "Q", true)) != GEM_OK) return st;
  if ((st = check_sets(D, "D", false)) != GEM_OK) return st;
  if (C && (st = check_cands(C, Q->n_sets)) != GEM_OK) return st;
  const size_t need = score_layout(Q, D, C, D->dtype, k, scores != nullptr, ctx->n_cu / 8, ctx->topk_mode,
                                   ctx->gather_order).total;
  if (need > (size_t)GEM_STATIC_SCRATCH_BYTES)
    return fail(GEM_ERR_WORKSPACE, "this call needs %zu bytes of workspace; the static scratch holds %zu", need,
                (size_t)GEM_STATIC_SCRATCH_BYTES);
  return score_common(ctx, Q, D, C, D->dtype, k, scores, ld_scores, score_rows, top_scores, top_ids, ctx->scratch,
                      (size_t)GEM_STATIC_SCRATCH_BYTES, stream);
}

gem_status gem_topk(gem_ctx ctx, const float* scores, const int64_t* seg_offsets, const int32_t* seg_ids,
                    int64_t n_segs, int64_t seg_len, int64_t seg_ld, const int32_t* seg_rows, int32_t k,
                    float* top_scores, int32_t* top_ids, void* ws, size_t ws_bytes, hipStream_t stream) {
  (void)ws; (void)ws_bytes;
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  if (k < 0 || k > GEM_MAX_K) return fail(GEM_ERR_INVALID, "k = %d outside [0, %d]", k, GEM_MAX_K);
  if (n_segs < 0) return fail(GEM_ERR_INVALID, "negative n_segs");
  if (n_segs > INT32_MAX) return fail(GEM_ERR_UNSUPPORTED, "more than 2^31-1 segments");
  if (n_segs == 0 || k == 0) return GEM_OK;
  if (!top_scores || !top_ids) return fail(GEM_ERR_INVALID, "NULL output");
  TopkSegs S;
  S.scores = scores; S.off = seg_offsets; S.ids = seg_ids; S.rows = seg_rows; S.n_segs = n_segs;
  S.len = seg_len; S.ld = seg_ld;
  if (!seg_offsets) {
    if (seg_ids) return fail(GEM_ERR_INVALID, "uniform segments take positions as ids: seg_ids must be NULL");
    if (seg_len < 0) return fail(GEM_ERR_INVALID, "negative seg_len");
    if (seg_ld == 0) S.ld = seg_len;
    if (S.ld < seg_len) return fail(GEM_ERR_INVALID, "seg_ld < seg_len");
    S.rows = seg_rows;
  } else {
    S.rows = nullptr;
  }
  if (!scores) return fail(GEM_ERR_INVALID, "scores is NULL");
  hipError_t e = launch_topk(S, k, top_scores, top_ids, stream);
  return e == hipSuccess ? GEM_OK : hip_fail(e, "top-k");
}

gem_status gem_expand_batch(gem_ctx ctx, const gem_sets* Q8, const gem_sets* D8, const gem_cands* C, gem_beam* beam,
                            float* cand_scores, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  gem_status st;
  if ((st = check_sets(Q8, "Q8", true)) != GEM_OK) return st;
  if ((st = check_sets(D8, "D8", false)) != GEM_OK) return st;
  if (!quant_dtype(D8->dtype)) return fail(GEM_ERR_INVALID, "D8 must be FP8 E4M3, MXFP4 or MXFP6");
  const int32_t cd = D8->dtype;
  if (Q8->dtype != cd && Q8->dtype != GEM_F32) return fail(GEM_ERR_INVALID, "Q8 must be in D8's format or F32");
  if (!C) return fail(GEM_ERR_INVALID, "cands is NULL");
  if ((st = check_cands(C, Q8->n_sets)) != GEM_OK) return st;
  if (!beam) return fail(GEM_ERR_INVALID, "beam is NULL");
  if (beam->ef < 1 || beam->ef > GEM_MAX_EF) return fail(GEM_ERR_INVALID, "ef = %d outside [1, %d]", beam->ef, GEM_MAX_EF);
  if (Q8->n_sets > 0 && (!beam->scores || !beam->ids)) return fail(GEM_ERR_INVALID, "beam buffers are NULL");
  if ((int64_t)beam->ef + list_len_bound(C) > kBeamMaxEntries)
    return fail(GEM_ERR_UNSUPPORTED, "ef + longest list = %d exceeds %d", beam->ef + list_len_bound(C), kBeamMaxEntries);
  const ScoreLayout L = score_layout(Q8, D8, C, cd, 1, cand_scores != nullptr, ctx->n_cu / 8);
  if (ws_bytes < L.total) return fail(GEM_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, L.total);
  if (L.total > 0 && !ws) return fail(GEM_ERR_INVALID, "workspace is NULL");
  if (Q8->n_sets == 0) return GEM_OK;
  if ((st = device_check(ctx, Q8, D8, C, D8->n_sets, stream, "expansion")) != GEM_OK) return st;
  gem_sets Qc;
  if ((st = convert_query(Q8, cd, ws, L, &Qc, stream)) != GEM_OK) return st;
  float* es = cand_scores ? cand_scores : reinterpret_cast<float*>(at(ws, L.staged));
  CandsView cv = cview(C);
  GatherOpts go;
  hipError_t e = sort_for_walk(L, ws, list_len_bound(C), &cv, &go, stream);
  if (e != hipSuccess) return hip_fail(e, "candidate sort");
  e = launch_score_gather(cd, view(&Qc), view(D8), cv, list_len_bound(C), Q8->max_set_len, es,
                          lookup_gather(ctx, cd, C->n_lists, list_len_bound(C)), stream, go);
  if (e != hipSuccess) return hip_fail(e, "gathered scoring");
  e = launch_beam_merge(es, cview(C), Q8->n_sets, beam->ef, beam->scores, beam->ids,
                        list_len_bound(C) > 0 ? beam->ef + list_len_bound(C) : 0, stream);
  if (e != hipSuccess) return hip_fail(e, "beam merge");
  return GEM_OK;
}

size_t gem_emd_workspace_bytes(int64_t n_pairs) { return n_pairs > 0 ? emd_ws_bytes(n_pairs) : 0; }

gem_status gem_emd_sinkhorn(gem_ctx ctx, const gem_sets* A, const gem_sets* B, const int32_t* a_idx,
                            const int32_t* b_idx, int64_t n_pairs, float eps, int32_t n_iter, float* out, void* ws,
                            size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  gem_status st;
  if ((st = check_sets(A, "A", false)) != GEM_OK) return st;
  if ((st = check_sets(B, "B", false)) != GEM_OK) return st;
  if (A->dtype != GEM_F32 || B->dtype != GEM_F32) return fail(GEM_ERR_INVALID, "EMD takes float32 sets");
  if (A->max_set_len > 256 || B->max_set_len > 256)
    return fail(GEM_ERR_UNSUPPORTED, "set lengths %d, %d exceed 256", A->max_set_len, B->max_set_len);
  if (!(eps > 0.0f) || eps > 1e30f) return fail(GEM_ERR_INVALID, "eps = %g", (double)eps);
  if (n_iter < 1 || n_iter > 100000) return fail(GEM_ERR_INVALID, "n_iter = %d", n_iter);
  if (n_pairs < 0) return fail(GEM_ERR_INVALID, "negative n_pairs");
  if (n_pairs > 0 && (!a_idx || !b_idx || !out)) return fail(GEM_ERR_INVALID, "NULL buffer");
  const size_t need = emd_ws_bytes(n_pairs);
  if (n_pairs > 0 && (ws_bytes < need || !ws)) return fail(GEM_ERR_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
  if ((st = device_check_extra(ctx, A, B, nullptr, 0, a_idx, n_pairs, A->n_sets, b_idx, n_pairs, B->n_sets, stream,
                               "emd")) != GEM_OK)
    return st;
  EmdParams P;
  P.A = view(A); P.B = view(B); P.a_idx = a_idx; P.b_idx = b_idx; P.n_pairs = n_pairs;
  P.eps = eps; P.n_iter = n_iter; P.out = out;
  hipError_t e = launch_emd_sinkhorn(P, ws, stream);
  return e == hipSuccess ? GEM_OK : hip_fail(e, "emd");
}

gem_status gem_set_clusters(gem_ctx ctx, const int32_t* vec_clusters, const int64_t* set_offsets, int64_t n_sets,
                            int32_t k2, int32_t r, uint32_t* set_masks, int64_t* member_offsets, int32_t* members,
                            void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  if (k2 < 1 || k2 > kMaxSearchClusters) return fail(GEM_ERR_UNSUPPORTED, "k2 = %d outside [1, %d]", k2, kMaxSearchClusters);
  if (r < 1 || r > k2) return fail(GEM_ERR_INVALID, "r = %d outside [1, k2]", r);
  if (n_sets < 0 || n_sets > INT32_MAX) return fail(GEM_ERR_INVALID, "n_sets out of range");
  if (ws_bytes < GEM_SEARCH_CLUSTER_WS || !ws) return fail(GEM_ERR_WORKSPACE, "workspace of %d bytes needed", GEM_SEARCH_CLUSTER_WS);
  if (!member_offsets || (n_sets > 0 && (!vec_clusters || !set_offsets || !set_masks || !members)))
    return fail(GEM_ERR_INVALID, "NULL buffer");
  hipError_t e = launch_set_clusters(vec_clusters, set_offsets, n_sets, k2, r, set_masks, member_offsets, members,
                                     static_cast<int32_t*>(ws), stream);
  return e == hipSuccess ? GEM_OK : hip_fail(e, "set clusters");
}

gem_status gem_query_clusters(gem_ctx ctx, const gem_sets* Q, const float* centroids, int32_t k2, int32_t t,
                              uint32_t* query_masks, hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  gem_status st;
  if ((st = check_sets(Q, "Q", false)) != GEM_OK) return st;
  if (Q->dtype != GEM_F32 || Q->codes) return fail(GEM_ERR_INVALID, "Q must be float32 rows");
  if (k2 < 1 || k2 > kMaxSearchClusters) return fail(GEM_ERR_UNSUPPORTED, "k2 = %d outside [1, %d]", k2, kMaxSearchClusters);
  if (t < 1) return fail(GEM_ERR_INVALID, "t = %d", t);
  if (Q->n_sets > 0 && (!centroids || !query_masks)) return fail(GEM_ERR_INVALID, "NULL buffer");
  hipError_t e = launch_query_clusters(Q->offsets, static_cast<const float*>(Q->vecs), Q->n_sets, centroids, k2, t,
                                       query_masks, stream);
  return e == hipSuccess ? GEM_OK : hip_fail(e, "query clusters");
}

namespace {

gem_status check_search(const gem_sets* Q, const gem_sets* D, const gem_graph* G, const gem_search_state* S,
                        const gem_beam* beam, SearchView* v, int32_t* row) {
  gem_status st;
  if ((st = check_sets(Q, "Q", true)) != GEM_OK) return st;
  if ((st = check_sets(D, "D", false)) != GEM_OK) return st;
  if (!G || !S || !beam) return fail(GEM_ERR_INVALID, "NULL argument");
  if (Q->dtype != D->dtype) return fail(GEM_ERR_INVALID, "Q must be in D's dtype");
  if (G->n_sets != D->n_sets) return fail(GEM_ERR_INVALID, "graph has %lld sets, D %lld", (long long)G->n_sets,
                                          (long long)D->n_sets);
  if (G->k2 < 1 || G->k2 > kMaxSearchClusters) return fail(GEM_ERR_UNSUPPORTED, "k2 = %d", G->k2);
  if (G->degree < 1 || G->degree > 64) return fail(GEM_ERR_UNSUPPORTED, "degree = %d outside [1, 64]", G->degree);
  if (S->width < 1 || S->width > 64) return fail(GEM_ERR_UNSUPPORTED, "width = %d outside [1, 64]", S->width);
  if (beam->ef < 1 || beam->ef > GEM_MAX_EF) return fail(GEM_ERR_INVALID, "ef = %d outside [1, %d]", beam->ef, GEM_MAX_EF);
  *row = std::max(G->k2, S->width * G->degree);
  if ((int64_t)beam->ef + *row > kBeamMaxEntries)
    return fail(GEM_ERR_UNSUPPORTED, "ef + candidate row = %d exceeds %d", beam->ef + *row, kBeamMaxEntries);
  if (Q->n_sets > 0 && (!G->neighbors || !G->set_masks || !G->member_offsets || !G->members || !S->query_masks ||
                        !S->visited || !S->expanded || !S->frontier || !S->cand_ids || !S->cand_scores || !S->active ||
                        !beam->scores || !beam->ids))
    return fail(GEM_ERR_INVALID, "NULL buffer");
  v->k2 = G->k2; v->width = S->width; v->degree = G->degree;
  v->neighbors = G->neighbors; v->set_mask = G->set_masks; v->qmask = S->query_masks;
  v->member_off = G->member_offsets; v->members = G->members;
  v->visited = S->visited; v->expanded = S->expanded; v->frontier = S->frontier; v->active = S->active;
  v->bitmap_words = (G->n_sets + 31) / 32;
  return GEM_OK;
}

gem_status search_score_merge(gem_ctx ctx, const gem_sets* Q, const gem_sets* D, const gem_search_state* S,
                              gem_beam* beam, int32_t row, hipStream_t stream) {
  CandsView c;
  c.off = nullptr; c.ids = S->cand_ids; c.n_lists = Q->n_sets; c.stride = row;
  hipError_t e = launch_score_gather(D->dtype, view(Q), view(D), c, row, Q->max_set_len, S->cand_scores,
                                     lookup_gather(ctx, D->dtype, Q->n_sets, row), stream);
  if (e != hipSuccess) return hip_fail(e, "search scoring");
  e = launch_beam_merge(S->cand_scores, c, Q->n_sets, beam->ef, beam->scores, beam->ids, beam->ef + row, stream);
  return e == hipSuccess ? GEM_OK : hip_fail(e, "search merge");
}

}  // namespace

gem_status gem_search_begin(gem_ctx ctx, const gem_sets* Q, const gem_sets* D, const gem_graph* G,
                            gem_search_state* S, const uint32_t* random_words, gem_beam* beam, hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  SearchView v;
  int32_t row = 0;
  gem_status st = check_search(Q, D, G, S, beam, &v, &row);
  if (st != GEM_OK) return st;
  if (Q->n_sets > 0 && !random_words) return fail(GEM_ERR_INVALID, "random_words is NULL");
  if (Q->n_sets == 0) return GEM_OK;
  {
    // GEM_CHECK mode: the sets and the graph's neighbour lists (ids < n_sets, -1 padding)
    gem_cands nb{};
    nb.n_lists = G->n_sets; nb.n_entries = G->n_sets * (int64_t)G->degree; nb.stride = G->degree;
    nb.max_list_len = G->degree; nb.offsets = nullptr; nb.ids = G->neighbors;
    if ((st = device_check(ctx, Q, D, &nb, G->n_sets, stream, "search")) != GEM_OK) return st;
  }
  hipError_t e = launch_search_clear(v, Q->n_sets, stream);
  if (e == hipSuccess) e = launch_search_entries(v, Q->n_sets, random_words, S->cand_ids, row, stream);
  if (e == hipSuccess) e = launch_beam_reset(beam->scores, beam->ids, Q->n_sets * (int64_t)beam->ef, stream);
  if (e != hipSuccess) return hip_fail(e, "search start");
  return search_score_merge(ctx, Q, D, S, beam, row, stream);
}

gem_status gem_search_step(gem_ctx ctx, const gem_sets* Q, const gem_sets* D, const gem_graph* G,
                           gem_search_state* S, gem_beam* beam, hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  SearchView v;
  int32_t row = 0;
  gem_status st = check_search(Q, D, G, S, beam, &v, &row);
  if (st != GEM_OK) return st;
  hipError_t e = launch_search_step(v, Q->n_sets, beam->ids, beam->ef, S->cand_ids, row, stream);
  if (e != hipSuccess) return hip_fail(e, "search step");
  if (Q->n_sets == 0) return GEM_OK;
  return search_score_merge(ctx, Q, D, S, beam, row, stream);
}

gem_status gem_beam_merge(gem_ctx ctx, const float* cand_scores, const gem_cands* C, gem_beam* beam,
                          hipStream_t stream) {
  if (!ctx || !C || !beam) return fail(GEM_ERR_INVALID, "NULL argument");
  gem_status st = check_cands(C, C->n_lists);
  if (st != GEM_OK) return st;
  if (beam->ef < 1 || beam->ef > GEM_MAX_EF) return fail(GEM_ERR_INVALID, "ef = %d outside [1, %d]", beam->ef, GEM_MAX_EF);
  if (C->n_lists > 0 && (!beam->scores || !beam->ids)) return fail(GEM_ERR_INVALID, "beam buffers are NULL");
  if (C->n_entries > 0 && !cand_scores) return fail(GEM_ERR_INVALID, "cand_scores is NULL");
  if ((int64_t)beam->ef + list_len_bound(C) > kBeamMaxEntries)
    return fail(GEM_ERR_UNSUPPORTED, "ef + longest list = %d exceeds %d", beam->ef + list_len_bound(C), kBeamMaxEntries);
  hipError_t e = launch_beam_merge(cand_scores, cview(C), C->n_lists, beam->ef, beam->scores, beam->ids,
                                   list_len_bound(C) > 0 ? beam->ef + list_len_bound(C) : 0, stream);
  return e == hipSuccess ? GEM_OK : hip_fail(e, "beam merge");
}

gem_status gem_beam_reset(gem_ctx ctx, gem_beam* beam, int64_t n_queries, hipStream_t stream) {
  if (!ctx || !beam) return fail(GEM_ERR_INVALID, "NULL argument");
  if (beam->ef < 1 || beam->ef > GEM_MAX_EF) return fail(GEM_ERR_INVALID, "ef = %d outside [1, %d]", beam->ef, GEM_MAX_EF);
  if (n_queries < 0) return fail(GEM_ERR_INVALID, "negative n_queries");
  if (n_queries > 0 && (!beam->scores || !beam->ids)) return fail(GEM_ERR_INVALID, "beam buffers are NULL");
  hipError_t e = launch_beam_reset(beam->scores, beam->ids, n_queries * (int64_t)beam->ef, stream);
  return e == hipSuccess ? GEM_OK : hip_fail(e, "beam reset");
}

gem_status gem_validate_sets(gem_ctx ctx, const gem_sets* S, hipStream_t stream) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  gem_status st = check_sets(S, "sets", false);
  if (st != GEM_OK) return st;
  if ((st = reset_validation(stream)) != GEM_OK) return st;
  const hipError_t e = launch_set_validation(S, stream);
  if (e != hipSuccess) return hip_fail(e, "validation launch");
  return run_validation(stream, "sets");
}

gem_status gem_validate_cands(gem_ctx ctx, const gem_cands* C, int64_t n_sets, hipStream_t stream) {
  if (!ctx || !C) return fail(GEM_ERR_INVALID, "NULL argument");
  gem_status st = check_cands(C, C->n_lists);
  if (st != GEM_OK) return st;
  if ((st = reset_validation(stream)) != GEM_OK) return st;
  const hipError_t e = launch_cand_validation(C, n_sets, stream);
  if (e != hipSuccess) return hip_fail(e, "validation launch");
  return run_validation(stream, "cands");
}


static void to_public(const DenseSchedule& d, gem_dense_schedule* out) {
  out->chunk_docs = d.chunk_docs;
  out->items_per_slot = d.items_per_slot;
  out->slots_per_xcd = d.slots_per_xcd;
  out->reserved = 0;
}

gem_status gem_get_dense_schedule(gem_ctx ctx, int32_t dtype, int64_t q_rows, int64_t n_docs,
                                  gem_dense_schedule* out) {
  if (!ctx || !out) return fail(GEM_ERR_INVALID, "NULL argument");
  if (!valid_dtype(dtype)) return fail(GEM_ERR_INVALID, "dtype %d", dtype);
  to_public(lookup_dense(ctx, dtype, q_rows, n_docs), out);
  return GEM_OK;
}

gem_status gem_set_dense_schedule(gem_ctx ctx, int32_t dtype, int64_t q_rows, int64_t n_docs,
                                  const gem_dense_schedule* sched) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  if (!valid_dtype(dtype)) return fail(GEM_ERR_INVALID, "dtype %d", dtype);
  const uint64_t key = dense_key(dtype, q_rows, n_docs);
  std::lock_guard<std::mutex> g(ctx->mu);
  if (!sched) {
    ctx->dense.erase(key);
    return GEM_OK;
  }
  DenseSchedule d{sched->chunk_docs, sched->items_per_slot, sched->slots_per_xcd};
  if (!dense_schedule_valid(d, ctx->n_cu / 8))
    return fail(GEM_ERR_INVALID, "schedule (chunk_docs %d, items_per_slot %d, slots_per_xcd %d) outside the "
                "supported range", d.chunk_docs, d.items_per_slot, d.slots_per_xcd);
  ctx->dense[key] = d;
  return GEM_OK;
}

gem_status gem_autotune_dense(gem_ctx ctx, const gem_sets* Q, const gem_sets* D, int32_t compute, float* scores,
                              int64_t ld_scores, void* ws, size_t ws_bytes, hipStream_t stream, int32_t reps,
                              gem_dense_schedule* best, float* best_ms) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  if (!valid_dtype(compute)) return fail(GEM_ERR_INVALID, "compute dtype %d", compute);
  if (!scores) return fail(GEM_ERR_INVALID, "autotuning needs a scores buffer");
  if (reps < 1 || reps > 100) return fail(GEM_ERR_INVALID, "reps = %d outside [1, 100]", reps);
  if (!Q || !D) return fail(GEM_ERR_INVALID, "NULL sets");
  const int cpx = ctx->n_cu / 8;
  Timer T(stream);
  gem_status st = T.init();
  if (st != GEM_OK) return st;
  auto run = [&](const DenseSchedule& c) {
    return score_common(ctx, Q, D, nullptr, compute, 0, scores, ld_scores, nullptr, nullptr, nullptr, ws, ws_bytes,
                        stream, &c);
  };
  // stage 1: chunk size x items per workgroup at one workgroup per CU (the
  // library default first: it keeps ties); stage 2: fewer workgroups per XCD
  std::vector<DenseSchedule> cand;
  cand.push_back(default_dense_schedule(compute, Q->n_vecs, D->n_sets, cpx));
  for (int cd : {64, 32})
    for (int ips : {2, 4, 8, 16}) {
      const DenseSchedule c{cd, ips, cpx};
      if (c.chunk_docs != cand[0].chunk_docs || c.items_per_slot != cand[0].items_per_slot) cand.push_back(c);
    }
  DenseSchedule best_s = cand[0];
  float best_t = -1.0f;
  if ((st = T.pick(cand, run, reps, &best_s, &best_t)) != GEM_OK) return st;
  std::vector<DenseSchedule> cand2;
  for (int sl : {(3 * cpx) / 4, cpx / 2})
    if (sl >= 1 && sl != best_s.slots_per_xcd) cand2.push_back(DenseSchedule{best_s.chunk_docs, best_s.items_per_slot, sl});
  if ((st = T.pick(cand2, run, reps, &best_s, &best_t)) != GEM_OK) return st;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->dense[dense_key(compute, Q->n_vecs, D->n_sets)] = best_s;
  }
  if (best) to_public(best_s, best);
  if (best_ms) *best_ms = best_t;
  return GEM_OK;
}

gem_status gem_get_gather_schedule(gem_ctx ctx, int32_t dtype, int64_t n_lists, int64_t max_list_len,
                                   gem_gather_schedule* out) {
  if (!ctx || !out) return fail(GEM_ERR_INVALID, "NULL argument");
  if (!valid_dtype(dtype)) return fail(GEM_ERR_INVALID, "dtype %d", dtype);
  const GatherSchedule g = lookup_gather(ctx, dtype, n_lists, max_list_len);
  out->entries_per_wave = g.entries_per_wave;
  out->depth = g.depth > 0 ? g.depth : gather_depth_choice(dtype, 1);
  out->reserved[0] = out->reserved[1] = 0;
  return GEM_OK;
}

gem_status gem_set_gather_schedule(gem_ctx ctx, int32_t dtype, int64_t n_lists, int64_t max_list_len,
                                   const gem_gather_schedule* sched) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  if (!valid_dtype(dtype)) return fail(GEM_ERR_INVALID, "dtype %d", dtype);
  const uint64_t key = gather_key(dtype, n_lists, max_list_len);
  std::lock_guard<std::mutex> g(ctx->mu);
  if (!sched) {
    ctx->gather.erase(key);
    return GEM_OK;
  }
  const GatherSchedule gs{sched->entries_per_wave, sched->depth};
  if (!gather_schedule_valid(dtype, gs))
    return fail(GEM_ERR_INVALID, "gather schedule (entries_per_wave %d, depth %d) outside the supported set",
                gs.entries_per_wave, gs.depth);
  ctx->gather[key] = gs;
  return GEM_OK;
}

gem_status gem_autotune_gather(gem_ctx ctx, const gem_sets* Q, const gem_sets* D, const gem_cands* C,
                               int32_t compute, float* scores, void* ws, size_t ws_bytes, hipStream_t stream,
                               int32_t reps, gem_gather_schedule* best, float* best_ms) {
  if (!ctx) return fail(GEM_ERR_INVALID, "ctx is NULL");
  if (!valid_dtype(compute)) return fail(GEM_ERR_INVALID, "compute dtype %d", compute);
  if (!C) return fail(GEM_ERR_INVALID, "autotuning the gathered scorer needs candidate lists");
  if (!scores) return fail(GEM_ERR_INVALID, "autotuning needs a scores buffer");
  if (reps < 1 || reps > 100) return fail(GEM_ERR_INVALID, "reps = %d outside [1, 100]", reps);
  if (!Q || !D) return fail(GEM_ERR_INVALID, "NULL sets");
  Timer T(stream);
  gem_status st = T.init();
  if (st != GEM_OK) return st;
  auto run = [&](const GatherSchedule& g) {
    return score_common(ctx, Q, D, C, compute, 0, scores, 0, nullptr, nullptr, nullptr, ws, ws_bytes, stream,
                        nullptr, &g);
  };
  // the library's rule first (it keeps ties), then entries per wave x depth
  std::vector<GatherSchedule> cand{GatherSchedule{}};
  for (int e : {0, 8, 16, 32, 64})
    for (int i = 0; i < 3; ++i)
      if (!(e == 0 && i == 1)) cand.push_back(GatherSchedule{e, gather_depth_choice(compute, i)});
  GatherSchedule best_s = cand[0];
  float best_t = -1.0f;
  if ((st = T.pick(cand, run, reps, &best_s, &best_t)) != GEM_OK) return st;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->gather[gather_key(compute, C->n_lists, list_len_bound(C))] = best_s;
  }
  if (best) {
    best->entries_per_wave = best_s.entries_per_wave;
    best->depth = best_s.depth > 0 ? best_s.depth : gather_depth_choice(compute, 1);
    best->reserved[0] = best->reserved[1] = 0;
  }
  if (best_ms) *best_ms = best_t;
  return GEM_OK;
}

gem_status gem_save_tune_cache(gem_ctx ctx, const char* path) {
  if (!ctx || !path) return fail(GEM_ERR_INVALID, "NULL argument");
  std::string out;
  {
    std::lock_guard<std::mutex> g(ctx->mu);
    out = tune_cache_json(ctx);
  }
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(GEM_ERR_INVALID, "cannot write %s", path);
  const size_t n = std::fwrite(out.data(), 1, out.size(), f);
  const int c = std::fclose(f);
  if (n != out.size() || c != 0) return fail(GEM_ERR_INVALID, "write of %s failed", path);
  return GEM_OK;
}

gem_status gem_load_tune_cache(gem_ctx ctx, const char* path) {
  if (!ctx || !path) return fail(GEM_ERR_INVALID, "NULL argument");
  return load_tune_cache(ctx, path, false);
}

}  // extern "C"
