// Internal host-side interface between the C ABI (capi.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/gem.h"

namespace gem {

// A dispatch's work-item count is a 32-bit number: grids are capped at 2^31
// work-items and kernels stride over the rest.
constexpr int64_t kMaxGridThreads = int64_t(1) << 31;
inline unsigned capped_blocks(int64_t blocks, int threads_per_block) {
  const int64_t cap = kMaxGridThreads / threads_per_block;
  return (unsigned)(blocks < cap ? blocks : cap);
}

// Device view of a CSR set batch.
struct SetsView {
  const int64_t* off;     // [n_sets + 1], absolute entry indices
  const void* vecs;       // rows of kDim elements (the codebook of a code set)
  const float* scales;    // FP8: per-row power-of-two scale
  const int32_t* codes;   // code sets: entry r is row codes[r] of vecs; else NULL (entry r is row r)
  int64_t n_sets;
};

// Device view of candidate lists: list i = [off[i], off[i+1]) or [i*stride, (i+1)*stride).
struct CandsView {
  const int64_t* off;
  const int32_t* ids;
  int64_t n_lists;
  int32_t stride;
};

// Query blocks: block b = queries [qb_start[b], qb_start[b+1]); n_blocks_max + 2 entries,
// the last one holding the number of non-empty blocks.
// qcol[i]: first (16-aligned) column of query i in the padded layout, [n_q + 1].
constexpr int kBlockMaxQueries = 32;

// Row capacity (query vectors held in registers) of one pass of the dense scorer.
int dense_pass_rows(int dtype);
// Rows a query block may hold for a batch whose longest query has max_len rows.
int dense_block_rows(int dtype, int max_len);
int dense_block_rows_for(int dtype, int max_len, int64_t n_q, int64_t n_vecs);
int64_t dense_blocks_upper(int64_t n_q, int64_t n_rows, int block_rows, int max_len);

hipError_t launch_plan_query_blocks(const int64_t* q_off, int64_t n_q, int block_rows, int max_len,
                                    int32_t* qb_start, int64_t* qcol, int64_t n_blocks_max, hipStream_t s);

// Fused per-query top-k of the dense scorer (the k-argmax of Sec. 3.1 without a
// score matrix). Query q's documents are split into 8 * np pieces (np per
// XCD); the wave that scores piece p of query q keeps, in region (q, p) of
// `keys`, every document whose rank key beats the query's running threshold,
// and when the region is full it selects the region's k best, keeps them and
// raises the threshold to the k-th (also the shared bound gthr[q]). A merge
// then takes the k best of the regions: exactly the top-k of the whole row.
struct TopkFuse {
  int32_t k;                  // 0: the scores are stored instead
  int32_t cap;                // entries per region: >= k + 64, or >= the piece's documents
  int32_t np;                 // pieces per XCD
  uint64_t* keys;             // [n_q][8 np][cap] rank keys (score bits above the complemented id)
  int32_t* cnt;               // [n_q][8 np] entries per region (zero before the launch)
  unsigned long long* gthr;   // [n_q] a lower bound of the query's k-th key (zero before the launch)
};

struct DenseOut {
  float* scores;          // score (i, j) at scores[row(i) * ld + j]
  int64_t ld;
  const int32_t* rows;    // nullable
  TopkFuse tk;            // tk.k > 0: no scores are stored, the regions are filled instead
};

// Regions per XCD and entries per region of a fused top-k over n_docs documents
// for a batch whose block groups are at least n_bg_min, on a grid of
// `slots_per_xcd` workgroups per XCD (so that every workgroup gets an item).
void topk_fuse_shape(int32_t k, int64_t n_docs, int64_t n_bg_min, int slots_per_xcd, int32_t* np, int32_t* cap);
// The k best keys of each query's regions -> [n_q][k] scores and ids (padding
// (-inf, -1)), the same as gem_topk on the query's whole score row.
hipError_t launch_topk_regions(const uint64_t* keys, const int32_t* cnt, int64_t n_q, int32_t regions, int32_t cap,
                               int32_t k, float* top_scores, int32_t* top_ids, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);

// Schedule of the persistent dense scorer (never changes a result).
struct DenseSchedule {
  int32_t chunk_docs;       // documents per chunk: 32 or 64
  int32_t items_per_slot;   // target work items per workgroup
  int32_t slots_per_xcd;    // workgroups per XCD (at most one per CU)
};
DenseSchedule default_dense_schedule(int dtype, int64_t q_rows, int64_t n_docs, int cus_per_xcd);
bool dense_schedule_valid(const DenseSchedule& d, int cus_per_xcd);

hipError_t launch_score_dense(int dtype, const SetsView& Q, const SetsView& D, const int32_t* qb_start,
                              const int64_t* qcol, int64_t n_blocks_max, const DenseOut& out,
                              const DenseSchedule& sched, int32_t block_rows, hipStream_t s);

// Schedule of the gathered scorer (never changes a result): entries of a list
// per wave (0: the library's rule) and tiles in flight per wave (0: the
// format's default; else one of gather_depth_choice(dtype, 0..2)).
struct GatherSchedule {
  int32_t entries_per_wave = 0;
  int32_t depth = 0;
};
int gather_depth_choice(int dtype, int i);
bool gather_schedule_valid(int dtype, const GatherSchedule& g);

// Options of a gathered-scorer launch (none change a score):
//   item_start: entries of the documents that have work items in the
//     document-major scorer (the exclusive scan of its items per document,
//     item_start[d + 1] > item_start[d]) are left to it; their scores are not
//     written.
//   out_pos: the lists were reordered; entry e is the caller's entry
//     out_pos[e] (an index into the caller's entry array), and its score goes
//     there.
//   chunk_major: waves take chunk c of every list before chunk c + 1 of any
//     (with lists sorted by document id, every chunk then reads one region of
//     the corpus at a time, so that the listings of a document run close
//     together and find it in the Infinity Cache).
struct GatherOpts {
  const int32_t* item_start = nullptr;
  const int32_t* out_pos = nullptr;
  bool chunk_major = false;
};
hipError_t launch_score_gather(int dtype, const SetsView& Q, const SetsView& D, const CandsView& C,
                               int32_t max_list_len, int32_t max_q_len, float* scores, const GatherSchedule& g,
                               hipStream_t s, const GatherOpts& opts = GatherOpts{});
// Sorts every candidate list by document id (padding ids last): sorted_ids
// and pos (each sorted entry's index in the caller's entry array) in the
// lists' layout. Lists of at most kSortMaxList entries (a longer list keeps
// its order); at most 2^31 - 1 entries.
constexpr int kSortMaxList = 2048;
hipError_t launch_sort_lists(const CandsView& C, int32_t max_list_len, int32_t* sorted_ids, int32_t* pos,
                             hipStream_t s);
// Gathered scoring by document, for candidate lists that share documents (a
// batch of shortlists drawn from the same corpus region): the call's entries
// are grouped by document (a counting sort), and each workgroup stages one
// document in LDS once and scores it against up to kByDocListings of the
// queries that list it. Every score is bitwise the gathered scorer's.
// Documents of up to kByDocMaxRows vectors, sets without codes. Only documents
// with at least min_work listing-tiles (listings x 16-row tiles) are scored
// (every listed document for min_work <= 1); *skip receives what the gathered
// scorer needs to take the others.
constexpr int kByDocListings = 64;
constexpr int kByDocMaxRows = 256;
// The mixed order's threshold of a format: a document's listing-tiles from
// which scoring it by document takes less time than streaming it per listing.
int32_t bydoc_min_work(int dtype);
size_t bydoc_ws_bytes(int64_t n_docs, int64_t n_entries);
hipError_t launch_score_bydoc(int dtype, const SetsView& Q, const SetsView& D, const CandsView& C, int64_t n_entries,
                              float* scores, void* ws, int32_t min_work, GatherOpts* skip, hipStream_t s);
// The dense output of a small query batch by the gathered scorer: every
// document of D is an entry of every query's list (bitwise the dense scorer's
// scores, one wave per few documents: memory-bound streaming instead of one
// lightly loaded block group).
hipError_t launch_score_range(int dtype, const SetsView& Q, const SetsView& D, const DenseOut& out, hipStream_t s);

hipError_t launch_convert_bf16(const float* x, int64_t n_elems, uint16_t* out, hipStream_t s);
hipError_t launch_split_bf16x3(const float* x, int64_t n_rows, uint16_t* out, hipStream_t s);
hipError_t launch_quantize_fp8(const float* x, int64_t n_rows, uint8_t* out, float* scales, hipStream_t s);
hipError_t launch_quantize_mxfp4(const float* x, int64_t n_rows, uint8_t* out, uint8_t* exps, hipStream_t s);
hipError_t launch_quantize_mxfp6(const float* x, int64_t n_rows, uint8_t* out, uint8_t* exps, hipStream_t s);
// Codebook kernels (nearest centroid, k-means update).
size_t nearest_centroid_ws_bytes(int64_t n_rows, int64_t n_centroids);
hipError_t launch_nearest_centroid(int dtype, const void* x, int64_t n_rows, const void* centroids,
                                   int64_t n_centroids, int32_t* codes, void* ws, int n_cu, hipStream_t s);
size_t centroid_update_ws_bytes(int64_t n_rows, int64_t n_centroids);
hipError_t launch_centroid_update(const float* x, int64_t n_rows, const int32_t* codes, const float* centroids,
                                  int64_t n_centroids, float* new_centroids, int32_t* counts, void* ws, hipStream_t s);

hipError_t launch_copy_rows(const void* src, const int64_t* src_idx, void* dst, const int64_t* dst_idx, int64_t n,
                            int64_t row_bytes, hipStream_t s);

// Segments for top-k.
struct TopkSegs {
  const float* scores;
  const int64_t* off;     // CSR segments, or NULL for uniform segments
  const int32_t* ids;     // nullable: positions are the ids
  const int32_t* rows;    // uniform mode: row of segment i (nullable: i)
  int64_t n_segs;
  int64_t len;            // uniform mode: entries per segment
  int64_t ld;             // uniform mode: row stride
};

hipError_t launch_topk(const TopkSegs& segs, int32_t k, float* top_scores, int32_t* top_ids, hipStream_t s);

hipError_t launch_beam_merge(const float* cand_scores, const CandsView& C, int64_t n_q, int32_t ef,
                             float* beam_scores, int32_t* beam_ids, int32_t max_entries, hipStream_t s);
hipError_t launch_beam_reset(float* beam_scores, int32_t* beam_ids, int64_t n, hipStream_t s);

constexpr int kBeamMaxEntries = 4096;   // ef + longest candidate list of a merge

// Batched cluster-guided search (Alg. 5): the graph, the set clusters and one
// batch's state, all device memory owned by the caller.
struct SearchView {
  int32_t k2;                 // coarse clusters (<= 1024)
  int32_t width;              // sets expanded per query and step
  int32_t degree;             // neighbours per set
  const int32_t* neighbors;   // [n_sets][degree], -1 padded
  const uint32_t* set_mask;   // [n_sets][words] C_top masks
  const uint32_t* qmask;      // [n_q][words] C_query masks
  const int64_t* member_off;  // [k2 + 1]
  const int32_t* members;     // sets per cluster, in id order
  uint32_t* visited;          // [n_q][bitmap_words]
  uint32_t* expanded;         // [n_q][bitmap_words]
  int32_t* frontier;          // [n_q][width]
  uint32_t* active;           // [1]: queries with a frontier in the last select
  int64_t bitmap_words;       // (n_sets + 31) / 32
};
constexpr int kMaxSearchClusters = 1024;

hipError_t launch_set_clusters(const int32_t* vec_clusters, const int64_t* set_off, int64_t n_sets, int k2, int r,
                               uint32_t* mask, int64_t* member_off, int32_t* members, int32_t* ws, hipStream_t s);
hipError_t launch_query_clusters(const int64_t* q_off, const float* q, int64_t n_q, const float* C, int k2, int t,
                                 uint32_t* qmask, hipStream_t s);
hipError_t launch_search_clear(const SearchView& S, int64_t n_q, hipStream_t s);
hipError_t launch_search_entries(const SearchView& S, int64_t n_q, const uint32_t* u, int32_t* cand, int32_t stride,
                                 hipStream_t s);
// One search step's select and expand (clears *S.active first).
hipError_t launch_search_step(const SearchView& S, int64_t n_q, const int32_t* beam_ids, int32_t ef, int32_t* cand,
                              int32_t stride, hipStream_t s);

// Entropic EMD of set pairs (one workgroup per pair).
constexpr int kMaxEmdCost = 36864;     // entries of the LDS cost matrix (m1 * m2)
constexpr int kEmdMaxSet = 256;        // longest set
constexpr int kEmdBigBlocks = 256;     // workgroups of the pass over larger matrices
struct EmdParams {
  SetsView A, B;                       // float32 rows (or code sets over float32 codebooks)
  const int32_t* a_idx;                // [n_pairs] sets of A
  const int32_t* b_idx;                // [n_pairs] sets of B
  int64_t n_pairs;
  float eps;
  int32_t n_iter;
  float* out;                          // [n_pairs]
  uint8_t* flags;                      // [n_pairs] workspace: pairs for the second pass
  float* big;                          // workspace: kEmdBigBlocks matrices of kEmdMaxSet^2
};
size_t emd_ws_bytes(int64_t n_pairs);
hipError_t launch_emd_sinkhorn(EmdParams P, void* ws, hipStream_t s);

// Validation: returns number of violations found (synchronizes).
hipError_t validate_sets(const SetsView& S, int64_t n_vecs, int is_fp8, hipStream_t s, int64_t* bad);
hipError_t validate_cands(const CandsView& C, int64_t n_entries, int64_t n_sets, hipStream_t s, int64_t* bad);

}  // namespace gem
