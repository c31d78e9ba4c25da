/*
 * gem.h -- C ABI of the MI355X (gfx950) set-to-set scoring library.
 *
 * The library computes the Chamfer / MaxSim similarity of GEM (arXiv 2603.20336),
 * Def. 1 / Eq. (ch) of Sec. 3.1:
 *
 *     CH(Q, P) = sum over q in Q of  max over p in P of <q, p>
 *
 * for ragged batches of query sets against ragged document sets, in three forms:
 *   - exact, on float32 operands (float32 products and accumulation),
 *   - exact on bfloat16 operands (bf16 products, float32 accumulation),
 *   - the quantized estimate: OCP FP8 E4M3 operands with one power-of-two float32
 *     scale per vector, float32 accumulation. The paper's search scores
 *     neighbours with a cheap quantized Chamfer estimate (qCH, Sec. 4.5) and
 *     reranks the survivors with exact CH (Alg. 5, final step); here the estimate
 *     is the FP8 form, and the rerank is gem_score_exact over a candidate list.
 * plus the per-query top-k of the retrieval problem (Sec. 3.1, k-argmax of CH)
 * and one step of batched beam expansion: score each query's candidate ids with
 * the estimate and merge them into a bounded result set that keeps at most ef
 * entries, evicting the worst (the set R of Alg. 5).
 *
 * Conventions (all entry points):
 *   - Pointers marked [device] point to device memory on the context's device;
 *     the caller owns every buffer, including the workspace. The library never
 *     allocates device memory, and never synchronizes the stream except in the
 *     validation calls, the autotuners, gem_check_status and in GEM_OPT_CHECK
 *     mode.
 *   - Every call enqueues its kernels on `stream` (0 = the null stream) and
 *     returns once they are enqueued; results are ready when the stream reaches
 *     that point.
 *   - Host-checkable argument errors return a status before anything is
 *     enqueued; gem_last_error() then holds a message. Device data (offsets,
 *     ids, values) is trusted: offsets must be non-decreasing and inside the
 *     vector array, ids inside [0, n_sets) or negative (padding), values finite.
 *     gem_validate_sets / gem_validate_cands check those conditions on demand.
 *   - Vector dimension is 128 (the paper's d = 128 for every dataset, Sec. 5.1).
 *   - Scores are float32. CH of an empty query set is 0 (empty sum); CH of a
 *     non-empty query against an empty document is -inf (max over nothing).
 *   - Top-k order is score descending, then id ascending; ids are distinct; a
 *     list shorter than k is padded with (-inf, -1).
 *   - Several host threads may share a context; its only mutable state, the
 *     table of dense-scorer schedules, is guarded by a lock.
 */
#ifndef GEM_H_
#define GEM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* hipStream_t;   /* the HIP runtime's stream handle */

typedef enum {
  GEM_OK = 0,
  GEM_ERR_INVALID = 1,       /* bad argument (null pointer, size, dtype, k, ...) */
  GEM_ERR_WORKSPACE = 2,     /* workspace smaller than gem_workspace_bytes() */
  GEM_ERR_UNSUPPORTED = 3,   /* valid request outside this build's limits (dim, set length) */
  GEM_ERR_HIP = 4,           /* a HIP runtime call or kernel launch failed */
  GEM_ERR_DEVICE_CHECK = 5   /* a validation kernel found bad device data */
} gem_status;

typedef enum {
  GEM_F32 = 0,               /* float32 rows, 512 bytes per 128-d vector */
  GEM_BF16 = 1,              /* bfloat16 rows (uint16 bit patterns), 256 bytes */
  GEM_FP8_E4M3 = 2,          /* OCP E4M3 codes (uint8), 128 bytes, plus a float32 scale */
  GEM_MXFP4 = 3,             /* OCP MXFP4: E2M1 codes, 64 bytes (element t in byte t/2, the low
                                nibble for even t), plus 4 E8M0 block exponents (one per 32
                                elements) per row */
  GEM_MXFP6 = 4,             /* OCP MXFP6: E2M3 codes, 96 bytes: block j (elements 32j .. 32j + 31)
                                fills bytes 24j .. 24j + 23, its element t in bits 6t .. 6t + 5
                                of those 192 bits (least significant bit first), plus 4 E8M0
                                block exponents per row as for MXFP4 */
  GEM_BF16X3 = 5             /* float32 values as two bfloat16 parts, x = hi + lo + e with
                                hi = bf16(x), lo = bf16(x - hi) (round to nearest even; x - hi
                                is exact in float32), |e| <= 2^-16 |x|. 512 bytes per row: four
                                128-byte blocks, block j holding hi of elements 32j .. 32j + 31
                                (64 bytes) and then lo of the same elements (64 bytes). A product
                                a*b is taken as ah*bh + ah*bl + al*bh on bf16 MFMA (the dropped
                                terms al*bl, ah*eb, ea*bh and smaller ones add up to at most
                                3.1 * 2^-16 |a||b|), accumulated in float32 */
} gem_dtype;

typedef enum {
  GEM_OP_SCORE_EXACT = 0,
  GEM_OP_SCORE_QUANT = 1,
  GEM_OP_TOPK = 2,
  GEM_OP_EXPAND = 3,
  GEM_OP_NEAREST_CENTROID = 4,
  GEM_OP_CENTROID_UPDATE = 5
} gem_op;

/* Largest query set (rows) a scoring call accepts. */
#define GEM_MAX_QUERY_LEN 256
/* Largest k of a top-k, and largest ef (beam width). */
#define GEM_MAX_K 2048
#define GEM_MAX_EF 1024
/* Vector dimension. */
#define GEM_DIM 128

typedef struct gem_ctx_s* gem_ctx;

/* A ragged batch of vector sets in CSR form.
 *   set i = rows offsets[i] .. offsets[i+1]-1 of `vecs` (absolute row indices,
 *   so a view of sets a..b of a larger batch is {offsets + a, n_sets = b - a}).
 *   vecs: [n_vecs][dim] row-major, element type `dtype`.
 *   scales: FP8: [n_vecs] float32; row r's values are scales[r] * decode(code).
 *           Scales must be powers of two (gem_quantize_fp8 writes such scales).
 *           MXFP4, MXFP6: [n_vecs] 32-bit words of 4 E8M0 bytes; byte j of row r's
 *           word is the exponent e + 127 of the scale 2^e of dims 32j .. 32j + 31.
 *   max_set_len: host-side upper bound of the set lengths (needed for query sets).
 *
 * Code sets (the quantized representation of Secs. 4.2 and 4.5, where every
 * vector is replaced by its nearest centroid NN(x) of the k-means vocabulary
 * C_quant): when `codes` is not NULL, the sets hold codes instead of rows.
 * Entry r of the batch (r < n_vecs, offsets index the entries) stands for row
 * codes[r] of `vecs`, which then holds the codebook: codebook_rows centroid
 * rows of element type `dtype` (FP8: scales[codes[r]] is that row's scale).
 * CH over code sets is the paper's quantized Chamfer estimate
 * qCH(Q, P) = sum_q max_p <NN(q), NN(p)>, computed in the compute dtype
 * (float32 compute gives the centroid products of the paper's float table).
 * Codes must lie in [0, codebook_rows) (gem_validate_sets checks them).
 */
typedef struct {
  int32_t dtype;               /* gem_dtype */
  int32_t dim;                 /* must be GEM_DIM */
  int64_t n_sets;
  int64_t n_vecs;              /* rows addressable in vecs (>= every offset); code sets: entries of codes */
  int32_t max_set_len;
  int32_t reserved;
  const int64_t* offsets;      /* [device] [n_sets + 1] */
  const void* vecs;            /* [device] rows, or the codebook of a code set */
  const float* scales;         /* [device] FP8 only, else NULL (code sets: per codebook row) */
  int64_t codebook_rows;       /* code sets: rows of vecs; else 0 */
  const int32_t* codes;        /* [device] [n_vecs] code sets only, else NULL */
} gem_sets;

/* Candidate-id lists, one per query set.
 *   list i = entries offsets[i] .. offsets[i+1]-1 of `ids` (offsets[0] may be > 0;
 *   outputs are indexed by the absolute entry index). If offsets is NULL, list i
 *   is entries i*stride .. i*stride + stride - 1.
 *   An id < 0 is padding: it scores -inf and never enters a top-k or a beam.
 *   n_entries: host-side size of `ids` (and of a per-entry score output).
 */
typedef struct {
  int64_t n_lists;             /* must equal the query batch's n_sets */
  int64_t n_entries;
  int32_t stride;              /* list length when offsets == NULL */
  int32_t max_list_len;        /* host-side upper bound of list lengths (0 = unknown) */
  const int64_t* offsets;      /* [device] [n_lists + 1] or NULL */
  const int32_t* ids;          /* [device] [n_entries] */
} gem_cands;

/* Bounded per-query result set R of Alg. 5: [n_queries][ef] (score, id), ordered
 * by score descending then id ascending, padded with (-inf, -1). */
typedef struct {
  int32_t ef;
  int32_t reserved;
  float* scores;               /* [device] [n_queries * ef] */
  int32_t* ids;                /* [device] [n_queries * ef] */
} gem_beam;

/* Create a context bound to HIP device `device`. Reads device properties once
 * and takes the address of the device's static scratch (gem_score_quant_static).
 * tune_cache_json: NULL, or the path of a tune cache written by
 * gem_save_tune_cache; its schedules for this GPU's architecture are installed
 * (entries of other architectures are skipped). A path that does not exist
 * is an empty cache; a file that is not a valid cache fails the call. */
gem_status gem_create(gem_ctx* out, int device, const char* tune_cache_json);
gem_status gem_destroy(gem_ctx ctx);
/* Static string naming a status code. */
const char* gem_status_string(gem_status s);
/* Message of the last failing call made on this host thread ("" if none). */
const char* gem_last_error(void);
/* Library version string. */
const char* gem_version(void);

/* Context options.
 *   GEM_OPT_TOPK_FUSION: how an exhaustive scoring call (C == NULL) with k > 0
 *   and no `scores` buffer finds the per-query top-k.
 *     GEM_TOPK_AUTO (default): fused into the dense scorer (no score matrix:
 *       each query keeps, per piece of the corpus, the documents that beat its
 *       running k-th best, and a merge takes the k best of those) when that
 *       needs less workspace than staging the [n_q][n_docs] scores, else staged.
 *     GEM_TOPK_FUSED: always fused for k <= 1024 (small batches then run the
 *       dense scorer instead of the streamed path).
 *     GEM_TOPK_STAGED: always staged, then gem_topk's kernel.
 *   Every mode returns the same top-k, bitwise. gem_workspace_bytes follows the
 *   option, so set it before sizing a workspace.
 *
 *   GEM_OPT_CHECK (0 = off, the default; 1 = on): device-data checking. Every
 *   scoring, expansion, search-start and EMD call first validates its device
 *   inputs (the conditions gem_validate_sets / gem_validate_cands check, plus
 *   finite float32 rows, and EMD pair indices inside their batches) and, if
 *   any is violated, returns GEM_ERR_DEVICE_CHECK without computing anything.
 *   The check synchronizes the stream; it is a debugging aid. The violations
 *   are also counted for gem_check_status.
 *
 *   GEM_OPT_GATHER_ORDER: how a gathered scoring call (C != NULL) of
 *   gem_score_exact / gem_score_quant reads the listed documents (the final
 *   rerank of Alg. 5 over a batch of shortlists, or any candidate lists).
 *     GEM_GATHER_BY_QUERY: one wave per query and run of its entries, each
 *       listed document read once per listing. A call with n_lists x longest
 *       list >= 65,536 and lists of at most 2048 entries (rows, not code
 *       sets) sorts every list by document id into the workspace first and
 *       walks the sorted lists chunk-major (as gem_expand_batch does).
 *     GEM_GATHER_BY_DOCUMENT: the entries are grouped by document on the
 *       device (a counting sort in the workspace); each document is staged in
 *       LDS once and scored against every query that lists it. Pays when the
 *       lists share documents (a batch of top-1000 shortlists lists each of
 *       its documents tens of times). Needs D->max_set_len in [1, 256] (a bound
 *       of every document's length; a longer document scored by document
 *       gets NaN scores) and no code sets; otherwise the call reads by query.
 *     GEM_GATHER_AUTO (default): when those conditions hold and the lists
 *       hold at least two entries per document of D (four in bf16, FP8 and
 *       the MX formats), the mixed order: the counting sort counts each
 *       document's listings, and a document whose listings times its 16-row
 *       tiles reach a threshold of the format (f32 192, split bf16 96, others
 *       64) is scored by document, the other entries by query. Else by query.
 *   Every order gives the same scores, bitwise. gem_workspace_bytes follows
 *   the option. gem_expand_batch always reads by query. */
typedef enum { GEM_OPT_TOPK_FUSION = 0, GEM_OPT_CHECK = 1, GEM_OPT_GATHER_ORDER = 2 } gem_option;
typedef enum { GEM_TOPK_AUTO = 0, GEM_TOPK_FUSED = 1, GEM_TOPK_STAGED = 2 } gem_topk_mode;
typedef enum { GEM_GATHER_AUTO = 0, GEM_GATHER_BY_QUERY = 1, GEM_GATHER_BY_DOCUMENT = 2 } gem_gather_order;
gem_status gem_set_option(gem_ctx ctx, int32_t option, int64_t value);
gem_status gem_get_option(gem_ctx ctx, int32_t option, int64_t* value);
/* Synchronizes `stream` and reports what happened since the last call:
 * GEM_ERR_HIP if a kernel on the stream failed, GEM_ERR_DEVICE_CHECK if
 * checked calls (GEM_OPT_CHECK) found invalid device values (the count is
 * then cleared), else GEM_OK. */
gem_status gem_check_status(gem_ctx ctx, hipStream_t stream);

/* Workspace bytes that the matching call needs for these arguments (0 if none).
 * For GEM_OP_SCORE_*: `compute` is the gem_dtype the scoring runs in, and
 * `scores_given` says whether the caller passes its own dense/entry score
 * buffer (if not and k > 0, the scores are staged in the workspace). */
size_t gem_workspace_bytes(gem_ctx ctx, int32_t op, const gem_sets* Q, const gem_sets* D,
                           const gem_cands* C, int32_t compute, int32_t k, int32_t scores_given);

/* float32 rows -> bfloat16 rows, round to nearest even (corpus / query conversion).
 *   x: [device] [n_rows * dim] float32; out: [device] [n_rows * dim] uint16. */
gem_status gem_convert_bf16(gem_ctx ctx, const float* x, int64_t n_rows, int32_t dim,
                            uint16_t* out, hipStream_t stream);

/* float32 rows -> GEM_BF16X3 rows (hi = bf16(x), lo = bf16(x - hi), round to
 * nearest even), for the exact mode that runs float32 products as three
 * bfloat16 products.
 *   x: [device] [n_rows * dim] float32; out: [device] [n_rows * dim] pairs of
 *   uint16 in the GEM_BF16X3 row layout (512 bytes per row). dim must be 128. */
gem_status gem_split_bf16x3(gem_ctx ctx, const float* x, int64_t n_rows, int32_t dim, uint16_t* out,
                            hipStream_t stream);

/* float32 rows -> OCP FP8 E4M3 codes + one power-of-two scale per row.
 *   scale = smallest 2^e (e clamped to [-126, 127]) with max|x| <= 448 * 2^e
 *   (1 for an all-zero row); code = E4M3(x / scale), round to nearest, ties to
 *   even, saturating at 448. out: [device] [n_rows * dim] uint8;
 *   scales: [device] [n_rows] float32. */
gem_status gem_quantize_fp8(gem_ctx ctx, const float* x, int64_t n_rows, int32_t dim,
                            uint8_t* out, float* scales, hipStream_t stream);

/* Nearest centroid (the map NN of Sec. 4.2 onto the k-means vocabulary of
 * Sec. 4.1): codes[i] = argmin_j ||x_i - c_j||^2, ties to the smallest j,
 * evaluated as argmax_j (<x_i, c_j> - ||c_j||^2 / 2) with MFMA inner products
 * in `dtype` (GEM_F32: float32 products; GEM_BF16: bfloat16 operands) and
 * float32 accumulation. The result is the same for any launch split.
 *   x: [device] [n_rows * dim] rows of `dtype`; centroids: [device]
 *   [n_centroids * dim] rows of `dtype`; codes: [device] [n_rows] int32.
 *   ws: [device] at least gem_codebook_workspace_bytes(GEM_OP_NEAREST_CENTROID,
 *   n_rows, n_centroids) bytes. Values must be finite. */
gem_status gem_nearest_centroid(gem_ctx ctx, const void* x, int64_t n_rows, const void* centroids,
                                int64_t n_centroids, int32_t dim, int32_t dtype, int32_t* codes, void* ws,
                                size_t ws_bytes, hipStream_t stream);

/* One k-means centroid update (Lloyd's step behind C_quant, Sec. 4.1): centroid
 * j becomes the mean of the rows x_i with codes[i] == j; a centroid with no
 * rows keeps its old value. The sums are exact integer sums of the rows scaled
 * by a power of two chosen from max |x| and n_rows (rounding each element to
 * that grid, below 2^-30 relative to max |x|), so the result does not depend on
 * the order of the atomic adds.
 *   x: [device] [n_rows * dim] float32; codes: [device] [n_rows] in
 *   [0, n_centroids); centroids (old), new_centroids: [device]
 *   [n_centroids * dim] float32 (may be the same buffer); counts: [device]
 *   [n_centroids] int32 (rows per centroid), or NULL. ws: [device] at least
 *   gem_codebook_workspace_bytes(GEM_OP_CENTROID_UPDATE, n_rows, n_centroids). */
gem_status gem_centroid_update(gem_ctx ctx, const float* x, int64_t n_rows, int32_t dim, const int32_t* codes,
                               const float* centroids, int64_t n_centroids, float* new_centroids, int32_t* counts,
                               void* ws, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes of gem_nearest_centroid / gem_centroid_update (op is
 * GEM_OP_NEAREST_CENTROID or GEM_OP_CENTROID_UPDATE; 0 for anything else). */
size_t gem_codebook_workspace_bytes(int32_t op, int64_t n_rows, int64_t n_centroids);

/* float32 rows -> OCP MXFP4: per block of 32 consecutive dims, the scale 2^e
 * with the smallest e in [-127, 127] such that max|x| <= 6 * 2^e (2^0 for an
 * all-zero block), and each element's E2M1 code of x / 2^e (nearest value,
 * ties to the even code; zero is code 0). The ultra-low-bit form of the
 * quantized estimate (named as future work in the paper's conclusion, Sec. 6).
 *   out: [device] [n_rows * 64] packed codes; exps: [device] [n_rows * 4] E8M0
 *   bytes (the `scales` of a GEM_MXFP4 set). */
gem_status gem_quantize_mxfp4(gem_ctx ctx, const float* x, int64_t n_rows, int32_t dim, uint8_t* out,
                              uint8_t* exps, hipStream_t stream);

/* float32 rows -> OCP MXFP6 with E2M3 elements: per block of 32 consecutive
 * dims, the scale 2^e with the smallest e in [-127, 127] such that
 * max|x| <= 7.5 * 2^e (2^0 for an all-zero block), and each element's E2M3
 * code of x / 2^e (nearest value, ties to the even code; zero is code 0).
 * Like MXFP4, an ultra-low-bit form of the quantized estimate (Sec. 6).
 *   out: [device] [n_rows * 96] packed codes (layout of GEM_MXFP6); exps:
 *   [device] [n_rows * 4] E8M0 bytes (the `scales` of a GEM_MXFP6 set).
 *   dim must be 128; errors as gem_quantize_mxfp4. */
gem_status gem_quantize_mxfp6(gem_ctx ctx, const float* x, int64_t n_rows, int32_t dim, uint8_t* out,
                              uint8_t* exps, hipStream_t stream);

/* Row copies for assembling batches (a serving loop gathers the active
 * requests' query rows from per-request slots, and writes admitted requests'
 * rows into their slots): for i < n, row (dst_idx ? dst_idx[i] : i) of dst
 * receives row (src_idx ? src_idx[i] : i) of src. Rows are row_bytes bytes (a
 * multiple of 4); src, dst [device], 4-byte aligned; src_idx, dst_idx [device]
 * int64 or NULL. Indices are trusted (device data); destination rows must be
 * distinct. Not part of the paper's method: plumbing around it. */
gem_status gem_copy_rows(gem_ctx ctx, const void* src, const int64_t* src_idx, void* dst, const int64_t* dst_idx,
                         int64_t n, int64_t row_bytes, hipStream_t stream);

/* Exact Chamfer scores CH(Q_i, D_j) (Def. 1).
 *   compute = GEM_F32, GEM_BF16 or GEM_BF16X3: the operand type of the products;
 *   D->dtype must equal it. Q->dtype may equal it, or be GEM_F32 when compute is
 *   GEM_BF16 or GEM_BF16X3 (Q is then converted into the workspace). GEM_F32
 *   runs float32 MFMA products; GEM_BF16X3 runs each float32 product as three
 *   bfloat16 products (see gem_dtype), several times the float32 MFMA rate,
 *   with a dot product off the exact one by at most 3.1 * 2^-16 *
 *   sum_t |a_t b_t| plus the float32 accumulation; GEM_BF16 takes the products
 *   of bfloat16-rounded operands.
 *   C == NULL: every query against every document. Score (i, j) is written to
 *     scores[row(i) * ld_scores + j], row(i) = score_rows ? score_rows[i] : i,
 *     ld_scores >= D->n_sets (0 means D->n_sets).
 *   C != NULL: scores[e] = CH(Q_i, D_ids[e]) for each entry e of list i (the
 *     exact rerank of a shortlist, Alg. 5 final step).
 *   k > 0: per-query top-k of those scores into top_scores / top_ids [n_q][k]
 *     (ids are document indices of D). `scores` may then be NULL: with C == NULL
 *     the top-k is fused into the scorer or the scores are staged in ws
 *     (GEM_OPT_TOPK_FUSION); with C != NULL the entry scores are staged.
 *   k == 0: scores only.
 *   Limits: Q->max_set_len <= GEM_MAX_QUERY_LEN, k <= GEM_MAX_K (the fused top-k
 *   takes k <= 1024; a larger k is staged).
 */
gem_status gem_score_exact(gem_ctx ctx, const gem_sets* Q, const gem_sets* D, const gem_cands* C,
                           int32_t compute, int32_t k,
                           float* scores, int64_t ld_scores, const int32_t* score_rows,
                           float* top_scores, int32_t* top_ids,
                           void* ws, size_t ws_bytes, hipStream_t stream);

/* Quantized estimate: the same outputs as gem_score_exact, computed on the
 * quantized operands of D's format with their scales (products and float32
 * accumulation of scaled code products): D->dtype is GEM_FP8_E4M3 (a scale per
 * vector), GEM_MXFP4 or GEM_MXFP6 (a scale per 32-element block). Q is either
 * in D's format, or GEM_F32 and is quantized into the workspace by the rule of
 * gem_quantize_fp8 / gem_quantize_mxfp4 / gem_quantize_mxfp6. */
gem_status gem_score_quant(gem_ctx ctx, const gem_sets* Q, const gem_sets* D, const gem_cands* C,
                           int32_t k,
                           float* scores, int64_t ld_scores, const int32_t* score_rows,
                           float* top_scores, int32_t* top_ids,
                           void* ws, size_t ws_bytes, hipStream_t stream);

/* gem_score_quant without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc. Its workspace is a static device array of
 * GEM_STATIC_SCRATCH_BYTES that the library holds on each device it runs on
 * (its address is taken once per device in gem_create). The call allocates
 * nothing and computes exactly what gem_score_quant computes with the same
 * arguments (bitwise). A call whose workspace (gem_workspace_bytes with
 * GEM_OP_SCORE_QUANT) exceeds the array returns GEM_ERR_WORKSPACE with nothing
 * enqueued. Every call on a device shares that device's array and keeps the
 * last call's contents: calls that overlap on one device (other streams,
 * other threads, other contexts of the device) race and must be serialized by
 * the caller. */
#define GEM_STATIC_SCRATCH_BYTES (64 << 20)
gem_status gem_score_quant_static(gem_ctx ctx, const gem_sets* Q, const gem_sets* D, const gem_cands* C,
                                  int32_t k,
                                  float* scores, int64_t ld_scores, const int32_t* score_rows,
                                  float* top_scores, int32_t* top_ids, hipStream_t stream);

/* Segmented top-k (the k-argmax of Sec. 3.1 applied per segment).
 *   seg_offsets != NULL: segment i = scores[seg_offsets[i] .. seg_offsets[i+1]-1],
 *     ids from seg_ids (NULL: position within the segment). Entries with a
 *     negative id are skipped. A repeated id keeps its best entry.
 *   seg_offsets == NULL: segment i = scores[r * seg_ld .. r * seg_ld + seg_len - 1]
 *     with r = seg_rows ? seg_rows[i] : i; ids are positions; seg_ids must be NULL.
 *   Outputs [n_segs][k]. k <= GEM_MAX_K. */
gem_status gem_topk(gem_ctx ctx, const float* scores, const int64_t* seg_offsets,
                    const int32_t* seg_ids, int64_t n_segs, int64_t seg_len, int64_t seg_ld,
                    const int32_t* seg_rows, int32_t k, float* top_scores, int32_t* top_ids,
                    void* ws, size_t ws_bytes, hipStream_t stream);

/* One batched beam-expansion step (Alg. 5 neighbour loop, all queries at once):
 * estimate CH(Q_i, D_id) with quantized operands for every entry of list i,
 * then replace beam row i by the best ef of (beam row i) U (scored entries),
 * ids distinct (a repeated id keeps its best entry). D8->dtype is
 * GEM_FP8_E4M3, GEM_MXFP4 or GEM_MXFP6; Q8 is in D8's format or GEM_F32
 * (quantized into ws). If cand_scores is not NULL the step's entry scores
 * are also written there ([C->n_entries], in the caller's entry order). The
 * beam is updated in place. A step with n_lists x longest list >= 65,536
 * and lists of at most 2048 entries (rows, not code sets) first sorts every
 * list by document id into ws and walks the sorted lists chunk-major, so that
 * the listings of a document run close together in time; the workspace then
 * holds 8 bytes per entry more (gem_workspace_bytes includes it). */
gem_status gem_expand_batch(gem_ctx ctx, const gem_sets* Q8, const gem_sets* D8, const gem_cands* C,
                            gem_beam* beam, float* cand_scores,
                            void* ws, size_t ws_bytes, hipStream_t stream);

/* The merge half of gem_expand_batch on scores the caller already has:
 * beam row i becomes the best ef of (beam row i) U {(cand_scores[e], ids[e]) :
 * e in list i}, ids distinct (a repeated id keeps its best entry), padding ids
 * skipped. cand_scores: [device] [C->n_entries]. */
gem_status gem_beam_merge(gem_ctx ctx, const float* cand_scores, const gem_cands* C, gem_beam* beam,
                          hipStream_t stream);

/* Fill a beam with its padding (-inf, -1): an empty R before the first step. */
gem_status gem_beam_reset(gem_ctx ctx, gem_beam* beam, int64_t n_queries, hipStream_t stream);

/* On-demand validation of device data. Checks that offsets are non-decreasing,
 * inside [0, n_vecs] and (FP8) scales are positive powers of two; for candidate
 * lists, that offsets are non-decreasing inside [0, n_entries] and ids < n_sets.
 * Synchronizes `stream`; returns GEM_ERR_DEVICE_CHECK on a violation. */
gem_status gem_validate_sets(gem_ctx ctx, const gem_sets* S, hipStream_t stream);
gem_status gem_validate_cands(gem_ctx ctx, const gem_cands* C, int64_t n_sets, hipStream_t stream);

/* Entropic Earth Mover's Distance of set pairs (Sec. 4.2, Eq. EMD: the
 * transport plan with row sums 1/m1 and column sums 1/m2 minimizing
 * sum_ij t_ij d(p_i, p'_j), d Euclidean; with code sets it is Eq. qEMD over
 * the centroids). The Sinkhorn iteration of Cuturi (2013) in the log domain:
 * from g = 0, n_iter rounds of f_i = -log m1 - logsumexp_j(g_j - C_ij / eps),
 * g_j = -log m2 - logsumexp_i(f_i - C_ij / eps); out[p] = sum_ij
 * exp(f_i + g_j - C_ij / eps) C_ij for the pair (A set a_idx[p], B set
 * b_idx[p]), float32 throughout. Converges to EMD from above as eps -> 0.
 *   A, B: GEM_F32 sets or code sets over float32 codebooks; max_set_len <= 256.
 *   a_idx, b_idx: [device] [n_pairs] set indices (trusted); out: [device]
 *   [n_pairs]; an empty set gives NaN. eps > 0, 1 <= n_iter <= 100000.
 *   ws: [device] gem_emd_workspace_bytes(n_pairs) bytes (pair flags, and the
 *   cost matrices of pairs with more than 36864 entries, which a second pass
 *   keeps in device memory instead of LDS). */
size_t gem_emd_workspace_bytes(int64_t n_pairs);
gem_status gem_emd_sinkhorn(gem_ctx ctx, const gem_sets* A, const gem_sets* B, const int32_t* a_idx,
                            const int32_t* b_idx, int64_t n_pairs, float eps, int32_t n_iter, float* out, void* ws,
                            size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- search
 * Cluster-guided beam search (Alg. 5, Sec. 4.5) for a batch of queries, over
 * a graph whose sets carry the set-level clusters of Sec. 4.1. */

/* Set-level clustering with TF-IDF guided pruning (Sec. 4.1): for every set P,
 * TF(j, P) = its vectors whose cluster is j (vec_clusters[i] in [0, k2): the
 * nearest C_index centroid, e.g. from gem_nearest_centroid), IDF(j) =
 * log(N / (1 + sets with TF(j, .) > 0)) in float32, and C_top(P) = the r
 * clusters with the largest TF * IDF (ties to the smaller cluster; only
 * clusters P touches). Writes set_masks [n_sets][(k2 + 31) / 32] (bit j of a
 * mask: cluster j), member_offsets [k2 + 1] and members [<= n_sets * r]: the
 * sets of each cluster in id order. k2 <= 1024. ws: GEM_SEARCH_CLUSTER_WS
 * bytes [device]. */
#define GEM_SEARCH_CLUSTER_WS 8192
gem_status gem_set_clusters(gem_ctx ctx, const int32_t* vec_clusters, const int64_t* set_offsets, int64_t n_sets,
                            int32_t k2, int32_t r, uint32_t* set_masks, int64_t* member_offsets, int32_t* members,
                            void* ws, size_t ws_bytes, hipStream_t stream);

/* Cluster filter (Sec. 4.5, S = C Q^T): query_masks row i = the union over
 * query i's vectors of their top-t centroids by inner product (float32
 * products, ties to the smaller index). Q: GEM_F32 sets; centroids: [device]
 * [k2][128] float32 (C_index). */
gem_status gem_query_clusters(gem_ctx ctx, const gem_sets* Q, const float* centroids, int32_t k2, int32_t t,
                              uint32_t* query_masks, hipStream_t stream);

/* The graph: neighbour lists plus the outputs of gem_set_clusters. */
typedef struct {
  int64_t n_sets;                 /* sets of the graph (the scored document sets) */
  int32_t k2;                     /* clusters, <= 1024 */
  int32_t degree;                 /* neighbours per set, <= 64 */
  const int32_t* neighbors;       /* [device] [n_sets][degree], -1 padded */
  const uint32_t* set_masks;      /* [device] [n_sets][(k2 + 31) / 32] */
  const int64_t* member_offsets;  /* [device] [k2 + 1] */
  const int32_t* members;         /* [device] */
} gem_graph;

/* One batch's search state, caller-owned device buffers for n_q queries.
 * cand_ids / cand_scores rows hold max(k2, width * degree) entries. */
typedef struct {
  int32_t width;                  /* sets expanded per query and step (w) */
  int32_t reserved;
  const uint32_t* query_masks;    /* [n_q][(k2 + 31) / 32] (gem_query_clusters) */
  uint32_t* visited;              /* [n_q][(n_sets + 31) / 32] */
  uint32_t* expanded;             /* [n_q][(n_sets + 31) / 32] */
  int32_t* frontier;              /* [n_q][width] */
  int32_t* cand_ids;              /* [n_q][row] */
  float* cand_scores;             /* [n_q][row] */
  uint32_t* active;               /* [1]: queries that expanded something in the last step */
} gem_search_state;

/* Start a batch: clears the visited and expanded maps, takes one entry per
 * cluster of each query's C_query (member floor(u * count / 2^32) of the
 * cluster, u = random_words[i * k2 + j], drawn by the caller), scores the
 * entries and makes them the beam (R of Alg. 5; ef <= GEM_MAX_EF). Scores are
 * CH in D's dtype (the estimate for FP8 / MX sets, qCH for code sets); Q
 * must already be in D's dtype. */
gem_status gem_search_begin(gem_ctx ctx, const gem_sets* Q, const gem_sets* D, const gem_graph* G,
                            gem_search_state* S, const uint32_t* random_words, gem_beam* beam, hipStream_t stream);

/* One step for every query: the w best entries of R not yet expanded are
 * expanded; their neighbours that are unvisited and share a cluster with
 * C_query are marked visited, scored and merged into R. *S->active (device)
 * counts the queries that still had something to expand; the batch is done
 * when it reads 0. */
gem_status gem_search_step(gem_ctx ctx, const gem_sets* Q, const gem_sets* D, const gem_graph* G,
                           gem_search_state* S, gem_beam* beam, hipStream_t stream);

/* Schedule of the exhaustive (dense) scorer: how the work of one call is laid
 * out over the GPU. Persistent workgroups (slots_per_xcd on each of the 8 XCDs)
 * step through chunks of chunk_docs documents; each XCD's chunks are cut into
 * pieces so that every workgroup gets about items_per_slot (piece, query block
 * group) items. A schedule changes the time of a call, never its results:
 * every schedule computes bitwise the same scores.
 *   chunk_docs: 32 or 64; items_per_slot: 1..64; slots_per_xcd: 1..(CUs / 8).
 */
typedef struct {
  int32_t chunk_docs;
  int32_t items_per_slot;
  int32_t slots_per_xcd;
  int32_t reserved;
} gem_dense_schedule;

/* Schedules are kept per shape class: the compute dtype and the power-of-two
 * classes (floor(log2(x + 1))) of the query batch's vector count and of the
 * document count. A class without an installed schedule uses the library's
 * default (64-document chunks, 8 items per workgroup, one workgroup per CU).
 *   gem_get_dense_schedule: the schedule a dense call of this shape would use.
 *   gem_set_dense_schedule: install `sched` for the class (NULL: back to the default).
 */
gem_status gem_get_dense_schedule(gem_ctx ctx, int32_t dtype, int64_t q_rows, int64_t n_docs,
                                  gem_dense_schedule* out);
gem_status gem_set_dense_schedule(gem_ctx ctx, int32_t dtype, int64_t q_rows, int64_t n_docs,
                                  const gem_dense_schedule* sched);

/* Autotuner for the dense scorer. Runs the exhaustive scoring of Q against D
 * (as gem_score_exact / gem_score_quant with C = NULL and k = 0 would, writing
 * scores [n_q][ld_scores]) once untimed and `reps` (1..100) times timed under
 * each candidate schedule, installs the fastest for the call's shape class and
 * returns it with its mean time per call in milliseconds. Synchronizes `stream`.
 * The candidates: the library default, then chunk_docs (64, 32) x
 * items_per_slot (2, 4, 8, 16) at one workgroup per CU, then 3/4 and 1/2 of
 * the workgroups per XCD for the best of those. A candidate's time is the
 * median of three rounds of `reps` calls, and it displaces the best so far
 * only when faster by more than 0.5 % (so near ties keep the earlier, and the
 * choice is stable from run to run). The workspace must hold
 * gem_workspace_bytes(ctx, op, Q, D, NULL, compute, 0, 1) bytes (op
 * GEM_OP_SCORE_EXACT, or GEM_OP_SCORE_QUANT for FP8 / MXFP4 / MXFP6).
 */
gem_status gem_autotune_dense(gem_ctx ctx, const gem_sets* Q, const gem_sets* D, int32_t compute, float* scores,
                              int64_t ld_scores, void* ws, size_t ws_bytes, hipStream_t stream, int32_t reps,
                              gem_dense_schedule* best, float* best_ms);

/* Schedule of the gathered scorer (candidate lists: the rerank, beam
 * expansion and search steps): entries of a list per wave (1..64; 0 = the
 * library's rule: 16, or fewer when a call has too few entries to fill the
 * GPU) and document tiles in flight per wave (one of three depths per format:
 * F32 1/2/3, BF16 2/4/6, FP8 4/6/8, MXFP4 6/8/12, MXFP6 4/6/8; 0 or the middle one is the
 * default). Kept per shape class: the compute dtype and the power-of-two
 * classes of the list count and of the longest list. A schedule changes the
 * time of a call, never its results. */
typedef struct {
  int32_t entries_per_wave;
  int32_t depth;
  int32_t reserved[2];
} gem_gather_schedule;
gem_status gem_get_gather_schedule(gem_ctx ctx, int32_t dtype, int64_t n_lists, int64_t max_list_len,
                                   gem_gather_schedule* out);
gem_status gem_set_gather_schedule(gem_ctx ctx, int32_t dtype, int64_t n_lists, int64_t max_list_len,
                                   const gem_gather_schedule* sched);

/* Autotuner for the gathered scorer: runs the scoring of Q's candidate lists C
 * against D (as gem_score_exact / gem_score_quant with k = 0 would, writing
 * scores [C->n_entries]) under the library rule and every entries_per_wave in
 * (0, 8, 16, 32, 64) x depth, with the timing and tie rule of
 * gem_autotune_dense; installs the fastest for the call's shape class.
 * Synchronizes `stream`. ws: gem_workspace_bytes(ctx, op, Q, D, C, compute, 0, 1). */
gem_status gem_autotune_gather(gem_ctx ctx, const gem_sets* Q, const gem_sets* D, const gem_cands* C,
                               int32_t compute, float* scores, void* ws, size_t ws_bytes, hipStream_t stream,
                               int32_t reps, gem_gather_schedule* best, float* best_ms);

/* The tune cache: every installed dense and gathered schedule of the context,
 * keyed by (architecture, kind, dtype, shape class), as a JSON document at
 * `path` (host file I/O only). gem_load_tune_cache installs a cache's entries
 * for this GPU's architecture (a missing or invalid file is an error;
 * nothing is installed from an invalid one); gem_create does the same. */
gem_status gem_save_tune_cache(gem_ctx ctx, const char* path);
gem_status gem_load_tune_cache(gem_ctx ctx, const char* path);

#ifdef __cplusplus
}
#endif

#endif /* GEM_H_ */
