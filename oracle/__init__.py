"""CPU oracle for set-to-set (Chamfer / MaxSim) scoring -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, float64 NumPy restatement of what the scoring
path computes, written from the paper (GEM, arXiv 2603.20336):

  * Chamfer similarity, Def. 1 / Eq. (ch) in Sec. 3.1:  CH(A,B) = sum_a max_b <a,b>
  * the multi-vector retrieval problem, Sec. 3.1: k-argmax of CH over the database
  * the bounded result set R of Alg. 5 (Sec. 4.5): keep at most ef, evict the worst
  * the final exact rerank of Alg. 5 and the #rerank pool (Sec. 5, "Effect of #rerank")
  * Recall@k, Sec. 5.1 "Evaluation Metrics"
  * the centroid codebook C_quant (k-means, Sec. 4.1), the nearest-centroid map
    NN (Sec. 4.2) and the quantized Chamfer estimate qCH (Sec. 4.5, Eq. qCH)
  * the cluster-guided beam search of Alg. 5 (Sec. 4.5) with the TF-IDF
    set-level clustering of Sec. 4.1, in a batched reading
  * EMD between vector sets (Sec. 4.2, Eq. EMD / qEMD), exact and as the
    entropic Sinkhorn approximation the GPU computes
  * MXFP4 and MXFP6 (OCP Microscaling, E2M1 / E2M3 elements with one
    power-of-two scale per 32-element block), the ultra-low-bit estimates the
    paper names as future work (Sec. 6)
  * the exact mode whose float32 products run as three bfloat16 products
    (each float32 value split into two bfloat16 parts)
  * the bf16 / OCP FP8 E4M3 codecs used for the quantized estimate (the paper's
    qCH replaces vectors by coarser codes, Sec. 4.2 "Quantization"; here the
    code is an FP8 E4M3 value times a per-vector power-of-two scale)

Only tests, the package's smoke check and the benchmark's CPU-baseline leg may
import it. The GPU library never calls it and shares no code with it: no
kernels, headers, helpers or tables.

Pins (what ties this oracle to something other than itself) live in
tests/test_oracle_pins.py: the paper's worked example (Sec. 1), closed forms,
invariants, reductions to BLAS / sorting, the OCP FP8 definition and torch's
independent float8 / bfloat16 casts.
"""
from .chamfer import (ch_pair, ch_dense, ch_cands, ch_dense_bf16x3, ch_cands_bf16x3, topk_rows, topk_segments,
                      beam_merge, beam_replay, recall_at_k, tie_aware_match)
from .codebook import (codebook_size, sq_distances, nn_assign, lloyd_update, kmeans, kmeans_objective,
                       qch_pair, qch_dense, qch_cands)
from .search import (tfidf_top_clusters, cluster_members, query_clusters, entry_points, beam_search,
                     ch_scorer)
from .emd import cost_matrix, emd_exact, sinkhorn, chamfer_distance
from .mx import (e2m1_decode, e2m1_table, e2m1_encode, block_exponent, quantize_mxfp4, dequantize_mxfp4,
                 e2m3_decode, e2m3_table, e2m3_encode, quantize_mxfp6, dequantize_mxfp6)
from .codecs import (bf16_round_bits, bf16_decode, split_bf16x3, e4m3_decode, e4m3_decode_table,
                     e4m3_encode, pow2_scale, quantize_fp8, dequantize_fp8)

__all__ = [
    "ch_pair", "ch_dense", "ch_cands", "ch_dense_bf16x3", "ch_cands_bf16x3", "topk_rows", "topk_segments",
    "beam_merge", "beam_replay", "recall_at_k", "tie_aware_match",
    "bf16_round_bits", "bf16_decode", "split_bf16x3", "e4m3_decode", "e4m3_decode_table", "e4m3_encode",
    "pow2_scale", "quantize_fp8", "dequantize_fp8",
    "codebook_size", "sq_distances", "nn_assign", "lloyd_update", "kmeans", "kmeans_objective",
    "qch_pair", "qch_dense", "qch_cands",
    "tfidf_top_clusters", "cluster_members", "query_clusters", "entry_points", "beam_search", "ch_scorer",
    "cost_matrix", "emd_exact", "sinkhorn", "chamfer_distance",
    "e2m1_decode", "e2m1_table", "e2m1_encode", "block_exponent", "quantize_mxfp4", "dequantize_mxfp4",
]
