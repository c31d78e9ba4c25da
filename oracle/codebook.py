"""Centroid codebook and the quantized Chamfer estimate qCH in float64 -- TEST INFRASTRUCTURE ONLY.

Restates from the paper (GEM, arXiv 2603.20336):
  * the vocabulary C_quant: k-means centroids of a sample of all document
    vectors (Sec. 4.1, first stage of the two-stage clustering);
  * NN(x), the centroid of C_quant nearest to x, which replaces every vector
    in the quantized distances (Sec. 4.2, "Quantization": d_X(p, p') is
    approximated by d_X(NN(p), NN(p')));
  * qCH(Q, P) = sum over q in Q of the best d_X(NN(q), NN(p)) over p in P
    (Sec. 4.5, Eq. qCH), here in the similarity form used throughout:
    sum_q max_p <NN(q), NN(p)>;
  * the codebook size rule: the power of two 2^floor(log2(16 sqrt(#vectors)))
    (Sec. 5.1, parameter settings).

Readings (each listed in the design notes):
  * NN is nearest in Euclidean distance, the k-means objective; ties go to the
    smallest centroid index.
  * One Lloyd iteration assigns every sample to NN and moves each centroid to
    the mean of its members; a centroid without members stays where it is.
  * The similarity inside qCH is the inner product of the two centroids, as in
    CH (Def. 1); centroids are not renormalized.
"""
from __future__ import annotations

import math

import numpy as np

from .chamfer import ch_dense, ch_cands, ch_pair


def _f64(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64)


def codebook_size(n_vectors: int) -> int:
    """|C_quant| = 2^floor(log2(16 * sqrt(n_vectors)))  (Sec. 5.1)."""
    return 1 << int(math.floor(math.log2(16.0 * math.sqrt(n_vectors))))


def sq_distances(x, C, chunk: int = 4096) -> np.ndarray:
    """||x_i - C_j||^2 for every row i and centroid j, summed term by term in float64."""
    x, C = _f64(x), _f64(C)
    out = np.empty((x.shape[0], C.shape[0]))
    for a in range(0, x.shape[0], chunk):
        xa = x[a:a + chunk]
        diff = xa[:, None, :] - C[None, :, :]
        out[a:a + chunk] = (diff * diff).sum(axis=2)
    return out


def nn_assign(x, C) -> np.ndarray:
    """NN(x_i) as a centroid index: argmin_j ||x_i - C_j||^2, smallest j on ties (Sec. 4.2)."""
    return np.argmin(sq_distances(x, C), axis=1).astype(np.int64)


def lloyd_update(x, codes, C) -> np.ndarray:
    """One k-means centroid update: each centroid becomes the mean of the rows
    assigned to it; a centroid with no rows keeps its position."""
    x, C = _f64(x), _f64(C)
    codes = np.asarray(codes, np.int64)
    new = C.copy()
    for j in range(C.shape[0]):
        members = x[codes == j]
        if members.shape[0] > 0:
            new[j] = members.sum(axis=0) / members.shape[0]
    return new


def kmeans(x, init, n_iter: int):
    """Lloyd's algorithm from the given initial centroids: n_iter rounds of
    (assign, update). Returns (centroids, codes of the last assignment)."""
    C = _f64(init).copy()
    codes = np.zeros(np.asarray(x).shape[0], np.int64)
    for _ in range(n_iter):
        codes = nn_assign(x, C)
        C = lloyd_update(x, codes, C)
    return C, codes


def kmeans_objective(x, codes, C) -> float:
    """Sum of squared distances of the rows to their assigned centroids."""
    x, C = _f64(x), _f64(C)
    d = x - C[np.asarray(codes, np.int64)]
    return float((d * d).sum())


def qch_pair(q_codes, p_codes, C) -> float:
    """qCH(Q, P) = sum_q max_p <NN(q), NN(p)>, with NN(.) given as codes into C (Sec. 4.5)."""
    C = _f64(C)
    return ch_pair(C[np.asarray(q_codes, np.int64)], C[np.asarray(p_codes, np.int64)])


def qch_dense(q_codes, q_offsets, d_codes, d_offsets, C) -> np.ndarray:
    """qCH of every query set against every document set -> [n_q, n_d] float64.
    The sets hold codes; each code stands for its centroid's vector."""
    C = _f64(C)
    return ch_dense(C[np.asarray(q_codes, np.int64)], q_offsets, C[np.asarray(d_codes, np.int64)], d_offsets)


def qch_cands(q_codes, q_offsets, d_codes, d_offsets, cand_offsets, cand_ids, C) -> np.ndarray:
    """qCH of each query set against its listed documents (CSR), in list order."""
    C = _f64(C)
    return ch_cands(C[np.asarray(q_codes, np.int64)], q_offsets, C[np.asarray(d_codes, np.int64)], d_offsets,
                    cand_offsets, cand_ids)
