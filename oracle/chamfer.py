"""Chamfer scoring, top-k, bounded beam and recall in float64 -- TEST INFRASTRUCTURE ONLY.

Plain NumPy restatements of the paper's definitions (GEM, arXiv 2603.20336).
A matrix product is used as the step that forms all inner products <a, p>;
nothing is blocked, fused or reordered beyond that.

Readings where the paper is silent or loose (each one is listed with its
justification in the design notes):
  * Sim(a, b) is the inner product (Def. 1 allows cosine; inputs are unit
    vectors, so the two coincide) and CH is a sum, not an average.
  * CH is a similarity: top-k means largest first. Ties order by smaller id.
  * An empty query set scores 0 (empty sum); a non-empty query against an
    empty document scores -inf (max over nothing).
  * top-k keeps ids distinct (the best entry of a repeated id wins) and pads
    with (-inf, -1) when fewer than k entries exist.
  * A negative id is padding (of a candidate list, a segment or the beam): it
    is never ranked, whatever its score.
"""
from __future__ import annotations

import numpy as np

from .codecs import bf16_decode, split_bf16x3

NEG_INF = -np.inf


def _f64(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64)


def ch_pair(A, B) -> float:
    """CH(A, B) = sum over a in A of max over b in B of <a, b>  (Def. 1, Eq. ch)."""
    A, B = _f64(A), _f64(B)
    if A.shape[0] == 0:
        return 0.0
    if B.shape[0] == 0:
        return NEG_INF
    S = A @ B.T                     # all inner products <a, b>
    return float(S.max(axis=1).sum())


def _segment_max_cols(S: np.ndarray, starts: np.ndarray, lens: np.ndarray) -> np.ndarray:
    """max over the columns of each segment; -inf for empty segments."""
    out = np.full((S.shape[0], len(starts)), NEG_INF)
    nz = lens > 0
    if nz.any():
        out[:, nz] = np.maximum.reduceat(S, starts[nz], axis=1)
    return out


def _dot_plain(A: np.ndarray, D: np.ndarray) -> np.ndarray:
    """<a, p> for every row a of A and p of D."""
    return _f64(A) @ _f64(D).T


def _split_parts(X) -> tuple[np.ndarray, np.ndarray]:
    hi, lo = split_bf16x3(X)
    return bf16_decode(hi), bf16_decode(lo)


def _dot_bf16x3(A: np.ndarray, D: np.ndarray) -> np.ndarray:
    """The split-bfloat16 inner products: with a = ah + al + ea and p = ph + pl + ep
    (codecs.split_bf16x3), <a, p> taken as <ah, ph> + <ah, pl> + <al, ph>, every
    term exact (float64 here), the al*pl and ea / ep terms dropped."""
    ah, al = _split_parts(A)
    ph, pl = _split_parts(D)
    return ah @ ph.T + (ah @ pl.T + al @ ph.T)


def ch_dense(q_vecs, q_offsets, d_vecs, d_offsets, max_rows: int = 1 << 20, dot=_dot_plain) -> np.ndarray:
    """CH(Q_i, P_j) for every query set i and document set j -> [n_q, n_d] float64.

    The problem statement of Sec. 3.1 ranks every document of the database by
    CH; this is that full score matrix. Documents are processed in groups of at
    most `max_rows` vectors to bound memory. `dot` gives the matrix of inner
    products of two row blocks (the exact one by default).
    """
    qv, dv = np.asarray(q_vecs), np.asarray(d_vecs)
    qo, do = np.asarray(q_offsets, np.int64), np.asarray(d_offsets, np.int64)
    n_q, n_d = len(qo) - 1, len(do) - 1
    out = np.zeros((n_q, n_d))
    # document groups of bounded row count
    groups, j = [], 0
    while j < n_d:
        j1 = j + 1
        while j1 < n_d and do[j1 + 1] - do[j] <= max_rows:
            j1 += 1
        groups.append((j, j1))
        j = j1
    for (j0, j1) in groups:
        r0, r1 = do[j0], do[j1]
        D = dv[r0:r1]
        starts = do[j0:j1] - r0
        lens = do[j0 + 1:j1 + 1] - do[j0:j1]
        for i in range(n_q):
            A = qv[qo[i]:qo[i + 1]]
            if A.shape[0] == 0:
                out[i, j0:j1] = 0.0
                continue
            S = dot(A, D)                                # <a, p> for all a in Q_i, p in group
            r = _segment_max_cols(S, starts, lens)       # max over p in each document
            out[i, j0:j1] = r.sum(axis=0)                # sum over a in Q_i
    return out


def ch_cands(q_vecs, q_offsets, d_vecs, d_offsets, cand_offsets, cand_ids, dot=_dot_plain) -> np.ndarray:
    """CH(Q_i, P_id) for every entry of each query's candidate list -> flat float64.

    The candidate lists stand for the neighbours a beam-search step scores
    (Alg. 5, neighbour loop) or for the shortlist that is reranked by exact CH
    (Alg. 5, final step). `dot` as in ch_dense.
    """
    qv, dv = np.asarray(q_vecs), np.asarray(d_vecs)
    qo, do = np.asarray(q_offsets, np.int64), np.asarray(d_offsets, np.int64)
    co, ci = np.asarray(cand_offsets, np.int64), np.asarray(cand_ids, np.int64)
    out = np.zeros(len(ci))
    for i in range(len(qo) - 1):
        a, b = co[i], co[i + 1]
        if a == b:
            continue
        A = qv[qo[i]:qo[i + 1]]
        ids = ci[a:b]
        if A.shape[0] == 0:
            out[a:b] = 0.0
            continue
        lens = do[ids + 1] - do[ids]
        rows = np.concatenate([np.arange(do[d], do[d + 1]) for d in ids]) if lens.sum() else np.zeros(0, np.int64)
        G = dv[rows]
        starts = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
        S = dot(A, G)
        r = _segment_max_cols(S, starts, lens)
        out[a:b] = r.sum(axis=0)
    return out


def ch_dense_bf16x3(q_vecs, q_offsets, d_vecs, d_offsets, max_rows: int = 1 << 20) -> np.ndarray:
    """CH of float32 sets with every inner product taken in the split-bfloat16
    form (_dot_bf16x3): what the three-bfloat16-product exact mode computes,
    up to its float32 accumulation."""
    return ch_dense(q_vecs, q_offsets, d_vecs, d_offsets, max_rows, dot=_dot_bf16x3)


def ch_cands_bf16x3(q_vecs, q_offsets, d_vecs, d_offsets, cand_offsets, cand_ids) -> np.ndarray:
    """ch_cands with the split-bfloat16 inner products."""
    return ch_cands(q_vecs, q_offsets, d_vecs, d_offsets, cand_offsets, cand_ids, dot=_dot_bf16x3)


def _order(scores: np.ndarray, ids: np.ndarray) -> np.ndarray:
    """Indices ordering entries by score descending, then id ascending."""
    return np.lexsort((ids, -scores))


def _topk_one(scores: np.ndarray, ids: np.ndarray, k: int):
    live = np.asarray(ids) >= 0                          # a negative id is padding, never ranked
    scores, ids = np.asarray(scores)[live], np.asarray(ids)[live]
    o = _order(scores, ids)
    s, i = scores[o], ids[o]
    _, first = np.unique(i, return_index=True)         # first occurrence = best entry of each id
    keep = np.zeros(len(i), bool)
    keep[first] = True
    s, i = s[keep], i[keep]
    ts = np.full(k, NEG_INF)
    ti = np.full(k, -1, np.int64)
    n = min(k, len(s))
    ts[:n], ti[:n] = s[:n], i[:n]
    return ts, ti


def topk_rows(scores, k: int, ids=None):
    """Per row of a [n, L] score matrix: top-k (score desc, id asc), ids = column index."""
    S = _f64(scores)
    n, L = S.shape
    ts = np.full((n, k), NEG_INF)
    ti = np.full((n, k), -1, np.int64)
    col = np.arange(L, dtype=np.int64) if ids is None else np.asarray(ids, np.int64)
    for r in range(n):
        ts[r], ti[r] = _topk_one(S[r], col, k)
    return ts, ti


def topk_segments(scores, seg_offsets, k: int, seg_ids=None):
    """Top-k of each CSR segment. Ids are seg_ids entries, or positions within the segment."""
    s = _f64(scores)
    off = np.asarray(seg_offsets, np.int64)
    n = len(off) - 1
    ts = np.full((n, k), NEG_INF)
    ti = np.full((n, k), -1, np.int64)
    for r in range(n):
        a, b = off[r], off[r + 1]
        ids = np.arange(b - a, dtype=np.int64) if seg_ids is None else np.asarray(seg_ids[a:b], np.int64)
        ts[r], ti[r] = _topk_one(s[a:b], ids, k)
    return ts, ti


def beam_merge(beam_scores, beam_ids, cand_scores, cand_offsets, cand_ids, ef: int):
    """One update of the bounded result set R (Alg. 5): insert the step's scored
    candidates, keep ids distinct, keep the best ef (evicting the worst).

    beam_* are [n_q, ef]; candidates are CSR per query; padding ids (negative)
    on either side are ignored.
    """
    bs, bi = _f64(beam_scores), np.asarray(beam_ids, np.int64)
    cs, ci = _f64(cand_scores), np.asarray(cand_ids, np.int64)
    co = np.asarray(cand_offsets, np.int64)
    n = bs.shape[0]
    out_s = np.full((n, ef), NEG_INF)
    out_i = np.full((n, ef), -1, np.int64)
    for q in range(n):
        live = bi[q] >= 0
        s = np.concatenate([bs[q][live], cs[co[q]:co[q + 1]]])
        i = np.concatenate([bi[q][live], ci[co[q]:co[q + 1]]])
        out_s[q], out_i[q] = _topk_one(s, i, ef)
    return out_s, out_i


def beam_replay(n_q: int, ef: int, steps):
    """Run beam_merge over a list of steps [(cand_scores, cand_offsets, cand_ids)], from an empty beam."""
    bs = np.full((n_q, ef), NEG_INF)
    bi = np.full((n_q, ef), -1, np.int64)
    for (cs, co, ci) in steps:
        bs, bi = beam_merge(bs, bi, cs, co, ci, ef)
    return bs, bi


def recall_at_k(got_ids, exact_scores_row, k: int, tau: float = 0.0) -> float:
    """Recall@k (Sec. 5.1) with the exact top-k as ground truth, tie-aware.

    A returned id counts as a hit when its exact score is at least the exact
    k-th score minus tau, so that any member of a tie at the k-th place counts.
    Repeated or padding ids count once / never.
    """
    ex = _f64(exact_scores_row)
    k_eff = min(k, len(ex))
    if k_eff == 0:
        return 1.0
    sk = np.sort(ex)[::-1][k_eff - 1]
    got = [int(g) for g in np.asarray(got_ids)[:k] if int(g) >= 0]
    got = list(dict.fromkeys(got))
    hits = sum(1 for g in got if ex[g] >= sk - tau)
    return min(hits, k_eff) / k_eff


def tie_aware_match(got_ids, exact_scores_row, k: int, tau: float):
    """Check a returned top-k against exact scores outside the tie band.

    With s_k the exact k-th score: every returned id must score >= s_k - tau,
    and every document scoring > s_k + tau must be returned. Returns
    (ok, n_bad_members, n_missing).
    """
    ex = _f64(exact_scores_row)
    k_eff = min(k, len(ex))
    got = np.asarray(got_ids)[:k]
    got = got[got >= 0]
    if k_eff == 0:
        return len(got) == 0, len(got), 0
    sk = np.sort(ex)[::-1][k_eff - 1]
    bad = int(np.sum(ex[got] < sk - tau))
    must = np.nonzero(ex > sk + tau)[0]
    missing = int(len(np.setdiff1d(must, got)))
    dup = len(got) != len(np.unique(got))
    return (bad == 0 and missing == 0 and not dup and len(got) == k_eff), bad, missing
