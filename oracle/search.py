"""Cluster-guided beam search (Alg. 5) in float64 -- TEST INFRASTRUCTURE ONLY.

Restates from the paper (GEM, arXiv 2603.20336):
  * set-level clustering with TF-IDF guided pruning (Sec. 4.1): every vector
    p of a set P is assigned to its nearest coarse centroid NN(p) in C_index;
    TF(j, P) counts P's vectors assigned to cluster j; IDF(j) = log(N / (1 +
    #sets with TF(j, .) > 0)); C_top(P) is the r clusters of P with the
    highest TF * IDF;
  * cluster filtering (Sec. 4.5, Eq. S = C Q^T): C_query is the union over the
    query's vectors of their top-t centroids of C_index by inner product;
  * multi-entry initialization: one random set from each cluster of C_query;
  * the search of Alg. 5: sets are expanded from the best unexpanded result,
    a neighbour is scored only if it is unvisited and one of its C_top clusters
    is in C_query, the result set R keeps the best ef; the top-k of R are
    reranked by exact CH.

Readings (each listed in the design notes):
  * the second-stage k-means clusters the C_quant centroids (Sec. 4.1); a
    vector's cluster is the nearest C_index centroid (Euclidean, ties to the
    smaller index), as for NN in Sec. 4.2;
  * r (the number of clusters per set) is fixed per index; ties in TF * IDF and
    in the top-t go to the smaller cluster index; a cluster a set does not
    touch is never in its C_top (TF = 0);
  * members of a cluster are the sets whose C_top holds it, in id order; the
    random entry of cluster j is member floor(u_j * count_j / 2^32) for a
    random 32-bit word u_j the caller draws;
  * the parallel paths of Alg. 5 become one batched loop per query: each step
    takes the w best entries of R not yet expanded (all paths advance at once),
    marks them expanded, and scores their unvisited, unpruned neighbours
    (neighbour lists in order, visited marks set when a neighbour is taken); a
    query ends when R holds no unexpanded entry, which is where every path of
    Alg. 5 has stopped (a popped set worse than tau is not in R).
"""
from __future__ import annotations

import math

import numpy as np

from .chamfer import _order, ch_pair


def tfidf_top_clusters(vec_clusters, offsets, k2: int, r: int):
    """C_top(P) of every set: (list of sorted cluster arrays, IDF [k2] float64)."""
    vc = np.asarray(vec_clusters, np.int64)
    off = np.asarray(offsets, np.int64)
    n = len(off) - 1
    tf = np.zeros((n, k2), np.int64)
    for i in range(n):
        for j in vc[off[i]:off[i + 1]]:
            tf[i, j] += 1
    df = (tf > 0).sum(axis=0)
    idf = np.array([math.log(n / (1.0 + df[j])) for j in range(k2)])
    out = []
    for i in range(n):
        cand = [j for j in range(k2) if tf[i, j] > 0]
        cand.sort(key=lambda j: (-(tf[i, j] * idf[j]), j))
        out.append(np.array(sorted(cand[:r]), np.int64))
    return out, idf


def cluster_members(ctop, k2: int):
    """Members of each cluster: the sets whose C_top holds it, in id order."""
    members = [[] for _ in range(k2)]
    for i, cs in enumerate(ctop):
        for j in cs:
            members[int(j)].append(i)
    return [np.array(m, np.int64) for m in members]


def query_clusters(q_vecs, centroids, t: int) -> np.ndarray:
    """C_query: union over the query's vectors of the top-t centroids by <c, q>
    (S = C Q^T), ties to the smaller index. Returns the sorted cluster ids."""
    S = np.asarray(q_vecs, np.float64) @ np.asarray(centroids, np.float64).T     # [m_q, k2]
    chosen = set()
    for row in S:
        order = sorted(range(len(row)), key=lambda j: (-row[j], j))
        chosen.update(order[:t])
    return np.array(sorted(chosen), np.int64)


def entry_points(cq, members, u) -> np.ndarray:
    """One set per cluster of C_query (member floor(u_j * count_j / 2^32) for the
    random 32-bit words u), duplicates dropped."""
    out = []
    for j in cq:
        m = members[int(j)]
        if len(m) == 0:
            continue
        pick = int(m[(int(u[int(j)]) * len(m)) >> 32])
        if pick not in out:
            out.append(pick)
    return np.array(out, np.int64)


def _top(entries, ef):
    if not entries:
        return []
    s = np.array([e[0] for e in entries])
    i = np.array([e[1] for e in entries])
    o = _order(s, i)
    seen, out = set(), []
    for k in o:
        if int(i[k]) in seen:
            continue
        seen.add(int(i[k]))
        out.append((float(s[k]), int(i[k])))
        if len(out) == ef:
            break
    return out


def beam_search(score, neighbors, ctop, cq, entries, ef: int, w: int, max_steps: int = 10 ** 9):
    """The batched reading of Alg. 5 for one query.

    score(ids) -> scores of the listed sets; neighbors[p]: neighbour ids of set
    p (negative = none); ctop[p]: its C_top clusters; cq: C_query.
    Returns (R as a list of (score, id), best first; number of sets scored; steps).
    """
    cqs = set(int(j) for j in cq)
    visited = set(int(e) for e in entries)
    s0 = score(list(entries)) if len(entries) else []
    R = _top([(float(a), int(b)) for a, b in zip(s0, entries)], ef)
    n_scored = len(entries)
    expanded = set()
    steps = 0
    while steps < max_steps:
        frontier = [i for (_, i) in R if i not in expanded][:w]
        if not frontier:
            break
        expanded.update(frontier)
        cand = []
        for p in frontier:
            for nb in neighbors[p]:
                nb = int(nb)
                if nb < 0 or nb in visited:
                    continue
                if not (set(int(j) for j in ctop[nb]) & cqs):
                    continue
                visited.add(nb)
                cand.append(nb)
        if cand:
            sc = score(cand)
            n_scored += len(cand)
            R = _top(R + [(float(a), int(b)) for a, b in zip(sc, cand)], ef)
        steps += 1
    return R, n_scored, steps


def ch_scorer(q_vals, d_vals, d_offsets):
    """score(ids) for beam_search: CH of the query against the listed sets, on the given operand values."""
    d_off = np.asarray(d_offsets, np.int64)

    def score(ids):
        return [ch_pair(q_vals, d_vals[d_off[i]:d_off[i + 1]]) for i in ids]
    return score
