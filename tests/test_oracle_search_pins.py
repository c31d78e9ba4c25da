"""Pins for the oracle's cluster-guided search (Alg. 5, batched reading).

Sources of truth: reductions to brute force (a complete graph, or ef and w
large enough to exhaust a connected graph, give the exhaustive top-ef of every
reachable set), closed forms of the TF-IDF clustering for special shapes,
NumPy's stable argsort for the top-t of S = C Q^T, and invariants (a pruned
cluster is never scored, no set is scored twice).
"""
import math

import numpy as np

import oracle
from oracle import search as osr


def _csr(lengths):
    o = np.zeros(len(lengths) + 1, np.int64)
    o[1:] = np.cumsum(lengths)
    return o


def _unit(rng, n, d=16):
    x = rng.standard_normal((n, d))
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def test_tfidf_with_r_covering_all_is_the_touched_clusters():
    rng = np.random.default_rng(0)
    lens = rng.integers(0, 9, 40)
    vc = rng.integers(0, 12, int(lens.sum()))
    off = _csr(lens)
    ctop, idf = osr.tfidf_top_clusters(vc, off, 12, r=12)
    for i in range(40):
        np.testing.assert_array_equal(ctop[i], np.unique(vc[off[i]:off[i + 1]]))
    # IDF = log(N / (1 + DF)) with DF from bincount
    df = np.array([sum(1 for i in range(40) if j in set(vc[off[i]:off[i + 1]])) for j in range(12)])
    np.testing.assert_allclose(idf, np.log(40 / (1.0 + df)))


def test_tfidf_with_equal_document_frequency_ranks_by_count():
    # every set touches every cluster: DF is the same for all clusters, so the
    # top-r are the r most frequent clusters of each set (ties: smaller index)
    rng = np.random.default_rng(1)
    k2, n = 6, 30
    vc, lens = [], []
    for _ in range(n):
        extra = rng.integers(0, k2, rng.integers(0, 10))
        v = np.concatenate([np.arange(k2), extra])
        vc.append(v)
        lens.append(len(v))
    vc = np.concatenate(vc)
    off = _csr(lens)
    ctop, idf = osr.tfidf_top_clusters(vc, off, k2, r=2)
    for i in range(n):
        cnt = np.bincount(vc[off[i]:off[i + 1]], minlength=k2)
        want = sorted(np.argsort(-cnt, kind="stable")[:2])
        if idf[0] < 0:                      # log(N / (N + 1)) < 0: the ranking flips to the rarest
            want = sorted(np.argsort(cnt, kind="stable")[:2])
        np.testing.assert_array_equal(ctop[i], want)
    assert math.isclose(idf[0], math.log(n / (n + 1.0)))


def test_query_clusters_match_stable_argsort():
    rng = np.random.default_rng(2)
    C = _unit(rng, 20)
    q = _unit(rng, 7)
    got = osr.query_clusters(q, C, t=3)
    S = q @ C.T
    want = sorted(set(np.concatenate([np.argsort(-row, kind="stable")[:3] for row in S]).tolist()))
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(osr.query_clusters(q, C, t=20), np.arange(20))


def test_entry_points_closed_forms():
    members = [np.array([3, 5, 9]), np.array([]), np.array([5, 7])]
    top = 2 ** 32 - 1
    np.testing.assert_array_equal(osr.entry_points([0, 1, 2], members, np.zeros(3, np.uint64)), [3, 5])
    np.testing.assert_array_equal(osr.entry_points([0, 2], members, np.array([top, 0, 2 ** 31], np.uint64)), [9, 7])
    # 2^32 / 3 picks member 1 of 3 (5), and member 0 of cluster 2 is 5 again: dropped
    np.testing.assert_array_equal(osr.entry_points([0, 2], members, np.array([2 ** 32 // 3 + 1, 0, 0], np.uint64)), [5])


def _problem(seed, n=60):
    rng = np.random.default_rng(seed)
    lens = rng.integers(1, 6, n)
    dv = _unit(rng, int(lens.sum()))
    off = _csr(lens)
    q = _unit(rng, 4)
    score = osr.ch_scorer(q, dv, off)
    exact = np.array(score(list(range(n))))
    return rng, off, dv, q, score, exact


def test_complete_graph_gives_the_exhaustive_top_ef():
    rng, off, dv, q, score, exact = _problem(3)
    n = len(off) - 1
    nbrs = [np.array([j for j in range(n) if j != i]) for i in range(n)]
    ctop = [np.array([0])] * n
    R, scored, _ = osr.beam_search(score, nbrs, ctop, [0], [17], ef=10, w=1)
    want_s, want_i = oracle.topk_rows(exact[None], 10)
    assert [i for _, i in R] == list(want_i[0])
    np.testing.assert_allclose([s for s, _ in R], want_s[0])
    assert scored == n                       # every set scored exactly once


def test_exhausting_a_connected_graph_gives_the_reachable_top_ef():
    rng, off, dv, q, score, exact = _problem(4)
    n = len(off) - 1
    # a ring plus random chords: connected; ef = n keeps everything, so the
    # search expands every set and R is the exhaustive ranking
    nbrs = [np.array([(i + 1) % n, (i - 1) % n] + list(rng.integers(0, n, 3))) for i in range(n)]
    ctop = [np.array([i % 3]) for i in range(n)]
    R, scored, steps = osr.beam_search(score, nbrs, ctop, [0, 1, 2], [5], ef=n, w=2)
    want_s, want_i = oracle.topk_rows(exact[None], n)
    assert [i for _, i in R] == list(want_i[0])
    assert scored == n and steps >= n // 2


def test_pruned_clusters_are_never_scored():
    rng, off, dv, q, score, exact = _problem(5)
    n = len(off) - 1
    nbrs = [np.array([(i + 1) % n, (i + 7) % n, (i + 13) % n]) for i in range(n)]
    ctop = [np.array([i % 4]) for i in range(n)]
    seen = []

    def spy(ids):
        seen.extend(ids)
        return score(ids)
    R, scored, _ = osr.beam_search(spy, nbrs, ctop, [1, 3], [1], ef=8, w=3)
    assert all(i % 4 in (1, 3) for i in seen)
    assert len(seen) == len(set(seen)) == scored
    assert all(i % 4 in (1, 3) for _, i in R)
    # R is the top of what was scored
    s = np.array(score(seen))
    top = sorted(zip(-s, seen))[:8]
    assert [i for _, i in top] == [i for _, i in R]
