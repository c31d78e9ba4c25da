"""Pins for the oracle's cluster-guided search (Alg. 5, batched reading).

Sources of truth: reductions to brute force (a complete graph, or ef and w
large enough to exhaust a connected graph, give the exhaustive top-ef of every
reachable set), closed forms of the TF-IDF clustering for special shapes,
NumPy's stable argsort for the top-t of S = C Q^T, invariants (a pruned
cluster is never scored, no set is scored twice), hand traces of Alg. 5 on a
small graph with ef < N (the order in which sets are expanded, the sets
scored, the step count and R), and an independent priority-queue restatement
of Alg. 5 as printed, which the batched reading must follow step for step with
one entry point and one path.
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


# --------------------------------------------------------------------------
# Hand-traced runs of Alg. 5 on a 12-set graph with ef < N. Scores are given
# directly (similarities, larger is closer), so every step can be followed on
# paper. Set 11 sits in a cluster outside C_query (the pruning test of Alg. 5).
_HT_SCORE = {0: 1.0, 1: 2.0, 2: 5.0, 3: 3.0, 4: 8.0, 5: 4.0, 6: 9.0, 7: 0.5, 8: 7.0, 9: 6.0, 10: 10.0, 11: 2.5}
_HT_NBRS = {0: [1, 2, 3], 1: [0, 4], 2: [0, 5, 6], 3: [0, 7], 4: [1, 8], 5: [2, 9], 6: [2, 10, 11],
            7: [3], 8: [4, 9], 9: [5, 8, 10], 10: [6, 9], 11: [6]}
_HT_CTOP = [np.array([1 if i == 11 else 0]) for i in range(12)]


class _RecordingNeighbors:
    """Neighbour lists that record which set is expanded, in order."""

    def __init__(self, nbrs):
        self.nbrs = nbrs
        self.expanded = []

    def __getitem__(self, p):
        self.expanded.append(int(p))
        return np.array(self.nbrs[int(p)], np.int64)


def _ht_run(entries, ef, w):
    scored = []

    def score(ids):
        scored.extend(int(i) for i in ids)
        return [_HT_SCORE[int(i)] for i in ids]
    nb = _RecordingNeighbors(_HT_NBRS)
    R, n_scored, steps = osr.beam_search(score, nb, _HT_CTOP, [0], entries, ef=ef, w=w)
    return R, n_scored, steps, nb.expanded, scored


def test_alg5_single_path_hand_trace():
    # One entry (set 0), ef = 3, one path. By hand, Alg. 5 pops the closest
    # element of W and stops once it is worse than tau (the furthest of R):
    #   pop 0 (tau 1): score 1, 2, 3; R = {2, 3, 1} (0 evicted)
    #   pop 2 (tau 2): score 5, 6; R = {6, 2, 5}
    #   pop 6 (tau 4): score 10 (11 is pruned); R = {10, 6, 2}
    #   pop 10 (tau 5): score 9; R = {10, 6, 9}
    #   pop 9 (tau 6, itself): score 8; R = {10, 6, 8}
    #   pop 8 (tau 7, itself): score 4; R = {10, 6, 4}
    #   pop 4 (tau 8, itself): nothing new
    #   pop 5 (score 4 < tau 8): the path ends. 1, 3 and 5 are never expanded
    #   and 7 (reached only through 3) is never scored.
    R, n_scored, steps, expanded, scored = _ht_run([0], ef=3, w=1)
    assert expanded == [0, 2, 6, 10, 9, 8, 4]
    assert steps == 7
    assert scored == [0, 1, 2, 3, 5, 6, 10, 9, 8, 4]
    assert n_scored == 10
    assert [i for _, i in R] == [10, 6, 4]
    assert [s for s, _ in R] == [10.0, 9.0, 8.0]


def test_alg5_two_paths_hand_trace():
    # Entries 0 and 7, ef = 4, two paths advancing in synchronous steps (the
    # w best unexpanded entries of R expand together; a neighbour reached in
    # the step is marked visited when taken):
    #   step 1: expand 0, 7 -> score 1, 2, 3 (3 is taken from 0 first);
    #            R = {2, 3, 1, 0}
    #   step 2: expand 2, 3 -> score 5, 6; R = {6, 2, 5, 3}
    #   step 3: expand 6, 5 -> score 10, 9 (11 pruned); R = {10, 6, 9, 2}
    #   step 4: expand 10, 9 -> score 8; R = {10, 6, 8, 9}
    #   step 5: expand 8 -> score 4; R = {10, 6, 4, 8}
    #   step 6: expand 4 -> nothing; no unexpanded entry is left in R.
    R, n_scored, steps, expanded, scored = _ht_run([0, 7], ef=4, w=2)
    assert expanded == [0, 7, 2, 3, 6, 5, 10, 9, 8, 4]
    assert steps == 6
    assert scored == [0, 7, 1, 2, 3, 5, 6, 10, 9, 8, 4]
    assert n_scored == 11
    assert [i for _, i in R] == [10, 6, 4, 8]


def _alg5_as_printed(score_of, nbrs, ctop, cq, ep, ef):
    """Alg. 5 literally, for one entry point: a priority queue W popped
    closest-first, tau = the furthest element of R, the path ends at the first
    popped element worse than tau, each insertion into R evicts the furthest
    once R holds more than ef (ties: the larger id is the further)."""
    import heapq
    cqs = set(cq)
    V = {ep}
    R = {ep: score_of(ep)}
    W = [(-R[ep], ep)]
    order = []
    while W:
        negs, p = heapq.heappop(W)
        tau = min(R.items(), key=lambda kv: (kv[1], -kv[0]))
        if (-negs, -p) < (tau[1], -tau[0]):
            break
        order.append(p)
        for nb in nbrs[p]:
            if nb in V or not (set(int(j) for j in ctop[nb]) & cqs):
                continue
            s = score_of(nb)
            V.add(nb)
            heapq.heappush(W, (-s, nb))
            R[nb] = s
            if len(R) > ef:
                worst = min(R.items(), key=lambda kv: (kv[1], -kv[0]))
                del R[worst[0]]
    ranked = sorted(R.items(), key=lambda kv: (-kv[1], kv[0]))
    return order, [i for i, _ in ranked], len(V)


def test_alg5_single_path_equals_the_printed_algorithm_on_random_graphs():
    # With one entry point and w = 1 the batched reading must take exactly the
    # steps of Alg. 5 as printed (an independent priority-queue restatement).
    for seed in range(40):
        rng = np.random.default_rng(100 + seed)
        n = int(rng.integers(8, 40))
        sc = rng.permutation(n).astype(np.float64) + rng.random()       # distinct scores
        deg = int(rng.integers(1, 5))
        nbrs = [list(rng.integers(0, n, deg)) for _ in range(n)]
        ctop = [np.array([int(rng.integers(0, 3))]) for _ in range(n)]
        cq = [0, 1]
        ep = int(rng.integers(0, n))
        ef = int(rng.integers(1, 8))
        order, ids, n_seen = _alg5_as_printed(lambda i: sc[i], nbrs, ctop, cq, ep, ef)
        nb = _RecordingNeighbors({i: nbrs[i] for i in range(n)})
        R, n_scored, steps = osr.beam_search(lambda ids_: [sc[i] for i in ids_], nb, ctop, cq, [ep], ef=ef, w=1)
        assert nb.expanded == order, seed
        assert [i for _, i in R] == ids, seed
        assert n_scored == n_seen and steps == len(order), seed
