"""GPU parity of the cluster-guided search (Alg. 5) against the oracle.

The search takes data-dependent decisions at every step, so the main test
runs it on vectors of small integers: their FP8 codes are exact and every
Chamfer score is an exact float32 value, so the GPU and the float64 oracle see
identical scores and must take identical paths (ties by set id on both
sides). Cluster masks, members and entry draws given to the GPU come from the
oracle; the clustering kernels are checked against the oracle on their own.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_20336_amd as gem
from paper_2603_20336_amd import search as gs
from paper_2603_20336_amd import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _np(t):
    return t.detach().cpu().numpy()


def _csr(lengths):
    o = np.zeros(len(lengths) + 1, np.int64)
    o[1:] = np.cumsum(lengths)
    return o


def _masks(cluster_lists, k2):
    words = (k2 + 31) // 32
    m = np.zeros((len(cluster_lists), words), np.uint32)
    for i, cs in enumerate(cluster_lists):
        for j in cs:
            m[i, int(j) >> 5] |= np.uint32(1 << (int(j) & 31))
    return m


def _decode_masks(m, k2):
    m = np.asarray(m).view(np.uint32)
    return [np.array([j for j in range(k2) if (m[i, j >> 5] >> (j & 31)) & 1], np.int64) for i in range(m.shape[0])]


def test_set_clusters_match_oracle():
    rng = np.random.default_rng(0)
    k2, r, n = 40, 3, 700
    lens = rng.integers(0, 30, n)
    vc = (rng.zipf(1.6, int(lens.sum())) % k2).astype(np.int32)      # skewed cluster use: varied DF
    off = _csr(lens)
    masks, moff, members = gs.set_clusters(torch.from_numpy(vc).to(DEV), torch.from_numpy(off).to(DEV), k2, r)
    got = _decode_masks(_np(masks), k2)
    want, idf = oracle.tfidf_top_clusters(vc, off, k2, r)
    tf = [np.bincount(vc[off[i]:off[i + 1]], minlength=k2) for i in range(n)]
    for i in range(n):
        if np.array_equal(got[i], want[i]):
            continue
        # only a near-tie of TF * IDF (float32 on the GPU) may change the choice
        sc = tf[i] * idf
        assert len(got[i]) == len(want[i])
        assert abs(np.sort(sc[got[i]]).sum() - np.sort(sc[want[i]]).sum()) <= 1e-5 * max(1.0, abs(sc).max())
    # members: the sets of each cluster in id order, consistent with the masks
    mo, mem = _np(moff), _np(members)
    for j in range(k2):
        exp = [i for i in range(n) if j in set(got[i].tolist())]
        np.testing.assert_array_equal(mem[mo[j]:mo[j + 1]], exp)


def test_query_clusters_match_oracle_on_exact_integers():
    rng = np.random.default_rng(1)
    k2 = 70
    C = rng.integers(-2, 3, (k2, 128)).astype(np.float32)
    C[5] = C[60]                                                     # equal scores: the smaller index wins
    ql = rng.integers(0, 9, 25)
    qv = rng.integers(-2, 3, (int(ql.sum()), 128)).astype(np.float32)
    Q = gem.Sets(torch.from_numpy(qv).to(DEV), torch.from_numpy(_csr(ql)).to(DEV), "f32", int(ql.max()))
    for t in (1, 4):
        got = _decode_masks(_np(gs.query_clusters(Q, torch.from_numpy(C).to(DEV), t)), k2)
        off = _csr(ql)
        for i in range(25):
            want = oracle.query_clusters(qv[off[i]:off[i + 1]], C, t) if ql[i] else np.zeros(0, np.int64)
            np.testing.assert_array_equal(got[i], want)


def _int_sets(rng, lengths, lo=-3, hi=3):
    return rng.integers(lo, hi + 1, (int(np.sum(lengths)), 128)).astype(np.float32)


@pytest.mark.parametrize("ef,width", [(16, 1), (40, 4), (64, 8)])
def test_search_matches_oracle_exactly(ef, width):
    rng = np.random.default_rng(ef + width)
    n, deg, k2, n_q = 600, 12, 16, 20
    dl = rng.integers(1, 12, n)
    dv = _int_sets(rng, dl)
    do = _csr(dl)
    ql = rng.integers(1, 9, n_q)
    qv = _int_sets(rng, ql)
    qo = _csr(ql)
    # graph: random neighbours (some padding), clusters: r = 2 of k2 per set
    nbrs = rng.integers(0, n, (n, deg)).astype(np.int32)
    nbrs[rng.random((n, deg)) < 0.1] = -1
    ctop = [np.sort(rng.choice(k2, 2, replace=False)) for _ in range(n)]
    members = oracle.cluster_members(ctop, k2)
    moff = _csr([len(m) for m in members])
    cq = [np.sort(rng.choice(k2, rng.integers(1, 6), replace=False)) for _ in range(n_q)]
    u = rng.integers(0, 2 ** 32, (n_q, k2), dtype=np.uint64)
    # device side: FP8 sets (exact for these integers)
    D8 = gem.Sets(torch.from_numpy(dv).to(DEV), torch.from_numpy(do).to(DEV), "f32", int(dl.max())).to_fp8()
    Q8 = gem.Sets(torch.from_numpy(qv).to(DEV), torch.from_numpy(qo).to(DEV), "f32", int(ql.max())).to_fp8()
    index = gs.ClusterIndex(torch.from_numpy(nbrs).to(DEV), torch.from_numpy(_masks(ctop, k2).view(np.int32)).to(DEV),
                            torch.from_numpy(moff).to(DEV),
                            torch.from_numpy(np.concatenate(members).astype(np.int32)).to(DEV),
                            torch.zeros(k2, 128, device=DEV))
    qmask = torch.from_numpy(_masks(cq, k2).view(np.int32)).to(DEV)
    srch = gs.GraphSearch(Q8, D8, index, qmask, ef=ef, width=width)
    words = torch.from_numpy(u.astype(np.uint32).view(np.int32)).to(DEV)
    steps = srch.run(words, check_every=1, graph=False)
    bs, bi = _np(srch.beam.scores), _np(srch.beam.ids)
    # the same search from a captured graph of 3 steps, replayed, twice over
    # (with eager work and synchronizations between the runs)
    for _ in range(2):
        srch.run(words, check_every=3, graph=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(_np(srch.beam.ids), bi)
        np.testing.assert_array_equal(_np(srch.beam.scores), bs)
        gem.score_quant(Q8, D8, k=2)
    # on a side stream: begin, the replays and the active-count reads all
    # follow that stream, with no synchronization from the caller in between
    side = torch.cuda.Stream(device=DEV)
    side.wait_stream(torch.cuda.current_stream(DEV))
    srch.run(words, check_every=3, graph=True, stream=side)
    torch.cuda.current_stream(DEV).wait_stream(side)
    np.testing.assert_array_equal(_np(srch.beam.ids), bi)
    np.testing.assert_array_equal(_np(srch.beam.scores), bs)
    # the oracle on the same (exact) operand values
    dvals = oracle.dequantize_fp8(*oracle.quantize_fp8(dv))
    qvals = oracle.dequantize_fp8(*oracle.quantize_fp8(qv))
    assert np.array_equal(dvals, dv) and np.array_equal(qvals, qv)
    max_steps = 0
    for i in range(n_q):
        score = oracle.ch_scorer(qvals[qo[i]:qo[i + 1]], dvals, do)
        E = oracle.entry_points(cq[i], members, u[i])
        R, _, st = oracle.beam_search(score, nbrs, ctop, cq[i], E, ef=ef, w=width)
        max_steps = max(max_steps, st)
        ids = [d for _, d in R]
        np.testing.assert_array_equal(bi[i][:len(ids)], ids)
        assert (bi[i][len(ids):] == -1).all()
        np.testing.assert_array_equal(bs[i][:len(ids)], np.array([s for s, _ in R], np.float32))
    assert steps >= max_steps >= 1


def test_search_on_a_knn_graph_reaches_the_exhaustive_neighbours():
    # a small corpus, its kNN graph by the FP8 estimate, clusters from k-means:
    # with a generous ef the search finds nearly all of the exhaustive top-10
    w = wl.WORKLOADS[1]
    c, q = wl.corpus(w, n_docs=1500), wl.queries(w, n_queries=16)
    D32, Q32 = gem.Sets.from_batch(c, DEV), gem.Sets.from_batch(q, DEV)
    D8, Q8 = D32.to_fp8(), Q32.to_fp8()
    nbrs = gs.knn_graph(D32, D8, degree=16, batch=500)
    init = torch.from_numpy(np.random.default_rng(2).choice(D32.n_vecs, 32, replace=False).astype(np.int64))
    Cidx = gem.kmeans(D32.vecs, init, n_iter=4)
    vc = gem.nearest_centroid(D32.vecs, Cidx)
    masks, moff, members = gs.set_clusters(vc, D32.offsets, 32, 2)
    index = gs.ClusterIndex(nbrs, masks, moff, members, Cidx)
    qmask = gs.query_clusters(Q32, Cidx, 4)
    srch = gs.GraphSearch(Q8, D8, index, qmask, ef=64, width=4)
    u = torch.from_numpy(np.random.default_rng(3).integers(0, 2 ** 32, (16, 32), dtype=np.uint64)
                         .astype(np.uint32).view(np.int32)).to(DEV)
    srch.run(u)
    _, top = srch.rerank(Q32, D32, 10)
    _, exact = gem.score_exact(Q32, D32, k=10, compute="f32")
    t, e = _np(top), _np(exact)
    recall = np.mean([len(set(t[i]) & set(e[i])) / 10 for i in range(16)])
    assert recall >= 0.8, recall
