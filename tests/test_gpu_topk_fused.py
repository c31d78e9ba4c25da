"""The per-query top-k fused into the exhaustive scorer (no score matrix):
bitwise the top-k that gem_topk takes from the staged score rows, for every
format, for k from 1 to 1024, for corpora whose order makes every document
beat the running threshold (the regions' selections run many times), for
heavy ties, empty sets and fewer documents than k."""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_20336_amd as gem
from paper_2603_20336_amd import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _csr(lengths):
    o = np.zeros(len(lengths) + 1, np.int64)
    o[1:] = np.cumsum(lengths)
    return o


def _ragged(lengths, seed):
    centers = wl.mixture_centers(8, seed)
    g = torch.Generator().manual_seed(seed + 1)
    vecs = wl.mixture_vectors(int(sum(lengths)), centers, 0.1, g)
    return wl.SetBatch(vecs, torch.from_numpy(_csr(lengths)))


def _dev(batch, dtype):
    S = gem.Sets.from_batch(batch, DEV)
    return {"f32": S, "bf16": S.to_bf16(), "fp8": S.to_fp8(), "mxfp4": S.to_mxfp4()}[dtype]


def _topk(Q, D, dtype, k, mode):
    gem.set_topk_fusion(mode)
    try:
        if dtype in ("fp8", "mxfp4"):
            out = gem.score_quant(Q, D, k=k)
        else:
            out = gem.score_exact(Q, D, compute=dtype, k=k)
    finally:
        gem.set_topk_fusion("auto")
    torch.cuda.synchronize()
    return out[0].cpu().numpy(), out[1].cpu().numpy()


def _same(Q, D, dtype, k):
    """Fused and staged top-k of the same call agree bitwise; returns them."""
    fs, fi = _topk(Q, D, dtype, k, "fused")
    ss, si = _topk(Q, D, dtype, k, "staged")
    np.testing.assert_array_equal(fi, si, err_msg=f"{dtype} k={k} ids")
    np.testing.assert_array_equal(fs.view(np.uint32), ss.view(np.uint32), err_msg=f"{dtype} k={k} scores")
    return fs, fi


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8", "mxfp4"])
def test_fused_equals_staged_ragged(dtype):
    rng = np.random.default_rng(31)
    ql = [int(x) for x in rng.integers(1, 65, 70)]
    ql[5] = 0                                                  # an empty query: every score is 0
    dl = [int(x) for x in rng.integers(0, 40, 9000)]          # empty documents score -inf
    Q = gem.Sets.from_batch(_ragged(ql, 80), DEV)
    D = _dev(_ragged(dl, 81), dtype)
    for k in (1, 10, 100, 1000, 1024):
        _same(Q, D, dtype, k)


def test_fused_matches_oracle_f32():
    rng = np.random.default_rng(32)
    q = _ragged([int(x) for x in rng.integers(1, 40, 12)], 82)
    c = _ragged([int(x) for x in rng.integers(1, 30, 5000)], 83)
    Q, D = gem.Sets.from_batch(q, DEV), gem.Sets.from_batch(c, DEV)
    ts, ti = _same(Q, D, "f32", 50)
    ref = oracle.ch_dense(q.vecs.numpy(), q.offsets.numpy(), c.vecs.numpy(), c.offsets.numpy())
    for r in range(q.n_sets):
        tau = 2e-4 * max(abs(np.sort(ref[r])[::-1][49]), 1.0)
        ok, bad, missing = oracle.tie_aware_match(ti[r], ref[r], 50, tau)
        assert ok, (r, bad, missing)


def _monotone_corpus(n_docs, increasing, seed):
    """One vector per document, <u, v_i> strictly monotone in i (every later
    document beats every earlier one when increasing)."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(128)
    u /= np.linalg.norm(u)
    w = rng.standard_normal(128)
    w -= (w @ u) * u
    w /= np.linalg.norm(w)
    th = np.linspace(1.2, 0.05, n_docs)
    if not increasing:
        th = th[::-1]
    v = np.cos(th)[:, None] * u[None] + np.sin(th)[:, None] * w[None]
    c = wl.SetBatch(torch.from_numpy(v.astype(np.float32)), torch.from_numpy(_csr([1] * n_docs)))
    return c, u


@pytest.mark.parametrize("dtype,increasing", [("bf16", True), ("bf16", False), ("fp8", True), ("f32", True)])
def test_fused_every_document_beats_the_threshold(dtype, increasing):
    """Enough queries for one piece per XCD, and documents in increasing score
    order: each region fills and selects its k best many times, and the shared
    bounds from later pieces filter earlier ones."""
    n_docs = 40000
    c, u = _monotone_corpus(n_docs, increasing, 33)
    n_q = 1024 if dtype != "f32" else 256
    qv = np.repeat(u[None].astype(np.float32), 32 * n_q, axis=0)
    q = wl.SetBatch(torch.from_numpy(qv), torch.from_numpy(_csr([32] * n_q)))
    Q, D = gem.Sets.from_batch(q, DEV), _dev(c, dtype)
    for k in (100, 1000):
        ts, ti = _same(Q, D, dtype, k)
        if dtype == "f32":
            want = np.arange(n_docs - 1, n_docs - 1 - k, -1) if increasing else np.arange(k)
            np.testing.assert_array_equal(ti[0], want)
            assert (ti == ti[0]).all()


def test_fused_heavy_ties():
    """30,000 documents that are copies of 37: equal scores order by id."""
    base = _ragged([int(x) for x in np.random.default_rng(34).integers(1, 20, 37)], 84)
    idx = [i % 37 for i in range(30000)]
    c = base.subset(idx)
    c = wl.SetBatch(c.vecs, c.offsets)
    q = _ragged([int(x) for x in np.random.default_rng(35).integers(1, 50, 300)], 85)
    Q = gem.Sets.from_batch(q, DEV)
    for dtype in ("bf16", "fp8"):
        D = _dev(c, dtype)
        for k in (7, 100, 1000):
            ts, ti = _same(Q, D, dtype, k)
            # copies of the best base document come first, in id order (37 apart)
            assert (np.diff(ti[:, :min(k, 20)].astype(np.int64), axis=1) == 37).all()


def test_fused_fewer_documents_than_k():
    q = _ragged([10, 0, 33, 64, 5], 86)
    c = _ragged([3, 0, 7, 12, 1, 0, 9], 87)
    Q, D = gem.Sets.from_batch(q, DEV), gem.Sets.from_batch(c, DEV)
    ts, ti = _same(Q, D, "f32", 20)
    assert (ti[:, 7:] == -1).all() and np.isneginf(ts[:, 7:]).all()
    assert (np.sort(ti[:, :7], axis=1) == np.arange(7)).all()


def test_fused_schedules_give_the_same_top_k():
    rng = np.random.default_rng(36)
    q = _ragged([int(x) for x in rng.integers(1, 65, 150)], 88)
    c = _ragged([int(x) for x in rng.integers(0, 60, 20000)], 89)
    Q, D = gem.Sets.from_batch(q, DEV), _dev(c, "bf16")
    base = _topk(Q, D, "bf16", 100, "staged")
    spx = gem.dense_schedule("bf16", Q.n_vecs, D.n_sets)["slots_per_xcd"]
    try:
        for cd in (32, 64):
            for ips in (1, 8):
                for slots in (spx, max(1, spx // 4)):
                    gem.set_dense_schedule("bf16", Q.n_vecs, D.n_sets,
                                           {"chunk_docs": cd, "items_per_slot": ips, "slots_per_xcd": slots})
                    got = _topk(Q, D, "bf16", 100, "fused")
                    np.testing.assert_array_equal(got[1], base[1])
                    np.testing.assert_array_equal(got[0], base[0])
    finally:
        gem.set_dense_schedule("bf16", Q.n_vecs, D.n_sets, None)


def test_auto_mode_workspace_is_small_for_large_batches():
    """The exhaustive-100k shape: the fused top-k's workspace is a small
    fraction of the 400 MB score matrix that staging would need."""
    w2 = wl.WORKLOADS[2]
    q = wl.queries(w2, device=DEV)
    Q = gem.Sets(q.vecs, q.offsets, "f32", q.max_len())
    n_docs, n_vecs = 100000, 8014384
    D = gem.Sets(torch.empty(1, 128, dtype=torch.uint16, device=DEV), torch.zeros(n_docs + 1, dtype=torch.int64,
                 device=DEV), "bf16", 256, n_sets=n_docs)
    staged = 1000 * n_docs * 4
    auto = gem.score_workspace_bytes(Q, D, k=100, compute="bf16")
    assert auto < staged / 4, (auto, staged)
    gem.set_topk_fusion("staged")
    try:
        assert gem.score_workspace_bytes(Q, D, k=100, compute="bf16") >= staged
    finally:
        gem.set_topk_fusion("auto")
