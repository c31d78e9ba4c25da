"""GPU parity of the document-major gathered scorer (GEM_OPT_GATHER_ORDER).

Scoring candidate lists by document (entries grouped by document, each
document staged once and scored against every query that lists it) performs
the same products, the same running max over the document's tiles and the
same column sums in tile order as the per-query gathered scorer, so every
entry's score must match that scorer's bitwise; the per-query scorer is in
turn checked against the oracle, and the float32 case is checked against the
oracle here as well (3e-4 relative: queries of up to 200 vectors, see the
tolerance note of the dense parity tests).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_20336_amd as gem
from paper_2603_20336_amd import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda"
DTYPES = ["f32", "bf16x3", "bf16", "fp8", "mxfp4", "mxfp6"]


@pytest.fixture(autouse=True)
def _restore_order():
    yield
    gem.set_gather_order("auto")


def _csr(lengths):
    o = np.zeros(len(lengths) + 1, np.int64)
    o[1:] = np.cumsum(lengths)
    return o


def _ragged(lengths, seed):
    centers = wl.mixture_centers(8, seed)
    g = torch.Generator().manual_seed(seed + 1)
    vecs = wl.mixture_vectors(int(sum(lengths)), centers, 0.1, g)
    return wl.SetBatch(vecs, torch.from_numpy(_csr(lengths)))


def _docs(batch, dtype):
    S = gem.Sets.from_batch(batch, DEV)
    return {"f32": S, "bf16x3": S.to_bf16x3() if dtype == "bf16x3" else None,
            "bf16": S.to_bf16() if dtype == "bf16" else None,
            "fp8": S.to_fp8() if dtype == "fp8" else None,
            "mxfp4": S.to_mxfp4() if dtype == "mxfp4" else None,
            "mxfp6": S.to_mxfp6() if dtype == "mxfp6" else None}[dtype]


def _run(Q, D, dtype, C, order, **kw):
    gem.set_gather_order(order)
    if dtype in ("fp8", "mxfp4", "mxfp6"):
        q = {"fp8": gem.quantize_fp8, "mxfp4": gem.quantize_mxfp4, "mxfp6": gem.quantize_mxfp6}[dtype](Q)
        out = gem.score_quant(q, D, cands=C, **kw)
    else:
        out = gem.score_exact(Q, D, cands=C, compute=dtype, **kw)
    torch.cuda.synchronize()
    return out


def _bits(t):
    return t.detach().cpu().contiguous().view(torch.int32).numpy()


def _lists(rng, n_q, n_docs):
    """Ragged lists with heavy sharing: one popular document in every list
    (more than one work item of 64 listings), repeats inside a list, padding
    ids, an empty list and lists longer than a wave's entries."""
    lists = []
    for i in range(n_q):
        n = int(rng.integers(0, 150))
        ids = rng.integers(0, n_docs, n)
        ids = np.concatenate([ids, [7, 7, 0, n_docs - 1]])
        ids[rng.random(ids.size) < 0.05] = -1
        lists.append(ids)
    lists[3] = np.array([], np.int64)
    return lists


@pytest.mark.parametrize("dtype", DTYPES)
def test_by_document_is_the_per_query_scorer_bitwise(dtype):
    # documents of 0..256 rows (one exactly 256: the most this path stages),
    # queries of 0..200 vectors (up to four passes of 64 columns)
    rng = np.random.default_rng(70)
    d_len = rng.integers(1, 257, 300)
    d_len[11] = 0
    d_len[7] = 256
    q_len = rng.integers(1, 201, 40)
    q_len[2] = 0
    q_len[5], q_len[6], q_len[8] = 64, 65, 1
    c, q = _ragged(d_len, 71), _ragged(q_len, 72)
    Q, D = gem.Sets.from_batch(q, DEV), _docs(c, dtype)
    lists = _lists(rng, 40, 300)
    co = _csr([len(x) for x in lists])
    ci = np.concatenate(lists).astype(np.int32)
    C = gem.Cands(torch.from_numpy(ci).to(DEV), torch.from_numpy(co).to(DEV))
    by_q = _run(Q, D, dtype, C, "query")
    by_d = _run(Q, D, dtype, C, "document")
    np.testing.assert_array_equal(_bits(by_d), _bits(by_q))
    assert np.all(np.isneginf(by_d.cpu().numpy()[ci < 0]))
    # the top-k over the lists, both orders
    tq = _run(Q, D, dtype, C, "query", k=10)
    td = _run(Q, D, dtype, C, "document", k=10)
    np.testing.assert_array_equal(_bits(td[0]), _bits(tq[0]))
    np.testing.assert_array_equal(td[1].cpu().numpy(), tq[1].cpu().numpy())
    if dtype == "f32":
        got = by_d.cpu().numpy()
        ref = oracle.ch_cands(q.vecs.numpy(), q.offsets.numpy(), c.vecs.numpy(), c.offsets.numpy(), co,
                              np.maximum(ci, 0))
        ref[ci < 0] = -np.inf
        inf = np.isinf(ref)
        assert np.array_equal(np.isinf(got), inf) and np.array_equal(got[inf], ref[inf])
        rel = np.abs(got[~inf] - ref[~inf]) / np.maximum(np.abs(ref[~inf]), 1.0)
        assert rel.max() <= 3e-4, rel.max()


@pytest.mark.parametrize("dtype", ["f32", "fp8"])
def test_strided_lists_and_auto_order(dtype):
    # fixed-length rows with padding at the tail; 4000 entries over 500
    # documents, so "auto" takes the document order too
    rng = np.random.default_rng(80)
    d_len = rng.integers(16, 120, 500)
    q_len = rng.integers(4, 65, 20)
    c, q = _ragged(d_len, 81), _ragged(q_len, 82)
    Q, D = gem.Sets.from_batch(q, DEV), _docs(c, dtype)
    ids = rng.integers(0, 500, (20, 200)).astype(np.int32)
    ids[:, 190:] = -1
    C = gem.Cands(torch.from_numpy(ids.reshape(-1)).to(DEV), stride=200, n_lists=20)
    by_q = _run(Q, D, dtype, C, "query")
    for order in ("document", "auto"):
        np.testing.assert_array_equal(_bits(_run(Q, D, dtype, C, order)), _bits(by_q))


def test_document_order_bounds():
    rng = np.random.default_rng(90)
    d_len = rng.integers(16, 100, 50)
    d_len[4] = 300                                        # longer than the 256 rows a stage holds
    c, q = _ragged(d_len, 91), _ragged([12, 40, 70], 92)
    S = gem.Sets.from_batch(c, DEV)
    ids = rng.integers(0, 50, 3 * 64).astype(np.int32)
    ids[:5] = 4
    C = gem.Cands(torch.from_numpy(ids).to(DEV), stride=64, n_lists=3)
    Q = gem.Sets.from_batch(q, DEV)
    by_q = _run(Q, S, "f32", C, "query")
    # the true bound (300 rows) is past what the document order takes: the
    # call keeps the query order
    np.testing.assert_array_equal(_bits(_run(Q, S, "f32", C, "document")), _bits(by_q))
    # a bound that understates the longest document: its entries get NaN,
    # every other entry its score
    under = gem.Sets(S.vecs, S.offsets, "f32", 256)
    got = _run(Q, under, "f32", C, "document").cpu().numpy()
    long_doc = ids == 4
    assert np.all(np.isnan(got[long_doc]))
    np.testing.assert_array_equal(got[~long_doc].view(np.int32), by_q.cpu().numpy()[~long_doc].view(np.int32))
    assert gem.get_gather_order() == "document"
    with pytest.raises(gem.GemError):
        gem._abi.check(gem.library().gem_set_option(gem._ctx(torch.device(DEV)), gem._abi.GEM_OPT_GATHER_ORDER, 7))


def test_rerank_shape_by_document_matches_oracle_sample():
    """A rerank in the shape of an FP8 shortlist: 400 queries x 500 ids over
    8000 documents drawn from a skewed popularity (about 25 listings per
    document), by document and in the mixed order against by query bitwise,
    and 6 lists against the oracle."""
    w = wl.WORKLOADS[2]
    rng = np.random.default_rng(100)
    n_docs, n_q, sl = 8000, 400, 500
    c = wl.corpus(w, n_docs=n_docs)
    q = wl.queries(w, n_queries=n_q)
    Q, D = gem.Sets.from_batch(q, DEV), gem.Sets.from_batch(c, DEV)
    pop = rng.zipf(1.3, (n_q, 4 * sl)) % n_docs
    ids = np.stack([np.unique(r)[:sl] if np.unique(r).size >= sl else
                    np.concatenate([np.unique(r), rng.integers(0, n_docs, sl - np.unique(r).size)]) for r in pop])
    ids = ids.astype(np.int32)
    C = gem.Cands(torch.from_numpy(ids.reshape(-1)).to(DEV), stride=sl, n_lists=n_q)
    by_q = _run(Q, D, "f32", C, "query")
    by_d = _run(Q, D, "f32", C, "document")
    np.testing.assert_array_equal(_bits(by_d), _bits(by_q))
    # the mixed order: popular documents by document, the rest by query
    cnt = np.bincount(ids.reshape(-1), minlength=n_docs)
    assert (cnt >= 8).any() and ((cnt > 0) & (cnt < 8)).any()
    np.testing.assert_array_equal(_bits(_run(Q, D, "f32", C, "auto")), _bits(by_q))
    got = by_d.cpu().numpy().reshape(n_q, sl)
    qv, qo, dv, do = q.vecs.numpy(), q.offsets.numpy(), c.vecs.numpy(), c.offsets.numpy()
    for r in rng.choice(n_q, 6, replace=False):
        ref = oracle.ch_cands(qv[qo[r]:qo[r + 1]], [0, qo[r + 1] - qo[r]], dv, do, [0, sl], ids[r])
        rel = np.abs(got[r] - ref) / np.maximum(np.abs(ref), 1.0)
        assert rel.max() <= 1e-4, (r, rel.max())
