"""GPU parity of the codebook path: nearest centroid, k-means update, and the
quantized Chamfer estimate qCH over code sets, against the float64 oracle.

Codes fed to the scorers come from the oracle's own nearest-centroid map, so
no oracle input comes from the GPU. Nearest-centroid decisions are compared
exactly wherever the oracle's margin between the best and the second-best
centroid exceeds the float32 evaluation error; inside that band the GPU's
choice must be a centroid within the band of the best distance.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_20336_amd as gem
from paper_2603_20336_amd import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL = 1e-4
NN_BAND = 2e-5       # float32 evaluation of <x, c> - |c|^2 / 2 for unit-scale rows: error well below this


def _np(t):
    return t.detach().cpu().numpy()


def _csr(lengths):
    o = np.zeros(len(lengths) + 1, np.int64)
    o[1:] = np.cumsum(lengths)
    return o


def _clustered(n, n_centers, seed, spread=0.25):
    centers = wl.mixture_centers(n_centers, seed)
    g = torch.Generator().manual_seed(seed + 1)
    return wl.mixture_vectors(n, centers, spread, g).numpy()


def _bf16_values(x):
    return oracle.bf16_decode(oracle.bf16_round_bits(np.asarray(x, np.float32)))


def _check_nn(got, x64, c64, what):
    d = oracle.sq_distances(x64, c64)
    best = np.argmin(d, axis=1)
    srt = np.sort(d, axis=1)
    margin = srt[:, 1] - srt[:, 0]
    clear = margin > NN_BAND
    np.testing.assert_array_equal(got[clear], best[clear], err_msg=f"{what}: clear decisions differ")
    rows = np.arange(len(got))
    assert (d[rows, got] - srt[:, 0] <= NN_BAND).all(), f"{what}: a chosen centroid is not nearest"
    return clear.mean()


@pytest.mark.parametrize("assign", ["f32", "bf16"])
def test_nearest_centroid_matches_oracle(assign):
    x = _clustered(5003, 40, 11)                                  # ragged tail of row blocks
    C = _clustered(1003, 40, 12, spread=0.4)                      # ragged last centroid tile
    C[500] = C[7]                                                 # duplicate centroid: the smaller index wins
    x[:3] = C[7]
    xt, Ct = torch.from_numpy(x).to(DEV), torch.from_numpy(C).to(DEV)
    if assign == "bf16":
        xt, Ct = gem._bf16_rows(xt), gem._bf16_rows(Ct)
        x64, c64 = _bf16_values(x), _bf16_values(C)
    else:
        x64, c64 = x.astype(np.float64), C.astype(np.float64)
    got = _np(gem.nearest_centroid(xt, Ct)).astype(np.int64)
    frac = _check_nn(got, x64, c64, assign)
    assert frac > 0.95
    assert (got[:3] == 7).all()
    # the same rows in a launch with another slice split give the same codes
    part = _np(gem.nearest_centroid(xt[:77].contiguous(), Ct)).astype(np.int64)
    np.testing.assert_array_equal(part, got[:77])
    # one centroid: every row takes it
    one = _np(gem.nearest_centroid(xt[:50].contiguous(), Ct[:1].contiguous()))
    assert (one == 0).all()


def test_centroid_update_matches_oracle_and_is_deterministic():
    rng = np.random.default_rng(3)
    x = _clustered(20000, 30, 13)
    k = 301
    codes = rng.integers(0, k, x.shape[0]).astype(np.int32)
    codes[codes == 17] = 18                                       # centroid 17 has no rows
    C0 = _clustered(k, 30, 14)
    xt, ct, C0t = torch.from_numpy(x).to(DEV), torch.from_numpy(codes).to(DEV), torch.from_numpy(C0).to(DEV)
    new, counts = gem.centroid_update(xt, ct, C0t)
    new2, _ = gem.centroid_update(xt, ct, C0t)
    ref = oracle.lloyd_update(x, codes, C0)
    np.testing.assert_array_equal(_np(counts), np.bincount(codes, minlength=k))
    np.testing.assert_array_equal(_np(new)[17], C0[17])
    np.testing.assert_allclose(_np(new), ref, rtol=0, atol=2e-7)
    np.testing.assert_array_equal(_np(new), _np(new2))           # exact integer sums: no order effects
    # in place (new centroids over the old ones)
    C1 = C0t.clone()
    gem.centroid_update(xt, ct, C1, out=C1)
    np.testing.assert_array_equal(_np(C1), _np(new))


def test_kmeans_matches_oracle():
    # well-separated clusters, seeded with one row of each: no assignment is near a tie
    rng = np.random.default_rng(4)
    centers = rng.standard_normal((24, 128))
    centers /= np.linalg.norm(centers, axis=1, keepdims=True)
    lab = rng.integers(0, 24, 3000)
    lab[:24] = np.arange(24)
    x = centers[lab] + 0.05 * rng.standard_normal((3000, 128)) / np.sqrt(128)
    x = (x / np.linalg.norm(x, axis=1, keepdims=True)).astype(np.float32)
    init = np.arange(24)
    C = gem.kmeans(torch.from_numpy(x).to(DEV), torch.from_numpy(init), n_iter=4, assign="f32")
    ref, codes = oracle.kmeans(x, x[init], n_iter=4)
    np.testing.assert_array_equal(codes, lab)
    np.testing.assert_allclose(_np(C), ref, rtol=0, atol=1e-6)
    Cb = gem.kmeans(torch.from_numpy(x).to(DEV), torch.from_numpy(init), n_iter=4, assign="bf16")
    np.testing.assert_allclose(_np(Cb), ref, rtol=0, atol=1e-6)


def _qch_case(seed=5):
    rng = np.random.default_rng(seed)
    C = _clustered(300, 24, seed + 20, spread=0.4)
    d_len = rng.integers(1, 90, 500)
    d_len[[3, 250]] = 0                                           # empty documents
    q_len = rng.integers(1, 65, 40)
    q_len[7] = 0                                                  # an empty query
    xd = _clustered(int(d_len.sum()), 24, seed + 21)
    xq = _clustered(int(q_len.sum()), 24, seed + 22)
    dc, qc = oracle.nn_assign(xd, C), oracle.nn_assign(xq, C)     # the oracle's codes
    return C, _csr(q_len), qc, _csr(d_len), dc, int(q_len.max())


def _code_sets(C, off, codes, max_len, dtype):
    base = gem.Sets(torch.from_numpy(C).to(DEV), torch.from_numpy(off).to(DEV), "f32", max_len,
                    codes=torch.from_numpy(codes.astype(np.int32)).to(DEV))
    return {"f32": base, "bf16": base.to_bf16(), "fp8": base.to_fp8()}[dtype]


def _codebook_values(C, dtype):
    if dtype == "f32":
        return C.astype(np.float64)
    if dtype == "bf16":
        return _bf16_values(C)
    codes, scales = oracle.quantize_fp8(C)
    return oracle.dequantize_fp8(codes, scales)


def _rows_of(vecs, codes):
    """vecs[codes] written out (bit patterns gathered through a signed view)."""
    signed = {torch.uint16: torch.int16, torch.uint8: torch.int8}.get(vecs.dtype, vecs.dtype)
    return vecs.view(signed)[codes.long()].contiguous().view(vecs.dtype)


def _score(Q, D, dtype, **kw):
    if dtype == "fp8":
        return gem.score_quant(Q, D, **kw)
    return gem.score_exact(Q, D, compute=dtype, **kw)


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_qch_dense_matches_oracle_and_materialized_sets(dtype):
    C, qo, qc, do, dc, qmax = _qch_case()
    Q = _code_sets(C, qo, qc, qmax, dtype)
    D = _code_sets(C, do, dc, 90, dtype)
    gem.validate_sets(Q)
    gem.validate_sets(D)
    _, _, got = _score(Q, D, dtype, k=10, want_scores=True)
    ref = oracle.qch_dense(qc, qo, dc, do, _codebook_values(C, dtype))
    g = _np(got).astype(np.float64)
    assert np.array_equal(np.isinf(g), np.isinf(ref))
    fin = ~np.isinf(ref)
    rel = np.abs(g[fin] - ref[fin]) / np.maximum(np.abs(ref[fin]), 1.0)
    assert rel.max() <= TOL, f"qCH dense {dtype}: {rel.max():.3e}"
    # the same sets with every centroid row written out score bitwise the same
    Qm = gem.Sets(_rows_of(Q.vecs, Q.codes), Q.offsets, Q.dtype, qmax,
                  scales=None if Q.scales is None else Q.scales[Q.codes.long()].contiguous())
    Dm = gem.Sets(_rows_of(D.vecs, D.codes), D.offsets, D.dtype, 90,
                  scales=None if D.scales is None else D.scales[D.codes.long()].contiguous())
    _, _, mat = _score(Qm, Dm, dtype, k=10, want_scores=True)
    np.testing.assert_array_equal(_np(got), _np(mat))


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_qch_gather_matches_dense_and_oracle(dtype):
    C, qo, qc, do, dc, qmax = _qch_case(6)
    Q = _code_sets(C, qo, qc, qmax, dtype)
    D = _code_sets(C, do, dc, 90, dtype)
    rng = np.random.default_rng(9)
    lens = rng.integers(0, 70, 40)
    co = _csr(lens)
    ids = rng.integers(0, 500, int(co[-1])).astype(np.int32)
    ids[::13] = -1                                                # padding entries
    cands = gem.Cands(torch.from_numpy(ids).to(DEV), torch.from_numpy(co).to(DEV))
    _, _, dense = _score(Q, D, dtype, k=10, want_scores=True)
    _, _, got = _score(Q, D, dtype, cands=cands, k=5, want_scores=True)
    dn, gt = _np(dense), _np(got)
    for i in range(40):
        for e in range(co[i], co[i + 1]):
            want = -np.inf if ids[e] < 0 else dn[i, ids[e]]
            assert gt[e] == want or (np.isinf(want) and np.isinf(gt[e]))
    ref = oracle.qch_cands(qc, qo, dc, do, co, np.where(ids < 0, 0, ids), _codebook_values(C, dtype))
    ok = ids >= 0
    fin = ok & ~np.isinf(ref)
    rel = np.abs(gt[fin] - ref[fin]) / np.maximum(np.abs(ref[fin]), 1.0)
    assert rel.max() <= TOL


@pytest.mark.parametrize("order", ["document", "auto"])
def test_qch_gather_orders_fall_back_to_the_query_order(order):
    """Code sets are not scored by document: asking for the document order
    (or auto, with lists that hold many entries per document) gives the query
    order's scores bitwise, here on lists of 2000 entries over 500 documents."""
    C, qo, qc, do, dc, qmax = _qch_case(8)
    Q = _code_sets(C, qo, qc, qmax, "fp8")
    D = _code_sets(C, do, dc, 90, "fp8")
    rng = np.random.default_rng(10)
    n_q = len(qo) - 1
    ids = rng.integers(0, 500, n_q * 2000).astype(np.int32)
    cands = gem.Cands(torch.from_numpy(ids).to(DEV), stride=2000, n_lists=n_q)
    gem.set_gather_order("query")
    try:
        want = _np(_score(Q, D, "fp8", cands=cands))
        gem.set_gather_order(order)
        got = _np(_score(Q, D, "fp8", cands=cands))
    finally:
        gem.set_gather_order("auto")
    np.testing.assert_array_equal(got.view(np.int32), want.view(np.int32))


def test_code_set_validation_and_mixed_sets():
    C, qo, qc, do, dc, qmax = _qch_case(7)
    D = _code_sets(C, do, dc, 90, "bf16")
    bad = dc.astype(np.int32).copy()
    bad[5] = 300                                                  # past the codebook
    Dbad = gem.Sets(D.vecs, D.offsets, "bf16", 90, codes=torch.from_numpy(bad).to(DEV))
    with pytest.raises(gem.GemError) as e:
        gem.validate_sets(Dbad)
    assert e.value.status == gem._abi.GEM_ERR_DEVICE_CHECK
    # plain float32 queries against bf16 code documents: the query is converted,
    # the documents stay codes
    xq = C[qc] + 0.0
    Qp = gem.Sets(torch.from_numpy(xq.astype(np.float32)).to(DEV), torch.from_numpy(qo).to(DEV), "f32", qmax)
    _, _, got = gem.score_exact(Qp, D, compute="bf16", k=3, want_scores=True)
    Qc = _code_sets(C, qo, qc, qmax, "bf16")
    _, _, want = gem.score_exact(Qc, D, compute="bf16", k=3, want_scores=True)
    np.testing.assert_array_equal(_np(got), _np(want))
