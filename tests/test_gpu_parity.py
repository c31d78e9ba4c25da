"""GPU parity: the HIP path against the float64 CPU oracle on seeded inputs.

Tolerances. Every product of the bf16 / FP8 operands is exact in float32, so
the kernels differ from the oracle (run on the same rounded operands) only by
float32 accumulation: per dot product at most gamma_128 * sum|a_t p_t|
(gamma_n = n u / (1 - n u), u = 2^-24; about 7.6e-6 for unit vectors), and the
max is 1-Lipschitz, so a score of m_q maxima is off by at most about
m_q * 7.6e-6 + gamma_{m_q} |score|. Relative to max(|score|, 1) that is below
1e-4 for m_q <= 13 and below 3e-4 at m_q = 32 in the worst case; typical
errors are ~1e-6. The tests use 1e-4 relative (the exactness target), with
the worst-case bound asserted separately on the largest queries.
Top-k sets are compared outside a tie band of 2 * tol * max(|s_k|, 1).
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


def _np(t):
    return t.detach().cpu().numpy()


def _operands(vecs_f32: np.ndarray, dtype: str) -> np.ndarray:
    """The exact values the GPU multiplies, computed by the oracle's own codecs."""
    if dtype == "f32":
        return vecs_f32.astype(np.float64)
    if dtype == "bf16":
        return oracle.bf16_decode(oracle.bf16_round_bits(vecs_f32))
    codes, scales = oracle.quantize_fp8(vecs_f32)
    return oracle.dequantize_fp8(codes, scales)


def _device_sets(batch: wl.SetBatch, dtype: str) -> gem.Sets:
    S = gem.Sets.from_batch(batch, DEV)
    if dtype == "bf16":
        return S.to_bf16()
    if dtype == "fp8":
        return S.to_fp8()
    return S


def _score(Q, D, dtype, **kw):
    if dtype == "fp8":
        return gem.score_quant(Q, D, **kw)
    return gem.score_exact(Q, D, compute=dtype, **kw)


def assert_close(got, ref, tol=TOL, what=""):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    assert got.shape == ref.shape
    inf_ref = np.isinf(ref)
    assert np.array_equal(np.isinf(got), inf_ref), f"{what}: -inf pattern differs"
    assert np.array_equal(got[inf_ref], ref[inf_ref])
    fin = ~inf_ref
    if fin.any():
        rel = np.abs(got[fin] - ref[fin]) / np.maximum(np.abs(ref[fin]), 1.0)
        assert rel.max() <= tol, f"{what}: max rel err {rel.max():.3e} > {tol}"


def _csr(lengths):
    o = np.zeros(len(lengths) + 1, np.int64)
    o[1:] = np.cumsum(lengths)
    return o


def _ragged(lengths, seed):
    """Unit vectors from a small mixture, with the given set lengths."""
    centers = wl.mixture_centers(8, seed)
    g = torch.Generator().manual_seed(seed + 1)
    vecs = wl.mixture_vectors(int(sum(lengths)), centers, 0.1, g)
    return wl.SetBatch(vecs, torch.from_numpy(_csr(lengths)))


# ----------------------------------------------------------------------- conversions
def test_convert_bf16_bitwise():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(128 * 2000) * 10.0 ** rng.integers(-20, 20, 128 * 2000)).astype(np.float32)
    halfway = ((rng.integers(1, 254, 4096).astype(np.uint32) << 23) | (rng.integers(0, 128, 4096).astype(np.uint32) << 16)
               | np.uint32(0x8000)).view(np.float32)
    x[: halfway.size] = halfway
    x[5000:5004] = [0.0, -0.0, 3.39e38, -1e-45]
    b = wl.SetBatch(torch.from_numpy(x.reshape(-1, 128)), torch.tensor([0, 2000], dtype=torch.int64))
    got = _np(gem.Sets.from_batch(b, DEV).to_bf16().vecs).reshape(-1)
    np.testing.assert_array_equal(got, oracle.bf16_round_bits(x))


def test_quantize_fp8_bitwise():
    c = wl.corpus(wl.WORKLOADS[1], n_docs=200)
    x = c.vecs.numpy().copy()
    rng = np.random.default_rng(1)
    extra = [np.zeros(128, np.float32),                                      # all-zero row: scale 1
             (rng.standard_normal(128) * 1e3).astype(np.float32),
             (rng.standard_normal(128) * 1e-30).astype(np.float32),
             (rng.standard_normal(128) * 1e-42).astype(np.float32),          # subnormal row: clamped scale
             np.full(128, 448.0, np.float32),
             np.linspace(-1, 1, 128).astype(np.float32)]
    t = oracle.e4m3_decode_table()[:0x7F]
    mids = ((t[1:] + t[:-1]) / 2).astype(np.float32)                         # exact midpoints of the grid
    mids = np.concatenate([mids, [447.0, -3.0]]).astype(np.float32)         # 126 + 2 = one row
    extra.append(mids)
    x = np.vstack([x] + [e[None] for e in extra])
    b = wl.SetBatch(torch.from_numpy(x), torch.tensor([0, x.shape[0]], dtype=torch.int64))
    S = gem.Sets.from_batch(b, DEV).to_fp8()
    codes, scales = oracle.quantize_fp8(x)
    np.testing.assert_array_equal(_np(S.scales), scales)
    np.testing.assert_array_equal(_np(S.vecs), codes)


def test_quantize_fp8_beyond_one_dispatch():
    """More rows than one dispatch's 32-bit work-item count covers at one wave
    a row (2^32 / 64 = 67,108,864): rows past that bound are quantized too."""
    n_rows = 70_000_000
    free, _ = torch.cuda.mem_get_info()
    if free < n_rows * 128 * 6 + (4 << 30):
        pytest.skip("needs about 45 GB of free device memory")
    g = torch.Generator(device=DEV).manual_seed(7)
    x = torch.randn(n_rows, 128, device=DEV, generator=g)
    x[-1] *= 1e-3
    off = torch.tensor([0, n_rows], dtype=torch.int64, device=DEV)
    S = gem.quantize_fp8(gem.Sets(x, off, "f32", 0))
    rows = torch.tensor([0, 1, 2**26, 67_108_863, 67_108_864, 67_108_865, 68_000_000, n_rows - 1], device=DEV)
    xs = _np(x[rows])
    codes, scales = oracle.quantize_fp8(xs)
    np.testing.assert_array_equal(_np(S.scales[rows]), scales)
    np.testing.assert_array_equal(_np(S.vecs[rows]), codes)
    del S, x
    torch.cuda.empty_cache()


@pytest.mark.parametrize("row_bytes", [512, 128, 20])
def test_copy_rows_gather_scatter_bitwise(row_bytes):
    rng = np.random.default_rng(row_bytes)
    n_src, n_dst, n = 300, 260, 200
    src = torch.from_numpy(rng.integers(0, 2**32, (n_src, row_bytes // 4), dtype=np.uint32).view(np.int32)).to(DEV)
    dst0 = rng.integers(0, 2**32, (n_dst, row_bytes // 4), dtype=np.uint32).view(np.int32)
    si = rng.integers(0, n_src, n).astype(np.int64)
    di = rng.permutation(n_dst)[:n].astype(np.int64)
    dst = torch.from_numpy(dst0.copy()).to(DEV)
    gem.copy_rows(src, dst, src_idx=torch.from_numpy(si).to(DEV), dst_idx=torch.from_numpy(di).to(DEV))
    want = dst0.copy()
    want[di] = src.cpu().numpy()[si]
    np.testing.assert_array_equal(dst.cpu().numpy(), want)
    dst = torch.from_numpy(dst0.copy()).to(DEV)
    gem.copy_rows(src, dst, src_idx=torch.from_numpy(si).to(DEV), n=n)           # gather into the leading rows
    want = dst0.copy()
    want[:n] = src.cpu().numpy()[si]
    np.testing.assert_array_equal(dst.cpu().numpy(), want)
    gem.copy_rows(src, dst, n=0)                                                  # empty copy is a no-op
    np.testing.assert_array_equal(dst.cpu().numpy(), want)


# ----------------------------------------------------------------------- dense (exhaustive)
@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_dense_workload1_matches_oracle(dtype):
    w = wl.WORKLOADS[1]
    c, q = wl.corpus(w), wl.queries(w)
    D, Q = _device_sets(c, dtype), gem.Sets.from_batch(q, DEV)
    top_s, top_i, scores = _score(Q, D, dtype, k=w.k, want_scores=True)
    torch.cuda.synchronize()
    ref = oracle.ch_dense(_operands(q.vecs.numpy(), dtype), q.offsets.numpy(),
                          _operands(c.vecs.numpy(), dtype), c.offsets.numpy())
    assert_close(_np(scores), ref, what=f"dense {dtype}")
    ti, ts = _np(top_i), _np(top_s)
    for r in range(Q.n_sets):
        tau = 2 * TOL * max(abs(np.sort(ref[r])[::-1][w.k - 1]), 1.0)
        ok, bad, missing = oracle.tie_aware_match(ti[r], ref[r], w.k, tau)
        assert ok, (r, bad, missing)
        np.testing.assert_allclose(ts[r], ref[r][ti[r]], rtol=0, atol=TOL * max(1, abs(ts[r][0])))


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_dense_ragged_edges(dtype):
    qlens = [1, 2, 31, 32, 33, 64, 0, 17, 256, 5, 128, 129]
    dlens = [1, 15, 16, 17, 255, 256, 0, 3, 64, 65] + list(np.random.default_rng(2).integers(1, 90, 121))
    q, c = _ragged(qlens, 10), _ragged(dlens, 20)
    D, Q = _device_sets(c, dtype), gem.Sets.from_batch(q, DEV)
    scores = _score(Q, D, dtype)
    torch.cuda.synchronize()
    ref = oracle.ch_dense(_operands(q.vecs.numpy(), dtype), q.offsets.numpy(),
                          _operands(c.vecs.numpy(), dtype), c.offsets.numpy())
    # the 256-vector query may reach the worst-case accumulation bound
    assert_close(_np(scores), ref, tol=3e-4, what=f"ragged {dtype}")
    small = np.array(qlens) <= 64
    assert_close(_np(scores)[small], ref[small], what=f"ragged {dtype} (m_q <= 64)")


def test_dense_rows_and_ld_layout():
    """Scores land at row(i) * ld + j: the placement the serving loop uses."""
    q, c = _ragged([3, 7, 2], 30), _ragged([4, 9, 1, 6, 2] * 30, 31)
    D, Q = _device_sets(c, "bf16"), gem.Sets.from_batch(q, DEV)
    base = _score(Q, D, "bf16")
    out = torch.full((6, 200), 7.0, device=DEV)
    rows = torch.tensor([4, 0, 2], dtype=torch.int32, device=DEV)
    gem.score_exact(Q, D, compute="bf16", scores=out, ld=200, rows=rows)
    torch.cuda.synchronize()
    o = _np(out)
    for i, r in enumerate([4, 0, 2]):
        np.testing.assert_array_equal(o[r, :150], _np(base)[i])
        assert (o[r, 150:] == 7.0).all()
    assert (o[[1, 3, 5]] == 7.0).all()


def test_batch_independence_bitwise():
    """A query's scores are bitwise the same alone and inside a larger batch."""
    w = wl.WORKLOADS[1]
    c, q = wl.corpus(w, n_docs=300), wl.queries(w, n_queries=40, query_len=("uniform", 4, 64))
    for dtype in ("f32", "bf16", "fp8"):
        D = _device_sets(c, dtype)
        full = _np(_score(gem.Sets.from_batch(q, DEV), D, dtype))
        for i in (0, 17, 39):
            alone = _np(_score(gem.Sets.from_batch(q.subset([i]), DEV), D, dtype))
            np.testing.assert_array_equal(alone[0], full[i])
        sub = _np(_score(gem.Sets.from_batch(q.subset([5, 3, 30]), DEV), D, dtype))
        np.testing.assert_array_equal(sub, full[[5, 3, 30]])


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8", "mxfp4"])
def test_small_batches_stream_bitwise_as_dense(dtype):
    """A few queries (up to three; one for FP8) take the streamed path of a
    dense call, a few more short ones the narrow-block scorer: the same
    scores, bitwise, as the dense scorer gives them inside a larger batch (and
    the oracle's), with empty and long queries, empty and long documents, and
    the rows / ld placement."""
    qlens = [0, 1, 33, 64, 256, 17]
    dlens = [1, 15, 16, 17, 255, 256, 0, 3, 64, 65] + list(np.random.default_rng(3).integers(1, 90, 150))
    q, c = _ragged(qlens + [5, 9, 40, 2], 40), _ragged(dlens, 41)
    S = gem.Sets.from_batch(c, DEV)
    D = S.to_mxfp4() if dtype == "mxfp4" else _device_sets(c, dtype)
    score = (lambda Q, **kw: gem.score_quant(Q, D, **kw)) if dtype == "mxfp4" else \
        (lambda Q, **kw: _score(Q, D, dtype, **kw))
    big = _np(score(gem.Sets.from_batch(q, DEV)))                       # ten queries: the dense scorer
    for idx in ([0, 1, 2, 3, 4, 5], [4], [2, 0, 5], [1, 3]):
        small = _np(score(gem.Sets.from_batch(q.subset(idx), DEV)))
        np.testing.assert_array_equal(small, big[idx])
    out = torch.full((8, 200), 7.0, device=DEV)
    rows = torch.tensor([6, 1, 3], dtype=torch.int32, device=DEV)
    score(gem.Sets.from_batch(q.subset([3, 4, 5]), DEV), scores=out[:, 20:], ld=200, rows=rows)
    o = _np(out)
    for i, r in enumerate([6, 1, 3]):
        np.testing.assert_array_equal(o[r, 20:180], big[3 + i])
        assert (o[r, :20] == 7.0).all() and (o[r, 180:] == 7.0).all()
    assert (o[[0, 2, 4, 5, 7]] == 7.0).all()
    if dtype != "mxfp4":
        ref = oracle.ch_dense(_operands(q.vecs.numpy(), dtype), q.offsets.numpy(),
                              _operands(c.vecs.numpy(), dtype), c.offsets.numpy())
        assert_close(big[:6], ref[:6], tol=3e-4, what=f"streamed {dtype}")
    # a dozen short queries: the dense scorer with narrowed query blocks (one
    # per wave; for FP8 the narrow-block variant) against the same queries
    # inside a batch of 80 (full blocks)
    q2 = _ragged(list(np.random.default_rng(4).integers(1, 41, 80)), 42)
    big2 = _np(score(gem.Sets.from_batch(q2, DEV)))
    idx = [3, 7, 0, 12, 40, 41, 42, 43, 44, 60, 61, 79]
    np.testing.assert_array_equal(_np(score(gem.Sets.from_batch(q2.subset(idx), DEV))), big2[idx])
    idx = list(range(20, 45))                           # FP8: two block groups of narrow blocks
    np.testing.assert_array_equal(_np(score(gem.Sets.from_batch(q2.subset(idx), DEV))), big2[idx])
    if dtype != "mxfp4":
        ref2 = oracle.ch_dense(_operands(q2.vecs.numpy(), dtype), q2.offsets.numpy(),
                               _operands(c.vecs.numpy(), dtype), c.offsets.numpy())
        assert_close(big2, ref2, what=f"dense {dtype}, 80 short queries")


def test_fp8_narrow_blocks_over_many_block_groups():
    """A batch of 150 short FP8 queries takes 64-column blocks over many block
    groups (the narrow-block variant): the same scores, bitwise, as inside a
    batch of 400 (full-width blocks), the oracle's within the tolerance, and the
    fused top-k equal to the top-k of those scores."""
    rng = np.random.default_rng(14)
    q = _ragged(list(rng.integers(1, 65, 400)), 52)
    c = _ragged(list(rng.integers(1, 120, 900)), 53)
    D = _device_sets(c, "fp8")
    big = _np(gem.score_quant(gem.Sets.from_batch(q, DEV), D))
    idx = list(range(100, 250))
    Qs = gem.Sets.from_batch(q.subset(idx), DEV)
    small = gem.score_quant(Qs, D)
    np.testing.assert_array_equal(_np(small), big[idx])
    gem.set_topk_fusion("fused")
    try:
        ts, ti = gem.score_quant(Qs, D, k=10)
    finally:
        gem.set_topk_fusion("auto")
    rs, ri = gem.topk(small, 10)
    np.testing.assert_array_equal(_np(ti), _np(ri))
    np.testing.assert_array_equal(_np(ts), _np(rs))
    sub = q.subset(idx)
    ref = oracle.ch_dense(_operands(sub.vecs.numpy(), "fp8"), sub.offsets.numpy(),
                          _operands(c.vecs.numpy(), "fp8"), c.offsets.numpy())
    assert_close(_np(small), ref, what="fp8 narrow blocks, 150 queries")


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_dense_many_blocks_long_documents(dtype):
    """More than 32 block groups for every dtype (more groups than workgroups
    per XCD), documents of up to 1000 vectors and a chunk of them (a 64-document
    chunk holding hundreds of tiles), and a document count that leaves a partial
    last chunk."""
    rng = np.random.default_rng(12)
    qlens = list(rng.integers(1, 101, 1100))
    dlens = [300, 700, 0, 1, 1000] + list(rng.integers(1, 200, 126))
    q, c = _ragged(qlens, 50), _ragged(dlens, 51)
    D, Q = _device_sets(c, dtype), gem.Sets.from_batch(q, DEV)
    scores = _score(Q, D, dtype)
    torch.cuda.synchronize()
    ref = oracle.ch_dense(_operands(q.vecs.numpy(), dtype), q.offsets.numpy(),
                          _operands(c.vecs.numpy(), dtype), c.offsets.numpy())
    assert_close(_np(scores), ref, what=f"many blocks {dtype}")


@pytest.fixture(scope="module")
def exhaustive_100k():
    """The exhaustive-100k workload (1000 queries x 32 vectors, 100,000 documents
    with lognormal lengths), generated on the device as the benchmark does."""
    w2 = wl.WORKLOADS[2]
    c = wl.corpus(w2, device=DEV)
    q = wl.queries(w2, device=DEV)
    yield w2, c, q
    del c, q
    torch.cuda.empty_cache()


def _sub_host(batch: wl.SetBatch, idx) -> wl.SetBatch:
    s = batch.subset(list(idx))
    return wl.SetBatch(s.vecs.cpu(), s.offsets.cpu())


@pytest.mark.parametrize("dtype", ["bf16", "fp8", "f32"])
def test_dense_full_size_sampled(exhaustive_100k, dtype):
    """Full size, in the benchmark's launch configuration: sampled (query,
    document) pairs against the oracle, including chunk-boundary documents."""
    w2, c, q = exhaustive_100k
    D = _device_sets(c, dtype)
    Q = gem.Sets(q.vecs, q.offsets, "f32", q.max_len())
    scores = _score(Q, D, dtype)
    torch.cuda.synchronize()
    n_d = c.n_sets
    rng = np.random.default_rng(13)
    qs = [0, 1, 31, 32, 499, 998, 999]
    ds = sorted(set(rng.integers(0, n_d, 150).tolist()) | {0, 63, 64, 65, 127, 128, n_d - 65, n_d - 1})
    sq, sd = _sub_host(q, qs), _sub_host(c, ds)
    ref = oracle.ch_dense(_operands(sq.vecs.numpy(), dtype), sq.offsets.numpy(),
                          _operands(sd.vecs.numpy(), dtype), sd.offsets.numpy())
    got = _np(scores[qs][:, ds])
    assert_close(got, ref, what=f"full size {dtype}")


def test_dense_full_size_row_and_top100(exhaustive_100k):
    """Full size: one query's whole bf16 row against the oracle, and its top-100
    (the benchmark step's output) against the oracle's ranking outside ties."""
    w2, c, q = exhaustive_100k
    D = _device_sets(c, "bf16")
    Q = gem.Sets(q.vecs, q.offsets, "f32", q.max_len())
    scores = _score(Q, D, "bf16")
    top_s, top_i = gem.topk(scores, w2.k)
    torch.cuda.synchronize()
    qi = 7
    sq = _sub_host(q, [qi])
    qop = _operands(sq.vecs.numpy(), "bf16")
    off = c.offsets.cpu().numpy()
    row = np.empty(c.n_sets)
    step = 5000
    for j0 in range(0, c.n_sets, step):
        j1 = min(c.n_sets, j0 + step)
        r0, r1 = int(off[j0]), int(off[j1])
        dv = _operands(c.vecs[r0:r1].cpu().numpy(), "bf16")
        row[j0:j1] = oracle.ch_dense(qop, sq.offsets.numpy(), dv, off[j0:j1 + 1] - r0)[0]
    assert_close(_np(scores[qi]), row, what="full row")
    tau = 2 * TOL * max(abs(np.sort(row)[::-1][w2.k - 1]), 1.0)
    ok, bad, missing = oracle.tie_aware_match(_np(top_i[qi]), row, w2.k, tau)
    assert ok, (bad, missing)


def test_fused_topk_full_size(exhaustive_100k):
    """The benchmark's calls with the top-k fused into the scorer (no score
    matrix): bf16 top-100 and the FP8 shortlist of 1000, bitwise the top-k of
    the staged score rows."""
    w2, c, q = exhaustive_100k
    Q = gem.Sets(q.vecs, q.offsets, "f32", q.max_len())
    for dtype, k in (("bf16", 100), ("fp8", 1000)):
        D = _device_sets(c, dtype)
        assert gem.score_workspace_bytes(Q, D, k=k) < Q.n_sets * D.n_sets * 4
        fs, fi = _score(Q, D, dtype, k=k)
        scores = _score(Q, D, dtype)
        ss, si = gem.topk(scores, k)
        torch.cuda.synchronize()
        assert torch.equal(fi, si), dtype
        assert torch.equal(fs.view(torch.int32), ss.view(torch.int32)), dtype
        del D, scores


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_dense_schedules_bitwise_and_autotune(dtype):
    """Every dense schedule computes bitwise the same scores; the autotuner
    installs one of them for the call's shape class, and the default returns
    when the class is cleared."""
    rng = np.random.default_rng(14)
    q = _ragged(list(rng.integers(1, 65, 90)), 60)
    c = _ragged(list(rng.integers(0, 120, 700)), 61)
    D, Q = _device_sets(c, dtype), gem.Sets.from_batch(q, DEV)
    gem.set_dense_schedule(dtype, Q.n_vecs, D.n_sets, None)
    default = gem.dense_schedule(dtype, Q.n_vecs, D.n_sets)
    base = _np(_score(Q, D, dtype))
    ref = oracle.ch_dense(_operands(q.vecs.numpy(), dtype), q.offsets.numpy(),
                          _operands(c.vecs.numpy(), dtype), c.offsets.numpy())
    assert_close(base, ref, what=f"schedules {dtype}")
    spx = default["slots_per_xcd"]
    for cd in (32, 64):
        for ips in (1, 3, 8, 64):
            for slots in (spx, max(1, spx // 4)):
                gem.set_dense_schedule(dtype, Q.n_vecs, D.n_sets,
                                       {"chunk_docs": cd, "items_per_slot": ips, "slots_per_xcd": slots})
                got = _np(_score(Q, D, dtype))
                np.testing.assert_array_equal(got, base, err_msg=f"{dtype} {cd} {ips} {slots}")
    with pytest.raises(gem.GemError):
        gem.set_dense_schedule(dtype, Q.n_vecs, D.n_sets, {"chunk_docs": 48, "items_per_slot": 8,
                                                           "slots_per_xcd": spx})
    best, ms = gem.autotune_dense(Q, D, reps=1)
    assert ms > 0 and best["chunk_docs"] in (32, 64) and best["items_per_slot"] in (2, 4, 8, 16)
    assert best["slots_per_xcd"] in (spx, (3 * spx) // 4, spx // 2)
    assert gem.dense_schedule(dtype, Q.n_vecs, D.n_sets) == best
    np.testing.assert_array_equal(_np(_score(Q, D, dtype)), base)
    gem.set_dense_schedule(dtype, Q.n_vecs, D.n_sets, None)
    assert gem.dense_schedule(dtype, Q.n_vecs, D.n_sets) == default


# ----------------------------------------------------------------------- gathered
@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_gather_matches_oracle_and_dense(dtype):
    qlens = [32, 1, 0, 64, 200, 7]
    dlens = list(np.random.default_rng(3).integers(0, 130, 300))
    q, c = _ragged(qlens, 40), _ragged(dlens, 41)
    rng = np.random.default_rng(4)
    lists = [rng.integers(0, 300, 37), np.array([5, 5, -1, 7, 0]), np.array([], np.int64),
             rng.integers(-1, 300, 70), rng.integers(0, 300, 16), np.arange(300)]
    co = _csr([len(x) for x in lists])
    ci = np.concatenate(lists).astype(np.int32)
    C = gem.Cands(torch.from_numpy(ci).to(DEV), torch.from_numpy(co).to(DEV))
    D, Q = _device_sets(c, dtype), gem.Sets.from_batch(q, DEV)
    got = _np(_score(Q, D, dtype, cands=C))
    dense = _np(_score(Q, D, dtype))
    torch.cuda.synchronize()
    qo, do = _operands(q.vecs.numpy(), dtype), _operands(c.vecs.numpy(), dtype)
    ref = oracle.ch_cands(qo, q.offsets.numpy(), do, c.offsets.numpy(), co, np.maximum(ci, 0))
    ref[ci < 0] = -np.inf
    assert_close(got, ref, tol=3e-4, what=f"gather {dtype}")
    # the same (query, document) pair scores bitwise the same in both kernels
    for i in range(len(lists)):
        for e in range(co[i], co[i + 1]):
            if ci[e] >= 0:
                assert got[e] == dense[i, ci[e]], (dtype, i, e)


# ----------------------------------------------------------------------- top-k
@pytest.mark.parametrize("mode", ["csr_ids", "csr_pos", "rows"])
def test_topk_bitwise(mode):
    s, off = wl.random_scores(24, ("uniform", 0, 9000), seed=5, tie_frac=0.3)
    s_np, off_np = s.numpy(), off.numpy()
    rng = np.random.default_rng(6)
    ids = rng.integers(-1, 5000, s_np.size).astype(np.int32)        # repeats and padding ids
    for k in (1, 10, 100, 1000, 1024, 2048):
        if mode == "rows":
            n, L = 12, 7000
            mat = np.random.default_rng(7).standard_normal((n, L)).astype(np.float32)
            mat[:, ::7] = 0.5                                       # large ties
            rows = np.array([3, 0, 11, 5, 5], np.int32)
            ts, ti = gem.topk(torch.from_numpy(mat).to(DEV), k, seg_rows=torch.from_numpy(rows).to(DEV))
            rs, ri = oracle.topk_rows(mat[rows], k)
        elif mode == "csr_pos":
            ts, ti = gem.topk(s.to(DEV), k, seg_offsets=off.to(DEV))
            rs, ri = oracle.topk_segments(s_np, off_np, k)
        else:
            ts, ti = gem.topk(s.to(DEV), k, seg_offsets=off.to(DEV), seg_ids=torch.from_numpy(ids).to(DEV))
            keep = ids >= 0
            # the oracle skips padding ids: drop them from each segment first
            seg = np.repeat(np.arange(len(off_np) - 1), np.diff(off_np))
            o2 = np.zeros_like(off_np)
            o2[1:] = np.cumsum(np.bincount(seg[keep], minlength=len(off_np) - 1))
            rs, ri = oracle.topk_segments(s_np[keep], o2, k, ids[keep])
        torch.cuda.synchronize()
        np.testing.assert_array_equal(_np(ti), ri)
        np.testing.assert_array_equal(_np(ts), rs.astype(np.float32))


def test_topk_long_positional_segments_every_alignment():
    """Positional segments longer than the in-LDS capacity (the sampled path
    reads them with 16-byte loads) starting at every offset mod 4 and ending
    with 0-3 entries past the last whole vector: bitwise the oracle's top-k."""
    rng = np.random.default_rng(21)
    lens = [5001, 4097, 6002, 4099, 8192, 4103, 7000, 4098]
    off = np.zeros(len(lens) + 2, np.int64)
    off[1] = 1                                                      # segments start 1 entry in
    off[2:] = 1 + np.cumsum(lens)
    starts = off[1:-1]
    assert sorted(set(int(x) % 4 for x in starts)) == [0, 1, 2, 3]
    sc = rng.standard_normal(int(off[-1])).astype(np.float32)
    sc[off[1]:off[2]] = rng.integers(0, 40, lens[0]).astype(np.float32)   # heavy ties in one segment
    for k in (1, 100, 1000):
        ts, ti = gem.topk(torch.from_numpy(sc).to(DEV), k, seg_offsets=torch.from_numpy(off[1:]).to(DEV))
        rs, ri = oracle.topk_segments(sc, off[1:], k)
        np.testing.assert_array_equal(_np(ti), ri)
        np.testing.assert_array_equal(_np(ts), rs.astype(np.float32))


def test_topk_long_segments_with_repeats():
    """Radix path (segments longer than the in-LDS capacity) with repeated ids."""
    rng = np.random.default_rng(8)
    n = 3
    L = 20000
    sc = rng.standard_normal(n * L).astype(np.float32)
    ids = rng.integers(0, 150, n * L).astype(np.int32)              # heavy repetition
    sc[ids < 40] = 2.5                                              # repeated ids, equal scores
    off = np.arange(n + 1, dtype=np.int64) * L
    for k in (5, 100):
        ts, ti = gem.topk(torch.from_numpy(sc).to(DEV), k, seg_offsets=torch.from_numpy(off).to(DEV),
                          seg_ids=torch.from_numpy(ids).to(DEV))
        rs, ri = oracle.topk_segments(sc, off, k, ids)
        np.testing.assert_array_equal(_np(ti), ri)
        np.testing.assert_array_equal(_np(ts), rs.astype(np.float32))


# ----------------------------------------------------------------------- beam
@pytest.mark.parametrize("n_q,ef,max_list,n_docs", [(9, 50, 80, 2000), (6, 1000, 1000, 30000),
                                                    (5, 8, 1500, 20000), (5, 1024, 3000, 20000)])
def test_beam_merge_bitwise(n_q, ef, max_list, n_docs):
    """Beam updates against the oracle's replay: merges of up to 2048 entries
    with beams and lists of up to 1024 (the sorted-beam merge), lists longer
    than that (the full sort) and ef = 1024 with 3000-entry lists (the largest
    merge is ef + list = 4024 entries). Even steps draw scores with ties, so a
    listed id the beam holds may score above or below the beam's entry."""
    beam = gem.Beam(n_q, ef, DEV)
    steps = []
    for st in range(6):
        s, off = wl.random_scores(n_q, ("uniform", 0, max_list), seed=100 + st, tie_frac=0.2)
        ids = wl.candidate_ids(1, int(off[-1]) or 1, n_docs, seed=200 + st).reshape(-1)[: int(off[-1])]
        # a document keeps one score across steps
        s = torch.from_numpy(np.sin(ids.numpy().astype(np.float64) * 0.37).astype(np.float32)) if st % 2 else s
        C = gem.Cands(ids.contiguous().to(DEV), off.to(DEV))
        gem.beam_merge(s.to(DEV), C, beam)
        steps.append((s.numpy(), off.numpy(), ids.numpy()))
    torch.cuda.synchronize()
    rs, ri = oracle.beam_replay(n_q, ef, steps)
    np.testing.assert_array_equal(_np(beam.ids), ri)
    np.testing.assert_array_equal(_np(beam.scores), rs.astype(np.float32))


@pytest.mark.parametrize("ef", [1, 64, 1023])
def test_beam_merge_list_length_boundaries(ef):
    """Lists of exactly 1024 entries (the longest the sorted-beam merge takes),
    1025 (the full sort in the same launch), a single entry and none, merged
    twice (the second time into rows in the stored form), against the oracle."""
    rng = np.random.default_rng(ef)
    lens = [1024, 1025, 1, 0]
    beam = gem.Beam(len(lens), ef, DEV)
    steps = []
    for st in range(2):
        off = np.zeros(len(lens) + 1, np.int64)
        off[1:] = np.cumsum(lens)
        ids = rng.integers(0, 3000, int(off[-1])).astype(np.int32)       # repeats across and within lists
        sc = np.sin(ids.astype(np.float64) * 0.71 + st).astype(np.float32) if st else \
            rng.integers(0, 16, ids.size).astype(np.float32)            # ties, then one score per id
        gem.beam_merge(torch.from_numpy(sc).to(DEV), gem.Cands(torch.from_numpy(ids).to(DEV),
                                                                torch.from_numpy(off).to(DEV)), beam)
        steps.append((sc, off, ids))
    torch.cuda.synchronize()
    rs, ri = oracle.beam_replay(len(lens), ef, steps)
    np.testing.assert_array_equal(_np(beam.ids), ri)
    np.testing.assert_array_equal(_np(beam.scores), rs.astype(np.float32))


def test_beam_merge_rows_in_any_form():
    """Beam rows written by the caller: in the stored form (sorted, padded at
    the tail), out of order, with a repeated id, with padding in the middle and
    empty; lists with padding ids, repeated ids and ids the beam holds at a
    better, equal or worse score. Every row is the oracle's merge, bitwise."""
    rng = np.random.default_rng(31)
    ef, n_q = 64, 6
    bs = np.full((n_q, ef), -np.inf, np.float32)
    bi = np.full((n_q, ef), -1, np.int32)

    def stored(ids, sc):
        o = np.lexsort((ids, -sc))
        return sc[o], ids[o]

    for q in (0, 5):
        ids = rng.choice(500, 40, replace=False).astype(np.int32)
        sc = rng.integers(0, 8, 40).astype(np.float32)              # ties
        bs[q, :40], bi[q, :40] = stored(ids, sc)
    ids = rng.choice(500, ef, replace=False).astype(np.int32)
    bs[1], bi[1] = rng.standard_normal(ef).astype(np.float32), ids    # out of order
    sc2, id2 = stored(rng.choice(500, 30, replace=False).astype(np.int32),
                      rng.standard_normal(30).astype(np.float32))
    id2[20] = id2[3]                                                # a repeated id
    bs[2, :30], bi[2, :30] = sc2, id2
    sc3, id3 = stored(rng.choice(500, 30, replace=False).astype(np.int32),
                      rng.standard_normal(30).astype(np.float32))
    bs[3, :10], bi[3, :10] = sc3[:10], id3[:10]
    bs[3, 12:32], bi[3, 12:32] = sc3[10:], id3[10:]                 # padding in the middle
    lists_s, lists_i = [], []
    for q in range(n_q):
        n = int(rng.integers(0, 90))
        li = rng.integers(0, 500, n).astype(np.int32)
        ls = rng.integers(0, 8, n).astype(np.float32)
        held = bi[q][bi[q] >= 0]
        if held.size:                                               # ids the beam holds
            pick = rng.choice(held.size, min(12, held.size), replace=False)
            base = bs[q][bi[q] >= 0][pick]
            li = np.concatenate([li, held[pick]])
            ls = np.concatenate([ls, base + rng.choice([-1.0, 0.0, 1.0], pick.size).astype(np.float32)])
        li[rng.random(li.size) < 0.1] = -1                          # padding ids
        lists_s.append(ls), lists_i.append(li)
    off = np.zeros(n_q + 1, np.int64)
    off[1:] = np.cumsum([len(x) for x in lists_i])
    cs, ci = np.concatenate(lists_s), np.concatenate(lists_i).astype(np.int32)
    beam = gem.Beam(n_q, ef, DEV)
    beam.scores.copy_(torch.from_numpy(bs))
    beam.ids.copy_(torch.from_numpy(bi))
    gem.beam_merge(torch.from_numpy(cs).to(DEV), gem.Cands(torch.from_numpy(ci).to(DEV),
                                                            torch.from_numpy(off).to(DEV)), beam)
    torch.cuda.synchronize()
    rs, ri = oracle.beam_merge(bs, bi, cs, off, ci, ef)
    np.testing.assert_array_equal(_np(beam.ids), ri)
    np.testing.assert_array_equal(_np(beam.scores), rs.astype(np.float32))


def test_expand_batch_matches_oracle():
    w = wl.WORKLOADS[4]
    c = wl.corpus(w, n_docs=3000)
    q = wl.queries(w, n_queries=20)
    D8, Q = _device_sets(c, "fp8"), gem.Sets.from_batch(q, DEV)
    Q8 = Q.to_fp8()
    ef = 100
    beam = gem.Beam(Q.n_sets, ef, DEV)
    qo, do = _operands(q.vecs.numpy(), "fp8"), _operands(c.vecs.numpy(), "fp8")
    steps = []
    for st in range(4):
        off, ids = wl.step_candidates(w, st, n_queries=20, n_docs=3000)
        C = gem.Cands(ids.to(DEV), off.to(DEV), max_list_len=w.cands_per_step)
        cs = torch.empty(ids.numel(), device=DEV)
        gem.expand_batch(Q8 if st % 2 else Q, D8, C, beam, cand_scores=cs)
        ref = oracle.ch_cands(qo, q.offsets.numpy(), do, c.offsets.numpy(), off.numpy(), ids.numpy())
        steps.append((ref, off.numpy(), ids.numpy()))
        torch.cuda.synchronize()
        assert_close(_np(cs), ref, what="expand scores")
    rs, ri = oracle.beam_replay(Q.n_sets, ef, steps)
    bs, bi = _np(beam.scores), _np(beam.ids)
    assert_close(bs, rs, what="beam scores")
    # beam membership agrees outside the tie band at the ef-th score
    all_ids = np.concatenate([s[2].reshape(20, -1) for s in steps], axis=1)
    all_sc = np.concatenate([s[0].reshape(20, -1) for s in steps], axis=1)
    for r in range(Q.n_sets):
        u, first = np.unique(all_ids[r], return_index=True)
        exact = np.full(3000, -np.inf)
        exact[u] = all_sc[r][first]
        tau = 2 * TOL * max(abs(rs[r][ef - 1]), 1.0)
        ok, bad, missing = oracle.tie_aware_match(bi[r], exact, ef, tau)
        assert ok, (r, bad, missing)


def test_error_paths_enqueue_nothing():
    q = gem.Sets.from_batch(_ragged([3], 50), DEV)
    c = gem.Sets.from_batch(_ragged([3, 4], 51), DEV)
    with pytest.raises(gem.GemError) as e:
        gem.score_exact(q, c.to_bf16(), compute="f32")            # D dtype != compute
    assert e.value.status == gem._abi.GEM_ERR_INVALID
    with pytest.raises(gem.GemError) as e:
        gem.score_exact(q, c, k=4096)                              # k > GEM_MAX_K
    assert e.value.status == gem._abi.GEM_ERR_INVALID
    big = gem.Sets.from_batch(_ragged([300], 52), DEV)
    with pytest.raises(gem.GemError) as e:
        gem.score_exact(big, c)                                    # query longer than 256
    assert e.value.status == gem._abi.GEM_ERR_UNSUPPORTED
    # a workspace smaller than gem_workspace_bytes() is refused
    import ctypes
    lib = gem.library()
    qs, ds = q.struct(), c.to_bf16().struct()
    ts = torch.empty(1, 1, device=DEV)
    ti = torch.empty(1, 1, dtype=torch.int32, device=DEV)
    need = lib.gem_workspace_bytes(gem._ctx(q.device), 0, ctypes.byref(qs), ctypes.byref(ds), None, 1, 1, 0)
    assert need > 0
    ws = torch.empty(need - 1, dtype=torch.uint8, device=DEV)
    st = lib.gem_score_exact(gem._ctx(q.device), ctypes.byref(qs), ctypes.byref(ds), None, 1, 1, None, 0, None,
                             ts.data_ptr(), ti.data_ptr(), ws.data_ptr(), need - 1, None)
    assert st == gem._abi.GEM_ERR_WORKSPACE
    bad_off = gem.Sets(c.vecs, torch.tensor([0, 5, 3], dtype=torch.int64, device=DEV), "f32", 5)
    with pytest.raises(gem.GemError) as e:
        gem.validate_sets(bad_off)
    assert e.value.status == gem._abi.GEM_ERR_DEVICE_CHECK
    gem.validate_sets(c)


def test_expansion_graph_replays_equal_eager():
    """A graph of several expansion steps gives bitwise the eager result on every replay."""
    from paper_2603_20336_amd.search import ExpansionGraph
    w = wl.WORKLOADS[4]
    c = wl.corpus(w, n_docs=4000)
    q = wl.queries(w, n_queries=48)
    D8 = _device_sets(c, "fp8")
    Q8 = gem.Sets.from_batch(q, DEV).to_fp8()
    steps = []
    for st in range(5):
        off, ids = wl.step_candidates(w, st, n_queries=48, n_docs=4000)
        steps.append(gem.Cands(ids.to(DEV), off.to(DEV), max_list_len=w.cands_per_step))
    eg = ExpansionGraph(Q8, D8, steps, ef=300)
    eg.run_eager()
    torch.cuda.synchronize()
    ref_s, ref_i = eg.beam.scores.clone(), eg.beam.ids.clone()
    eg.capture()
    for rep in range(3):
        eg.beam.scores.fill_(123.0)                  # eager work between replays
        torch.cuda.synchronize()
        eg.replay()
        torch.cuda.synchronize()
        assert torch.equal(eg.beam.ids, ref_i), rep
        assert torch.equal(eg.beam.scores, ref_s), rep
    side = torch.cuda.Stream(device=DEV)                # a replay ordered on a side stream
    eg.beam.scores.fill_(123.0)
    side.wait_stream(torch.cuda.current_stream(DEV))
    eg.replay(stream=side)
    torch.cuda.current_stream(DEV).wait_stream(side)
    assert torch.equal(eg.beam.ids, ref_i) and torch.equal(eg.beam.scores, ref_s)


# --------------------------------------------- gathered scorer at its full split
def _sampled_lists_ref(q_ops, q_off, d_ops, d_off, off, ids, rows):
    """Oracle scores of the listed queries' candidate entries, CSR over `rows`."""
    so = _csr([int(off[r + 1] - off[r]) for r in rows])
    si = np.concatenate([ids[off[r]:off[r + 1]] for r in rows])
    qsel = np.concatenate([np.arange(q_off[r], q_off[r + 1]) for r in rows])
    qo = _csr([int(q_off[r + 1] - q_off[r]) for r in rows])
    return oracle.ch_cands(q_ops[qsel], qo, d_ops, d_off, so, si), so, si


def test_expand_batch_full_split_matches_oracle():
    """Beam expansion in its full-size launch shape: 4096 queries x 512 ids a
    step, so that every wave of the gathered scorer takes 16 entries. 64
    sampled lists against the oracle, and their beams against its replay."""
    w = wl.WORKLOADS[4]
    n_docs, n_q, ef = 4000, 4096, 100
    c = wl.corpus(w, n_docs=n_docs)
    q = wl.queries(w, n_queries=n_q)
    D8 = _device_sets(c, "fp8")
    Q8 = gem.Sets.from_batch(q, DEV).to_fp8()
    beam = gem.Beam(n_q, ef, DEV)
    rows = sorted(set(np.random.default_rng(21).integers(0, n_q, 61).tolist()) | {0, 1, n_q - 1})
    qo_all = q.offsets.numpy()
    q_ops = _operands(q.vecs.numpy(), "fp8")
    d_ops = _operands(c.vecs.numpy(), "fp8")
    steps = []
    for st in range(2):
        off, ids = wl.step_candidates(w, st, n_queries=n_q, n_docs=n_docs)
        C = gem.Cands(ids.to(DEV), off.to(DEV), max_list_len=w.cands_per_step)
        assert C.n_lists * C.max_list_len >= 16 * 4096              # the 16-entries-per-wave split
        cs = torch.empty(ids.numel(), device=DEV)
        gem.expand_batch(Q8, D8, C, beam, cand_scores=cs)
        torch.cuda.synchronize()
        ref, so, si = _sampled_lists_ref(q_ops, qo_all, d_ops, c.offsets.numpy(), off.numpy(), ids.numpy(), rows)
        got = np.concatenate([_np(cs[int(off[r]):int(off[r + 1])]) for r in rows])
        assert_close(got, ref, what=f"full-split expansion step {st}")
        steps.append((ref, so, si))
    rs, ri = oracle.beam_replay(len(rows), ef, steps)
    bs, bi = _np(beam.scores)[rows], _np(beam.ids)[rows]
    assert_close(bs, rs, what="full-split beam scores")
    for j in range(len(rows)):
        exact = np.full(n_docs, -np.inf)
        for (sc_, so_, si_) in steps:
            seg = slice(so_[j], so_[j + 1])
            exact[si_[seg]] = sc_[seg]
        tau = 2 * TOL * max(abs(rs[j][ef - 1]), 1.0)
        ok, bad, missing = oracle.tie_aware_match(bi[j], exact, ef, tau)
        assert ok, (rows[j], bad, missing)


@pytest.mark.parametrize("fmt", ["fp8", "mxfp4"])
def test_expand_batch_sorted_lists_match_the_query_order(fmt):
    """Steps large enough for the sorted, chunk-major walk (n_lists x longest
    list >= 65,536): ragged CSR lists (empty ones, padding ids, repeated ids,
    lengths up to 700) give bitwise the per-query scorer's entry scores, in
    the caller's order, and the same beam as merging those scores."""
    rng = np.random.default_rng(33)
    n_docs, n_q, ef = 3000, 200, 64
    c = _ragged(list(rng.integers(1, 120, n_docs)), 34)
    q = _ragged(list(rng.integers(1, 65, n_q)), 35)
    S = gem.Sets.from_batch(c, DEV)
    D = S.to_fp8() if fmt == "fp8" else S.to_mxfp4()
    Qf = gem.Sets.from_batch(q, DEV)
    Qx = Qf.to_fp8() if fmt == "fp8" else Qf.to_mxfp4()
    lens = rng.integers(0, 701, n_q)
    lens[[3, 9]] = 0
    lens[0] = 700
    lists = [rng.integers(0, n_docs, int(m)) for m in lens]
    for ids in lists[10:20]:
        ids[rng.random(ids.size) < 0.1] = -1
        if ids.size > 4:
            ids[:3] = ids[3]
    off = _csr(lens)
    ids = np.concatenate(lists).astype(np.int32)
    C = gem.Cands(torch.from_numpy(ids).to(DEV), torch.from_numpy(off).to(DEV), max_list_len=700)
    assert C.n_lists * C.max_list_len >= 65536
    beam, beam_ref = gem.Beam(n_q, ef, DEV), gem.Beam(n_q, ef, DEV)
    cs = torch.full((ids.size,), 7.0, device=DEV)
    gem.expand_batch(Qx, D, C, beam, cand_scores=cs)
    gem.set_gather_order("query")
    try:
        ref = gem.score_quant(Qx, D, cands=C)
    finally:
        gem.set_gather_order("auto")
    gem.beam_merge(ref, C, beam_ref)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_np(cs).view(np.int32), _np(ref).view(np.int32))
    assert np.all(np.isneginf(_np(cs)[ids < 0]))
    assert torch.equal(beam.ids, beam_ref.ids) and torch.equal(beam.scores, beam_ref.scores)


def test_expansion_graph_sorted_lists_replay_equal_eager():
    """The sorted walk's sort kernel inside a captured step graph: replays,
    with eager work between them, reproduce the eager beams exactly."""
    from paper_2603_20336_amd.search import ExpansionGraph
    w = wl.WORKLOADS[4]
    n_q = 256
    c = wl.corpus(w, n_docs=4000)
    q = wl.queries(w, n_queries=n_q)
    D8 = _device_sets(c, "fp8")
    Q8 = gem.Sets.from_batch(q, DEV).to_fp8()
    steps = []
    for st in range(4):
        off, ids = wl.step_candidates(w, st, n_queries=n_q, n_docs=4000)
        steps.append(gem.Cands(ids.to(DEV), off.to(DEV), max_list_len=w.cands_per_step))
    assert n_q * w.cands_per_step >= 65536
    eg = ExpansionGraph(Q8, D8, steps, ef=200)
    eg.run_eager()
    torch.cuda.synchronize()
    ref_s, ref_i = eg.beam.scores.clone(), eg.beam.ids.clone()
    eg.capture()
    for rep in range(3):
        eg.beam.scores.fill_(123.0)
        torch.cuda.synchronize()
        eg.replay()
        torch.cuda.synchronize()
        assert torch.equal(eg.beam.ids, ref_i), rep
        assert torch.equal(eg.beam.scores, ref_s), rep


@pytest.mark.parametrize("order", ["auto", "query"])
def test_rerank_f32_full_split_matches_oracle_and_dense(order):
    """The float32 rerank in its full-size shape (1000 queries x 1000
    candidates): sampled lists against the oracle and bitwise against the
    dense float32 scorer, in the auto order (here every document is listed
    about 166 times: the document-major scorer) and in the query order (16
    entries per wave, the lists sorted by document id and walked
    chunk-major)."""
    gem.set_gather_order(order)
    try:
        _rerank_f32_full_split()
    finally:
        gem.set_gather_order("auto")


def _rerank_f32_full_split():
    w2 = wl.WORKLOADS[2]
    n_docs, n_q, sl = 6000, 1000, 1000
    c = wl.corpus(w2, n_docs=n_docs)
    q = wl.queries(w2, n_queries=n_q)
    rng = np.random.default_rng(22)
    ids = np.argsort(rng.random((n_q, n_docs)), axis=1)[:, :sl].astype(np.int32)
    D, Q = gem.Sets.from_batch(c, DEV), gem.Sets.from_batch(q, DEV)
    C = gem.Cands(torch.from_numpy(ids.reshape(-1)).to(DEV), stride=sl)
    assert C.n_lists * C.max_list_len >= 16 * 4096
    got = _np(gem.score_exact(Q, D, cands=C, compute="f32")).reshape(n_q, sl)
    dense = _np(gem.score_exact(Q, D, compute="f32"))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got, np.take_along_axis(dense, ids.astype(np.int64), axis=1))
    rows = [0, 1, 2, 499, 998, 999] + sorted(rng.integers(3, 998, 10).tolist())
    off = np.arange(0, (n_q + 1) * sl, sl, dtype=np.int64)
    ref, _, _ = _sampled_lists_ref(q.vecs.numpy().astype(np.float64), q.offsets.numpy(), c.vecs.numpy(),
                                   c.offsets.numpy(), off, ids.reshape(-1), rows)
    assert_close(got[rows].reshape(-1), ref, what="full-split f32 rerank")


def test_streamed_fp8_query_full_split():
    """One FP8 query streamed over 70,000 short documents (range mode, 16
    documents a wave), written through a row map and row stride: bitwise the
    dense scorer's row for the same query, and the oracle on sampled documents."""
    rng = np.random.default_rng(23)
    n_docs = 70000
    c = _ragged(list(rng.integers(0, 9, n_docs)), 70)
    q = _ragged([37, 5, 64, 12], 71)
    D8 = _device_sets(c, "fp8")
    Q = gem.Sets.from_batch(q, DEV)
    ld = n_docs + 13
    out = torch.full((3, ld), 7.0, device=DEV)
    rows = torch.tensor([2], dtype=torch.int32, device=DEV)
    gem.score_quant(Q.view(0, 1), D8, scores=out, ld=ld, rows=rows)
    dense = _np(gem.score_quant(Q, D8))                                # four queries: the dense scorer
    torch.cuda.synchronize()
    o = _np(out)
    np.testing.assert_array_equal(o[2, :n_docs], dense[0])
    assert (o[2, n_docs:] == 7.0).all() and (o[:2] == 7.0).all()
    ds = sorted(set(rng.integers(0, n_docs, 300).tolist()) | {0, 15, 16, 17, n_docs - 1})
    sq, sd = _sub_host(q, [0]), _sub_host(c, ds)
    ref = oracle.ch_dense(_operands(sq.vecs.numpy(), "fp8"), sq.offsets.numpy(),
                          _operands(sd.vecs.numpy(), "fp8"), sd.offsets.numpy())
    assert_close(o[2, ds][None], ref, what="streamed fp8 full split")
