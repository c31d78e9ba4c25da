"""GPU parity of the MXFP6 estimate (E2M3 codes, one E8M0 scale per 32 dims)
against the float64 oracle: the quantizer bit for bit, and the dense and the
gathered scorer on the oracle's own decoded operands."""
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


def _csr(lengths):
    o = np.zeros(len(lengths) + 1, np.int64)
    o[1:] = np.cumsum(lengths)
    return o


def _ragged(lengths, seed):
    centers = wl.mixture_centers(8, seed)
    g = torch.Generator().manual_seed(seed + 1)
    vecs = wl.mixture_vectors(int(sum(lengths)), centers, 0.1, g)
    return wl.SetBatch(vecs, torch.from_numpy(_csr(lengths)))


def _pack6(codes):
    """Oracle codes [n, 128] -> the library's row layout: element t of a row in
    bits 6t .. 6t + 5 of its 96 bytes, least significant bit first (four codes
    fill three bytes; a 32-element block fills 24)."""
    c = np.asarray(codes, np.uint32).reshape(codes.shape[0], -1, 4)
    u = c[..., 0] | (c[..., 1] << 6) | (c[..., 2] << 12) | (c[..., 3] << 18)
    return np.stack([u & 0xFF, (u >> 8) & 0xFF, (u >> 16) & 0xFF], axis=-1).reshape(codes.shape[0], -1).astype(np.uint8)


def _mx_values(x):
    codes, exps = oracle.quantize_mxfp6(np.asarray(x, np.float32))
    return oracle.dequantize_mxfp6(codes, exps)


def assert_close(got, ref, what=""):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    assert np.array_equal(np.isinf(got), np.isinf(ref)), f"{what}: -inf pattern"
    fin = ~np.isinf(ref)
    rel = np.abs(got[fin] - ref[fin]) / np.maximum(np.abs(ref[fin]), 1.0)
    assert rel.max() <= TOL, f"{what}: max rel err {rel.max():.3e}"


def test_pack6_layout_pin():
    # a hand-checked row: codes 1, 2, 3, 4 -> bits 000001 000010 000011 000100
    codes = np.zeros((1, 128), np.uint8)
    codes[0, :4] = [1, 2, 3, 4]
    codes[0, 127] = 0x3F
    b = _pack6(codes)
    assert b.shape == (1, 96)
    assert list(b[0, :3]) == [0x81, 0x30, 0x10] and b[0, 95] == 0xFC and not b[0, 3:95].any()


def test_quantize_mxfp6_bitwise():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal((500, 128)) * 10.0 ** rng.integers(-6, 6, (500, 1))).astype(np.float32)
    grid = oracle.e2m3_table()[:32]
    mids = (grid[1:] + grid[:-1]) / 2
    x[0, :32] = mids[:31].tolist() + [7.5]               # block amax 7.5 -> scale 1: every midpoint is a tie
    x[0, 32:64] = (-mids[:31]).tolist() + [-7.5]
    x[0, 64:96] = 0.0                                    # all-zero block
    x[1, 64:96] = 1e-40                                  # subnormal block: clamped exponent
    x[2, :] = -0.0
    x[3, 96:] = 7.5 * 2.0 ** 20                          # exactly on the top of the grid
    x[4, :32] = grid * 2.0 ** -9                         # every magnitude once, scaled
    b = wl.SetBatch(torch.from_numpy(x), torch.tensor([0, x.shape[0]], dtype=torch.int64))
    S = gem.Sets.from_batch(b, DEV).to_mxfp6()
    codes, exps = oracle.quantize_mxfp6(x)
    np.testing.assert_array_equal(_np(S.scales).astype(np.int64), exps.astype(np.int64) + 127)
    np.testing.assert_array_equal(_np(S.vecs), _pack6(codes))


@pytest.mark.parametrize("case", ["workload1", "ragged"])
def test_mxfp6_dense_matches_oracle(case):
    if case == "workload1":
        w = wl.WORKLOADS[1]
        c, q = wl.corpus(w), wl.queries(w)
        k = w.k
    else:
        rng = np.random.default_rng(3)
        dl = rng.integers(1, 300, 150)
        dl[[4, 77]] = 0
        ql = rng.integers(1, 200, 21)
        ql[5] = 0
        c, q = _ragged(dl, 11), _ragged(ql, 12)
        k = 7
    D = gem.Sets.from_batch(c, DEV).to_mxfp6()
    Q = gem.Sets.from_batch(q, DEV)
    top_s, top_i, scores = gem.score_quant(Q, D, k=k, want_scores=True)
    ref = oracle.ch_dense(_mx_values(q.vecs.numpy()), q.offsets.numpy(), _mx_values(c.vecs.numpy()),
                          c.offsets.numpy())
    assert_close(_np(scores), ref, f"mxfp6 dense {case}")
    # queries handed over already quantized give the same bits
    _, _, again = gem.score_quant(Q.to_mxfp6(), D, k=k, want_scores=True)
    np.testing.assert_array_equal(_np(again), _np(scores))
    ts, ti = _np(top_s), _np(top_i)
    for r in range(Q.n_sets):
        kk = min(k, D.n_sets)
        tau = 2 * TOL * max(abs(np.sort(ref[r])[::-1][kk - 1]), 1.0)
        ok, bad, missing = oracle.tie_aware_match(ti[r][:kk], ref[r], kk, tau)
        assert ok, (case, r, bad, missing)
    # the top-k fused into the scorer equals the top-k of the staged rows
    try:
        gem.set_topk_fusion("fused")
        fs, fi = gem.score_quant(Q, D, k=k)
    finally:
        gem.set_topk_fusion("auto")
    ss, si = gem.topk(scores, k)
    np.testing.assert_array_equal(_np(fi), _np(si))
    np.testing.assert_array_equal(_np(fs), _np(ss))


def test_mxfp6_gather_equals_dense_and_expands():
    rng = np.random.default_rng(5)
    c, q = _ragged(rng.integers(1, 120, 400), 21), _ragged(rng.integers(1, 80, 30), 22)
    D = gem.Sets.from_batch(c, DEV).to_mxfp6()
    Q = gem.Sets.from_batch(q, DEV).to_mxfp6()
    _, _, dense = gem.score_quant(Q, D, k=5, want_scores=True)
    lens = rng.integers(0, 90, 30)
    co = _csr(lens)
    ids = rng.integers(0, 400, int(co[-1])).astype(np.int32)
    ids[::17] = -1
    cands = gem.Cands(torch.from_numpy(ids).to(DEV), torch.from_numpy(co).to(DEV))
    _, _, got = gem.score_quant(Q, D, cands=cands, k=5, want_scores=True)
    dn, gt = _np(dense), _np(got)
    for i in range(30):
        for e in range(co[i], co[i + 1]):
            want = -np.inf if ids[e] < 0 else dn[i, ids[e]]
            assert gt[e] == want
    # one expansion step on MXFP6 sets: the beam is the best of the scored entries
    beam = gem.Beam(30, 16, DEV)
    gem.expand_batch(Q, D, cands, beam)
    bs, bi = _np(beam.scores), _np(beam.ids)
    for i in range(30):
        seg = [(gt[e], ids[e]) for e in range(co[i], co[i + 1]) if ids[e] >= 0]
        best = {}
        for s_, d_ in seg:
            best[d_] = max(best.get(d_, -np.inf), s_)
        want = sorted(best.items(), key=lambda t: (-t[1], t[0]))[:16]
        got_i = [(int(d), float(s)) for s, d in zip(bs[i], bi[i]) if d >= 0]
        assert got_i == [(int(d), float(np.float32(s))) for d, s in want]


def test_mxfp6_code_sets_equal_materialized_rows():
    rng = np.random.default_rng(6)
    C = _ragged([200], 31).vecs.numpy()
    dl, ql = rng.integers(1, 60, 120), rng.integers(1, 40, 9)
    dc = rng.integers(0, 200, int(dl.sum())).astype(np.int32)
    qc = rng.integers(0, 200, int(ql.sum())).astype(np.int32)
    Ct = torch.from_numpy(C).to(DEV)
    D = gem.Sets(Ct, torch.from_numpy(_csr(dl)).to(DEV), "f32", 60, codes=torch.from_numpy(dc).to(DEV)).to_mxfp6()
    Q = gem.Sets(Ct, torch.from_numpy(_csr(ql)).to(DEV), "f32", 40, codes=torch.from_numpy(qc).to(DEV)).to_mxfp6()
    _, _, got = gem.score_quant(Q, D, k=3, want_scores=True)
    Dm = gem.Sets(D.vecs[D.codes.long()].contiguous(), D.offsets, "mxfp6", 60,
                  scales=D.scales[D.codes.long()].contiguous())
    Qm = gem.Sets(Q.vecs[Q.codes.long()].contiguous(), Q.offsets, "mxfp6", 40,
                  scales=Q.scales[Q.codes.long()].contiguous())
    _, _, want = gem.score_quant(Qm, Dm, k=3, want_scores=True)
    np.testing.assert_array_equal(_np(got), _np(want))
    ref = oracle.qch_dense(qc, _csr(ql), dc, _csr(dl), _mx_values(C))
    assert_close(_np(got), ref, "mxfp6 qCH")

