"""gem_score_quant_static (no workspace argument: a static device scratch
array) against gem_score_quant with a caller-allocated workspace, through the
C ABI: two calls in a row, the second smaller, bitwise the same outputs, in
the staged and the fused top-k modes and for a dense score matrix; a call too
large for the scratch is refused with nothing enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2603_20336_amd as gem
from paper_2603_20336_amd import _abi
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


def _static(Q, D, k, scores=None, ld=0):
    lib = gem.library()
    qs, ds = Q.struct(), D.struct()
    ts = torch.full((Q.n_sets, max(k, 1)), 7.0, device=DEV)
    ti = torch.full((Q.n_sets, max(k, 1)), -7, dtype=torch.int32, device=DEV)
    st = lib.gem_score_quant_static(gem._ctx(D.device), ctypes.byref(qs), ctypes.byref(ds), None, int(k),
                                    None if scores is None else scores.data_ptr(), int(ld), None,
                                    ts.data_ptr() if k > 0 else None, ti.data_ptr() if k > 0 else None,
                                    torch.cuda.current_stream().cuda_stream)
    return st, ts, ti


@pytest.mark.parametrize("mode", ["staged", "fused"])
def test_static_scratch_matches_the_workspace_call(mode):
    gem.set_topk_fusion(mode)
    try:
        rng = np.random.default_rng(5)
        for nq, nd, k, seed in ((40, 20000, 100, 10), (9, 5000, 30, 20)):
            q = _ragged([int(x) for x in rng.integers(1, 65, nq)], seed)
            c = _ragged([int(x) for x in rng.integers(0, 50, nd)], seed + 1)
            Q, D8 = gem.Sets.from_batch(q, DEV), gem.Sets.from_batch(c, DEV).to_fp8()
            assert gem.score_workspace_bytes(Q, D8, k=k) <= _abi.GEM_STATIC_SCRATCH_BYTES
            ref_s, ref_i = gem.score_quant(Q, D8, k=k)
            st, ts, ti = _static(Q, D8, k)
            assert st == _abi.GEM_OK, gem.library().gem_last_error()
            torch.cuda.synchronize()
            assert torch.equal(ti, ref_i), (mode, nq, nd)
            assert torch.equal(ts.view(torch.int32), ref_s.view(torch.int32)), (mode, nq, nd)
    finally:
        gem.set_topk_fusion("auto")


def test_static_scratch_dense_scores():
    rng = np.random.default_rng(6)
    for nq, nd in ((12, 9000), (5, 3000)):
        q = _ragged([int(x) for x in rng.integers(1, 65, nq)], 30 + nd)
        c = _ragged([int(x) for x in rng.integers(0, 50, nd)], 31 + nd)
        Q, D8 = gem.Sets.from_batch(q, DEV), gem.Sets.from_batch(c, DEV).to_fp8()
        ref = gem.score_quant(Q, D8)
        out = torch.full((nq, nd), 7.0, device=DEV)
        st, _, _ = _static(Q, D8, 0, scores=out)
        assert st == _abi.GEM_OK, gem.library().gem_last_error()
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int32), ref.view(torch.int32))


def test_static_scratch_refuses_a_call_that_does_not_fit():
    gem.set_topk_fusion("staged")
    try:
        q = _ragged([32] * 200, 40)
        c = _ragged([1] * 100000, 41)
        Q, D8 = gem.Sets.from_batch(q, DEV), gem.Sets.from_batch(c, DEV).to_fp8()
        assert gem.score_workspace_bytes(Q, D8, k=10) > _abi.GEM_STATIC_SCRATCH_BYTES
        torch.cuda.synchronize()
        st, ts, ti = _static(Q, D8, 10)
        assert st == _abi.GEM_ERR_WORKSPACE
        assert b"static scratch" in gem.library().gem_last_error()
        torch.cuda.synchronize()
        assert (ts == 7.0).all() and (ti == -7).all()          # nothing was enqueued
    finally:
        gem.set_topk_fusion("auto")
