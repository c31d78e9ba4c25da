"""The autotuner: every gathered-scorer schedule computes bitwise the same
scores, the gather tuner installs one of them for the call's shape class, and
a saved tune cache reinstalls the same dense and gathered schedules in a new
context (gem_create with the cache path) and through gem_load_tune_cache."""
import ctypes
import json

import numpy as np
import pytest
import torch

import oracle
import paper_2603_20336_amd as gem
from paper_2603_20336_amd import _abi
from paper_2603_20336_amd import workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda"
DEPTHS = {"f32": (1, 2, 3), "bf16": (2, 4, 6), "fp8": (4, 6, 8), "mxfp4": (6, 8, 12)}


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


def _score(Q, D, dtype, **kw):
    if dtype in ("fp8", "mxfp4"):
        return gem.score_quant(Q, D, **kw)
    return gem.score_exact(Q, D, compute=dtype, **kw)


def _problem(seed, n_q=40, n_docs=3000, per=300):
    rng = np.random.default_rng(seed)
    q = _ragged([int(x) for x in rng.integers(1, 65, n_q)], seed)
    c = _ragged([int(x) for x in rng.integers(0, 90, n_docs)], seed + 1)
    lists = [rng.integers(-1, n_docs, int(rng.integers(0, per))) for _ in range(n_q)]
    co = _csr([len(x) for x in lists])
    ci = np.concatenate(lists).astype(np.int32)
    C = gem.Cands(torch.from_numpy(ci).to(DEV), torch.from_numpy(co).to(DEV))
    return q, c, C, co, ci


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8", "mxfp4"])
def test_gather_schedules_bitwise(dtype):
    q, c, C, co, ci = _problem(50)
    Q, D = gem.Sets.from_batch(q, DEV), _dev(c, dtype)
    key = (dtype, C.n_lists, C.max_list_len)
    gem.set_gather_schedule(*key, None)
    base = _score(Q, D, dtype, cands=C).cpu().numpy()
    if dtype in ("f32", "bf16"):
        ref = oracle.ch_cands(q.vecs.numpy() if dtype == "f32" else
                              oracle.bf16_decode(oracle.bf16_round_bits(q.vecs.numpy())), q.offsets.numpy(),
                              c.vecs.numpy() if dtype == "f32" else
                              oracle.bf16_decode(oracle.bf16_round_bits(c.vecs.numpy())), c.offsets.numpy(),
                              co, np.maximum(ci, 0))
        ref[ci < 0] = -np.inf
        fin = np.isfinite(ref)
        assert np.array_equal(np.isfinite(base), fin)
        assert (np.abs(base[fin] - ref[fin]) / np.maximum(np.abs(ref[fin]), 1)).max() < 3e-4
    try:
        for e in (0, 1, 8, 16, 32, 64):
            for d in DEPTHS[dtype]:
                gem.set_gather_schedule(*key, {"entries_per_wave": e, "depth": d})
                got = _score(Q, D, dtype, cands=C).cpu().numpy()
                np.testing.assert_array_equal(got, base, err_msg=f"{dtype} entries {e} depth {d}")
        with pytest.raises(gem.GemError):
            gem.set_gather_schedule(*key, {"entries_per_wave": 65, "depth": DEPTHS[dtype][0]})
        with pytest.raises(gem.GemError):
            gem.set_gather_schedule(*key, {"entries_per_wave": 8, "depth": 5})
        best, ms = gem.autotune_gather(Q, D, C, reps=1)
        assert ms > 0 and best["depth"] in DEPTHS[dtype] and best["entries_per_wave"] in (0, 8, 16, 32, 64)
        assert gem.gather_schedule(*key) == best
        np.testing.assert_array_equal(_score(Q, D, dtype, cands=C).cpu().numpy(), base)
    finally:
        gem.set_gather_schedule(*key, None)


def test_tune_cache_round_trip(tmp_path):
    q, c, C, co, ci = _problem(51)
    Q, D8 = gem.Sets.from_batch(q, DEV), _dev(c, "fp8")
    dense_key = ("fp8", Q.n_vecs, D8.n_sets)
    gather_key = ("fp8", C.n_lists, C.max_list_len)
    try:
        dbest, _ = gem.autotune_dense(Q.to_fp8(), D8, reps=1)
        gem.set_gather_schedule(*gather_key, {"entries_per_wave": 32, "depth": 4})
        path = str(tmp_path / "tune.json")
        gem.save_tune_cache(path)
        doc = json.load(open(path))
        assert doc["format"] == "gem-tune-cache"
        kinds = {(e["kind"], e["dtype"]) for e in doc["entries"]}
        assert ("dense", _abi.GEM_FP8_E4M3) in kinds and ("gather", _abi.GEM_FP8_E4M3) in kinds
        # a new context created from the cache has the same schedules
        lib = gem.library()
        h = ctypes.c_void_p()
        _abi.check(lib.gem_create(ctypes.byref(h), torch.cuda.current_device(), path.encode()))
        try:
            ds = _abi.gem_dense_schedule()
            _abi.check(lib.gem_get_dense_schedule(h, _abi.GEM_FP8_E4M3, Q.n_vecs, D8.n_sets, ctypes.byref(ds)))
            assert (ds.chunk_docs, ds.items_per_slot, ds.slots_per_xcd) == \
                (dbest["chunk_docs"], dbest["items_per_slot"], dbest["slots_per_xcd"])
            gs = _abi.gem_gather_schedule()
            _abi.check(lib.gem_get_gather_schedule(h, _abi.GEM_FP8_E4M3, C.n_lists, C.max_list_len, ctypes.byref(gs)))
            assert (gs.entries_per_wave, gs.depth) == (32, 4)
        finally:
            lib.gem_destroy(h)
        # clearing and loading into this context reinstalls them
        gem.set_dense_schedule(*dense_key, None)
        gem.set_gather_schedule(*gather_key, None)
        gem.load_tune_cache(path)
        assert gem.dense_schedule(*dense_key) == dbest
        assert gem.gather_schedule(*gather_key) == {"entries_per_wave": 32, "depth": 4}
        # a missing cache is an empty one for gem_create, an error for gem_load_tune_cache;
        # a malformed one fails both and installs nothing
        h2 = ctypes.c_void_p()
        _abi.check(lib.gem_create(ctypes.byref(h2), torch.cuda.current_device(), str(tmp_path / "none.json").encode()))
        lib.gem_destroy(h2)
        with pytest.raises(gem.GemError):
            gem.load_tune_cache(str(tmp_path / "none.json"))
        bad = tmp_path / "bad.json"
        bad.write_text('{"format": "gem-tune-cache", "version": 1, "entries": [{"arch": "%s", "kind": "dense", '
                       '"dtype": 2, "q_rows_class": 3, "n_docs_class": 4, "chunk_docs": 48, "items_per_slot": 8, '
                       '"slots_per_xcd": 32}]}' % doc["entries"][0]["arch"])
        assert lib.gem_create(ctypes.byref(h2), torch.cuda.current_device(), str(bad).encode()) == _abi.GEM_ERR_INVALID
        with pytest.raises(gem.GemError):
            gem.load_tune_cache(str(bad))
        (tmp_path / "junk.json").write_text("[1, 2")
        with pytest.raises(gem.GemError):
            gem.load_tune_cache(str(tmp_path / "junk.json"))
    finally:
        gem.set_dense_schedule(*dense_key, None)
        gem.set_gather_schedule(*gather_key, None)
