"""GEM_CHECK mode: calls validate their device inputs first and refuse bad
data with GEM_ERR_DEVICE_CHECK before computing anything; gem_check_status
reports the count once. The bad inputs used here stay inside their buffers
(ids past a view's end, non-finite values, a scale that is not a power of
two), so nothing could read out of bounds even unchecked."""
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


@pytest.fixture()
def checked():
    gem.set_check(True)
    gem.check_status()
    yield
    gem.set_check(False)
    gem.check_status()


def _status(fn):
    with pytest.raises(gem.GemError) as e:
        fn()
    return e.value.status


def test_good_calls_pass_and_match(checked):
    rng = np.random.default_rng(60)
    q = gem.Sets.from_batch(_ragged([int(x) for x in rng.integers(1, 40, 6)], 61), DEV)
    D = gem.Sets.from_batch(_ragged([int(x) for x in rng.integers(0, 30, 200)], 62), DEV)
    got = gem.score_exact(q, D, compute="f32")
    gem.set_check(False)
    ref = gem.score_exact(q, D, compute="f32")
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    gem.check_status()


def test_bad_device_data_is_refused_before_computing(checked):
    rng = np.random.default_rng(63)
    q = gem.Sets.from_batch(_ragged([int(x) for x in rng.integers(1, 40, 4)], 64), DEV)
    full = gem.Sets.from_batch(_ragged([int(x) for x in rng.integers(1, 30, 200)], 65), DEV)
    D = full.view(0, 100)                                      # ids 100..199 are past this batch's end
    ids = torch.tensor([3, 150, 7, 99, 120, 0], dtype=torch.int32, device=DEV)
    C = gem.Cands(ids, torch.tensor([0, 2, 3, 5, 6], dtype=torch.int64, device=DEV))
    out = torch.full((6,), 7.0, device=DEV)
    assert _status(lambda: gem.score_exact(q, D, cands=C, compute="f32", scores=out)) == _abi.GEM_ERR_DEVICE_CHECK
    torch.cuda.synchronize()
    assert (out == 7.0).all()                                  # nothing was computed
    # a non-finite float32 query value
    qv = q.vecs.clone()
    qv[5, 17] = float("nan")
    qn = gem.Sets(qv, q.offsets, "f32", q.max_len)
    assert _status(lambda: gem.score_exact(qn, D, compute="f32")) == _abi.GEM_ERR_DEVICE_CHECK
    # an FP8 scale that is not a power of two
    D8 = D.to_fp8()
    D8.scales[11] = 0.3
    assert _status(lambda: gem.score_quant(q, D8)) == _abi.GEM_ERR_DEVICE_CHECK
    # the violations are reported once, then cleared
    assert _status(lambda: gem.check_status()) == _abi.GEM_ERR_DEVICE_CHECK
    gem.check_status()


def test_check_mode_off_does_not_validate():
    gem.set_check(False)
    rng = np.random.default_rng(66)
    q = gem.Sets.from_batch(_ragged([int(x) for x in rng.integers(1, 40, 4)], 67), DEV)
    D = gem.Sets.from_batch(_ragged([int(x) for x in rng.integers(1, 30, 50)], 68), DEV)
    D8 = D.to_fp8()
    D8.scales[3] = 0.3                                         # unchecked: scored as given, no error
    gem.score_quant(q, D8)
    gem.check_status()
