"""The seeded input generator: reproducible, and shaped as each workload states."""
import torch

from paper_2603_20336_amd import workloads as wl


def test_corpus_is_seeded_and_unit_norm():
    w = wl.WORKLOADS[1]
    a = wl.corpus(w)
    b = wl.corpus(w)
    assert torch.equal(a.vecs, b.vecs) and torch.equal(a.offsets, b.offsets)
    assert a.n_sets == 2000 and a.vecs.dtype == torch.float32 and a.vecs.shape[1] == 128
    lens = a.lengths()
    assert int(lens.min()) >= 8 and int(lens.max()) <= 32
    n = a.vecs.double().norm(dim=1)
    assert float((n - 1).abs().max()) < 1e-6
    q = wl.queries(w)
    assert q.n_sets == 16 and bool((q.lengths() == 32).all())


def test_lognormal_lengths_clip_and_mean():
    g = torch.Generator().manual_seed(0)
    lens = wl.set_lengths(200000, ("lognormal", 80.0, 0.5, 32, 256), g)
    assert int(lens.min()) >= 32 and int(lens.max()) <= 256
    assert abs(float(lens.double().mean()) - 80.0) < 1.5


def test_candidate_ids_distinct_per_row():
    ids = wl.candidate_ids(64, 512, 1000, seed=3)
    assert ids.shape == (64, 512) and ids.dtype == torch.int32
    for r in range(64):
        assert torch.unique(ids[r]).numel() == 512
    assert int(ids.min()) >= 0 and int(ids.max()) < 1000
    assert torch.equal(ids, wl.candidate_ids(64, 512, 1000, seed=3))


def test_subset_and_arrivals():
    c = wl.corpus(wl.WORKLOADS[1], n_docs=10)
    s = c.subset([3, 1])
    assert s.n_sets == 2
    assert torch.equal(s.vecs[: int(c.lengths()[3])], c.vecs[int(c.offsets[3]): int(c.offsets[4])])
    t = wl.poisson_arrivals(1000.0, 5000, 0)
    assert bool((t[1:] > t[:-1]).all())
    assert abs(float(t[-1]) / 5000 - 1e-3) < 1e-4
