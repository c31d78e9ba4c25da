"""Seeded synthetic workloads for set-to-set scoring.

This module only draws inputs: vector sets on the unit sphere from a Gaussian
mixture, ragged set lengths, candidate-id lists and request arrival times. It
holds none of the scoring arithmetic, so both the GPU path and the CPU oracle
can consume what it produces without sharing any of the method's code.

The paper evaluates on ColBERTv2 / preFLMR embeddings of MS MARCO, LoTTE,
OK-VQA and EVQA (Sec. 5.1, dataset table): d = 128 and 68-194 vectors per set.
Those corpora are not available, so the recipes below stand in for them with
the same dimension and set-size range.

Recipe (every workload):
  * centres  c_k = g / |g|, g ~ N(0, I_d)                       (seed 100 + i)
  * vectors  x = normalize(c_z + sigma * eps), z ~ U{0..K-1} i.i.d. per
    vector, eps ~ N(0, I_d), computed in float64 and stored as float32
  * corpus set lengths per workload (uniform or clipped lognormal) (seed 1000 + i)
  * queries from the same mixture                                (seed 2000 + i)
  * candidate ids: per (query, step) distinct ids uniform over the corpus
                                                                 (seed 3000 + 100 i + step)
  * request arrivals: Poisson process                            (seed 4000 + rate index)
where i is the workload number (1..5). Workloads 3 and 5 reuse workload 2's
corpus; workload 3 also reuses its queries.

Workload 6 (graph search) gives the sets topical structure, as passages of
real text have: the K centres form T topics of K / T centres each, a topic's
centres scattered around a topic direction (c = normalize(g_t + 0.5 eps /
sqrt(d)), so that two centres of one topic have an inner product near 0.8);
every set picks a topic and draws each vector's centre from it with
probability 0.8, else from all K centres. T = 64 topics of 64 centres, so
that a topic holds about 1,500 sets, the cluster size the paper aims its
coarse clusters at (Sec. 5.1). Centres seed 600, topics and vectors seed 1006
(corpus) and 2006 (queries).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import torch

DIM = 128


@dataclasses.dataclass
class SetBatch:
    """A ragged batch of vector sets in CSR form (float32 rows, int64 offsets)."""

    vecs: torch.Tensor      # [n_vecs, dim] float32
    offsets: torch.Tensor   # [n_sets + 1] int64, offsets[0] = 0, non-decreasing

    @property
    def n_sets(self) -> int:
        return int(self.offsets.numel() - 1)

    @property
    def n_vecs(self) -> int:
        return int(self.vecs.shape[0])

    def lengths(self) -> torch.Tensor:
        return self.offsets[1:] - self.offsets[:-1]

    def max_len(self) -> int:
        if self.n_sets == 0:
            return 0
        return int(self.lengths().max().item())

    def to(self, device) -> "SetBatch":
        return SetBatch(self.vecs.to(device), self.offsets.to(device))

    def subset(self, idx) -> "SetBatch":
        """Sets `idx` (a sequence of set indices) packed into a new CSR batch."""
        off = self.offsets.cpu()
        rows, lens = [], []
        for i in idx:
            a, b = int(off[i]), int(off[i + 1])
            rows.append(self.vecs[a:b])
            lens.append(b - a)
        o = torch.zeros(len(lens) + 1, dtype=torch.int64)
        if lens:
            o[1:] = torch.cumsum(torch.tensor(lens, dtype=torch.int64), 0)
        v = torch.cat(rows, 0) if rows else self.vecs[:0]
        return SetBatch(v, o.to(self.vecs.device))


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload: corpus, queries and what is asked of them."""

    number: int
    name: str
    n_docs: int
    doc_len: tuple           # ("uniform", lo, hi) or ("lognormal", mean, ln_sigma, lo, hi)
    n_centers: int
    n_queries: int
    query_len: tuple         # ("fixed", m) or ("uniform", lo, hi)
    k: int
    sigma: float = 0.1
    shortlist: int = 0       # estimate shortlist size before the exact rerank
    cands_per_step: int = 0  # candidate ids scored per query per expansion step
    steps: int = 0
    ef: int = 0
    corpus_of: int = 0       # workload number whose corpus (and seeds) is reused
    queries_of: int = 0      # workload number whose queries are reused


WORKLOADS = {
    1: Workload(1, "exact-2k", 2000, ("uniform", 8, 32), 64, 16, ("fixed", 32), 10),
    2: Workload(2, "exhaustive-100k", 100_000, ("lognormal", 80.0, 0.5, 32, 256), 4096,
                1000, ("fixed", 32), 100),
    3: Workload(3, "fp8-rerank-100k", 100_000, ("lognormal", 80.0, 0.5, 32, 256), 4096,
                1000, ("fixed", 32), 100, shortlist=1000, corpus_of=2, queries_of=2),
    4: Workload(4, "beam-expand-1m", 1_000_000, ("uniform", 16, 128), 4096,
                4096, ("uniform", 8, 64), 0, cands_per_step=512, steps=20, ef=1000),
    # serving reranks an FP8 shortlist of 200: on its query mix (4 to 64
    # vectors) recall@100 after the float32 rerank is 0.99999 at 200 (one
    # miss in 100,000 results) and 1.0 from 300 on; 200 takes a third less
    # rerank work than 300
    5: Workload(5, "serving-100k", 100_000, ("lognormal", 80.0, 0.5, 32, 256), 4096,
                0, ("uniform", 4, 64), 100, shortlist=200, corpus_of=2),
    6: Workload(6, "graph-search-100k-topical", 100_000, ("lognormal", 80.0, 0.5, 32, 256), 4096,
                1000, ("fixed", 32), 10),
}

# topical structure of workload 6
TOPICS = 64
TOPIC_SPREAD = 0.5
P_TOPIC = 0.8


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return g


def mixture_centers(n_centers: int, seed: int, device="cpu", dim: int = DIM) -> torch.Tensor:
    """Centres uniform on the unit sphere (float64)."""
    g = _gen(seed, device)
    c = torch.randn(n_centers, dim, generator=g, dtype=torch.float64, device=device)
    return c / c.norm(dim=1, keepdim=True)


def mixture_vectors(n: int, centers: torch.Tensor, sigma: float, gen: torch.Generator,
                    chunk: int = 1 << 21) -> torch.Tensor:
    """n unit vectors: a random centre plus isotropic noise, renormalised (float32)."""
    device = centers.device
    K, dim = centers.shape
    out = torch.empty(n, dim, dtype=torch.float32, device=device)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        z = torch.randint(0, K, (b - a,), generator=gen, device=device)
        eps = torch.randn(b - a, dim, generator=gen, dtype=torch.float64, device=device)
        x = centers[z] + sigma * eps
        x = x / x.norm(dim=1, keepdim=True)
        out[a:b] = x.to(torch.float32)
    return out


def set_lengths(n: int, spec: tuple, gen: torch.Generator, device="cpu") -> torch.Tensor:
    kind = spec[0]
    if kind == "fixed":
        return torch.full((n,), int(spec[1]), dtype=torch.int64, device=device)
    if kind == "uniform":
        lo, hi = int(spec[1]), int(spec[2])
        return torch.randint(lo, hi + 1, (n,), generator=gen, device=device, dtype=torch.int64)
    if kind == "lognormal":
        mean, ln_sigma, lo, hi = float(spec[1]), float(spec[2]), int(spec[3]), int(spec[4])
        mu = math.log(mean) - ln_sigma * ln_sigma / 2.0
        x = torch.empty(n, dtype=torch.float64, device=device)
        x.log_normal_(mean=mu, std=ln_sigma, generator=gen)
        return torch.clamp(torch.round(x), lo, hi).to(torch.int64)
    raise ValueError(f"unknown length spec {spec!r}")


def _csr(lengths: torch.Tensor) -> torch.Tensor:
    o = torch.zeros(lengths.numel() + 1, dtype=torch.int64, device=lengths.device)
    o[1:] = torch.cumsum(lengths, 0)
    return o


def make_sets(n_sets: int, len_spec: tuple, centers: torch.Tensor, sigma: float, seed: int) -> SetBatch:
    device = centers.device
    g = _gen(seed, device)
    lens = set_lengths(n_sets, len_spec, g, device)
    off = _csr(lens)
    vecs = mixture_vectors(int(off[-1].item()), centers, sigma, g)
    return SetBatch(vecs, off)


def topical_centers(n_centers: int, n_topics: int, spread: float, seed: int, device="cpu", dim: int = DIM):
    """Centres grouped into topics: centre k belongs to topic k // (K / T) and is
    normalize(g_t + spread * eps / sqrt(d)) for the topic's direction g_t (float64)."""
    g = _gen(seed, device)
    dirs = torch.randn(n_topics, dim, generator=g, dtype=torch.float64, device=device)
    dirs = dirs / dirs.norm(dim=1, keepdim=True)
    per = n_centers // n_topics
    eps = torch.randn(n_topics * per, dim, generator=g, dtype=torch.float64, device=device)
    c = dirs.repeat_interleave(per, 0) + (spread / math.sqrt(dim)) * eps
    return c / c.norm(dim=1, keepdim=True)


def topical_sets(n_sets: int, len_spec: tuple, centers: torch.Tensor, n_topics: int, p_topic: float, sigma: float,
                 seed: int) -> SetBatch:
    """Sets whose vectors come from their topic's centres with probability p_topic."""
    device = centers.device
    K, dim = centers.shape
    per = K // n_topics
    g = _gen(seed, device)
    lens = set_lengths(n_sets, len_spec, g, device)
    off = _csr(lens)
    n = int(off[-1].item())
    topic = torch.randint(0, n_topics, (n_sets,), generator=g, device=device)
    owner = torch.repeat_interleave(torch.arange(n_sets, device=device), lens)
    in_topic = torch.rand(n, generator=g, device=device, dtype=torch.float64) < p_topic
    z_topic = topic[owner] * per + torch.randint(0, per, (n,), generator=g, device=device)
    z_any = torch.randint(0, K, (n,), generator=g, device=device)
    z = torch.where(in_topic, z_topic, z_any)
    out = torch.empty(n, dim, dtype=torch.float32, device=device)
    chunk = 1 << 21
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        eps = torch.randn(b - a, dim, generator=g, dtype=torch.float64, device=device)
        x = centers[z[a:b]] + sigma * eps
        out[a:b] = (x / x.norm(dim=1, keepdim=True)).to(torch.float32)
    return SetBatch(out, off)


def corpus(w: Workload, device="cpu", n_docs: Optional[int] = None) -> SetBatch:
    """The workload's document corpus (n_docs overrides the size for small tests)."""
    src = WORKLOADS[w.corpus_of] if w.corpus_of else w
    i = src.number
    n = n_docs if n_docs is not None else src.n_docs
    if i == 6:
        centers = topical_centers(src.n_centers, TOPICS, TOPIC_SPREAD, 600, device)
        return topical_sets(n, src.doc_len, centers, TOPICS, P_TOPIC, src.sigma, 1000 + i)
    centers = mixture_centers(src.n_centers, 100 + i, device)
    return make_sets(n, src.doc_len, centers, src.sigma, 1000 + i)


def queries(w: Workload, device="cpu", n_queries: Optional[int] = None,
            query_len: Optional[tuple] = None, seed_offset: int = 0) -> SetBatch:
    """The workload's query sets, drawn from the corpus's mixture (seed_offset:
    another draw from the same distribution, e.g. tuning samples kept apart
    from the measured queries)."""
    src = WORKLOADS[w.corpus_of] if w.corpus_of else w
    qsrc = WORKLOADS[w.queries_of] if w.queries_of else w
    n = n_queries if n_queries is not None else qsrc.n_queries
    if src.number == 6:
        centers = topical_centers(src.n_centers, TOPICS, TOPIC_SPREAD, 600, device)
        return topical_sets(n, query_len or qsrc.query_len, centers, TOPICS, P_TOPIC, src.sigma,
                            2000 + qsrc.number + seed_offset)
    centers = mixture_centers(src.n_centers, 100 + src.number, device)
    return make_sets(n, query_len or qsrc.query_len, centers, src.sigma, 2000 + qsrc.number + seed_offset)


def candidate_ids(n_queries: int, per_query: int, n_docs: int, seed: int, device="cpu",
                  extra: int = 16) -> torch.Tensor:
    """[n_queries, per_query] int32: distinct ids per row, uniform over [0, n_docs).

    Draw with replacement, keep the first occurrence of each id in draw order and
    take the first `per_query` survivors.
    """
    if per_query > n_docs:
        raise ValueError("per_query exceeds the number of documents")
    g = _gen(seed, device)
    while True:
        m = per_query + extra
        draw = torch.randint(0, n_docs, (n_queries, m), generator=g, device=device, dtype=torch.int64)
        srt, perm = torch.sort(draw, dim=1, stable=True)
        dup_sorted = torch.zeros_like(srt, dtype=torch.bool)
        dup_sorted[:, 1:] = srt[:, 1:] == srt[:, :-1]
        dup = torch.zeros_like(dup_sorted)
        dup.scatter_(1, perm, dup_sorted)
        keep = ~dup
        rank = torch.cumsum(keep.to(torch.int64), 1)
        take = keep & (rank <= per_query)
        if bool((take.sum(1) == per_query).all()):
            return draw[take].view(n_queries, per_query).to(torch.int32)
        extra *= 2


def step_candidates(w: Workload, step: int, n_queries: Optional[int] = None, device="cpu",
                    n_docs: Optional[int] = None):
    """CSR candidate lists for one beam-expansion step: (offsets int64, ids int32)."""
    nq = n_queries if n_queries is not None else w.n_queries
    nd = n_docs if n_docs is not None else w.n_docs
    ids = candidate_ids(nq, w.cands_per_step, nd, 3000 + 100 * w.number + step, device)
    off = torch.arange(nq + 1, dtype=torch.int64, device=device) * w.cands_per_step
    return off, ids.reshape(-1)


def poisson_arrivals(rate: float, n: int, rate_index: int) -> torch.Tensor:
    """Arrival times (seconds, float64, increasing) of a Poisson process."""
    g = _gen(4000 + rate_index, "cpu")
    gaps = torch.empty(n, dtype=torch.float64)
    gaps.exponential_(rate, generator=g)
    return torch.cumsum(gaps, 0)


def random_scores(n_segs: int, seg_len_spec: tuple, seed: int, tie_frac: float = 0.0,
                  device="cpu"):
    """Synthetic score segments for top-k tests: (scores f32, offsets int64).

    A fraction `tie_frac` of each segment is snapped to a few repeated values so
    that equal scores (ties) occur.
    """
    g = _gen(seed, device)
    lens = set_lengths(n_segs, seg_len_spec, g, device)
    off = _csr(lens)
    n = int(off[-1].item())
    s = torch.randn(n, generator=g, device=device, dtype=torch.float32)
    if tie_frac > 0 and n > 0:
        pick = torch.rand(n, generator=g, device=device) < tie_frac
        vals = torch.tensor([0.5, 1.0, -0.25], dtype=torch.float32, device=device)
        which = torch.randint(0, 3, (n,), generator=g, device=device)
        s = torch.where(pick, vals[which], s)
    return s, off
