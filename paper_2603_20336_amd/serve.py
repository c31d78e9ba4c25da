"""Serving loop for multi-vector queries: memory-admitted continuous batching.

The corpus stays resident on the device as FP8 codes (for the estimate) and
float32 rows (for the exact rerank). It is split into `n_chunks` document
chunks. Every iteration scores one chunk -- the next one in round-robin order
-- for every active request at once (the quantized Chamfer estimate of all
active queries against that chunk, one launch). A request that arrives while
others are running is admitted at the next iteration, whatever chunk comes
next, as soon as a slot and device memory are free; it has seen the whole
corpus after `n_chunks` iterations. It then finishes: the top `shortlist`
documents of its estimate row are reranked with exact float32 Chamfer scores
and the top k are returned (the rerank of GEM's search, Alg. 5 final step).

Because a (query, document) score does not depend on which other queries
share a launch, a request's result is bitwise the same alone and in any mix.

The engine only schedules. Device work goes through an executor with three
calls (set_batch, score_chunk, finish); `DeviceExecutor` runs them with the
library's kernels.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque
from typing import Callable, List, Optional, Sequence

import numpy as np
import torch


@dataclasses.dataclass
class Request:
    rid: int
    vecs: np.ndarray                 # [m_q, 128] float32 query vectors (host)
    t_arrival: float                 # seconds since the engine clock started
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    start_chunk: int = -1
    chunks_done: int = 0
    slot: int = -1
    top_scores: Optional[np.ndarray] = None
    top_ids: Optional[np.ndarray] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.t_done is None else self.t_done - self.t_arrival


class Executor:
    """Device work the engine schedules (interface)."""

    n_docs: int
    n_chunks: int
    bytes_per_request: int

    def set_batch(self, slots: Sequence[int], queries: Sequence[np.ndarray]) -> None:
        raise NotImplementedError

    def score_chunk(self, chunk: int) -> None:
        raise NotImplementedError

    def finish(self, slots: Sequence[int], queries: Sequence[np.ndarray]):
        """-> (top_scores [n, k], top_ids [n, k]) numpy arrays, results on the host."""
        raise NotImplementedError


class ServingEngine:
    """Admission, round-robin chunk schedule and completion bookkeeping."""

    def __init__(self, executor: Executor, max_slots: int, mem_budget_bytes: int,
                 clock: Optional[Callable[[], float]] = None):
        self.ex = executor
        self.max_slots = int(max_slots)
        self.mem_budget = int(mem_budget_bytes)
        self._t0 = None
        self._clock = clock
        self.waiting: deque = deque()
        self.active: List[Request] = []
        self.done: List[Request] = []
        self.free_slots = list(range(self.max_slots))[::-1]
        self.iteration = 0
        self.chunk = 0
        self.refused_for_memory = 0
        self.active_sum = 0               # sum over iterations of the active requests (mean batch size)
        self._batch_key = None

    # -- clock
    def now(self) -> float:
        if self._clock is not None:
            return self._clock()
        if self._t0 is None:
            self._t0 = time.perf_counter()
        return time.perf_counter() - self._t0

    def start_clock(self) -> None:
        self._t0 = time.perf_counter()

    # -- admission
    def memory_in_use(self) -> int:
        return len(self.active) * self.ex.bytes_per_request

    def can_admit(self) -> bool:
        if not self.free_slots:
            return False
        return self.memory_in_use() + self.ex.bytes_per_request <= self.mem_budget

    def submit(self, req: Request) -> None:
        self.waiting.append(req)

    def admit(self) -> int:
        n = 0
        now = self.now()
        while self.waiting and self.waiting[0].t_arrival <= now:
            if not self.can_admit():
                if self.free_slots:
                    self.refused_for_memory += 1
                break
            r = self.waiting.popleft()
            r.slot = self.free_slots.pop()
            r.start_chunk = self.chunk
            r.chunks_done = 0
            r.t_admit = now
            self.active.append(r)
            n += 1
        return n

    # -- one iteration: one corpus chunk for every active request
    def step(self) -> List[Request]:
        self.admit()
        if not self.active:
            return []
        key = tuple(r.slot for r in self.active)
        if key != self._batch_key:
            self.ex.set_batch([r.slot for r in self.active], [r.vecs for r in self.active])
            self._batch_key = key
        self.ex.score_chunk(self.chunk)
        self.active_sum += len(self.active)
        for r in self.active:
            r.chunks_done += 1
        finished = [r for r in self.active if r.chunks_done == self.ex.n_chunks]
        if finished:
            ts, ti = self.ex.finish([r.slot for r in finished], [r.vecs for r in finished])
            t = self.now()
            for i, r in enumerate(finished):
                r.top_scores, r.top_ids, r.t_done = ts[i], ti[i], t
                self.free_slots.append(r.slot)
            self.active = [r for r in self.active if r.chunks_done < self.ex.n_chunks]
            self.done.extend(finished)
        self.chunk = (self.chunk + 1) % self.ex.n_chunks
        self.iteration += 1
        return finished

    def run(self, requests: Sequence[Request], idle_sleep: float = 0.0) -> List[Request]:
        """Serve requests (sorted by arrival) until all are done."""
        for r in sorted(requests, key=lambda r: r.t_arrival):
            self.submit(r)
        if self._clock is None:
            self.start_clock()
        while self.waiting or self.active:
            if not self.active and self.waiting:
                wait = self.waiting[0].t_arrival - self.now()
                if wait > 0:
                    if self._clock is not None:
                        raise RuntimeError("a simulated clock must advance by itself")
                    if idle_sleep:
                        time.sleep(min(wait, idle_sleep))
                    continue
            self.step()
        return self.done


def latency_stats(reqs: Sequence[Request]) -> dict:
    lat = np.array([r.latency for r in reqs if r.latency is not None])
    if lat.size == 0:
        return {"n": 0}
    span = max(r.t_done for r in reqs) - min(r.t_arrival for r in reqs)
    return {"n": int(lat.size), "qps": float(lat.size / span) if span > 0 else float("nan"),
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3)}


class DeviceExecutor(Executor):
    """Executor on the library's kernels: FP8 estimate per chunk, float32 rerank at the end."""

    def __init__(self, D8, D32, n_chunks: int, max_slots: int, shortlist: int = 1000, k: int = 100,
                 max_query_len: int = 64, stream=None):
        import importlib
        self._gem = importlib.import_module(__package__)
        self.D8, self.D32 = D8, D32
        self.n_docs = D8.n_sets
        self.n_chunks = int(n_chunks)
        bounds = np.linspace(0, self.n_docs, self.n_chunks + 1).round().astype(np.int64)
        self.bounds = [int(b) for b in bounds]
        self.shortlist, self.k = int(shortlist), int(k)
        self.max_query_len = int(max_query_len)
        self.device = D8.device
        self.stream = stream
        self.est = torch.empty(max_slots, self.n_docs, dtype=torch.float32, device=self.device)
        self.bytes_per_request = self.n_docs * 4 + max_query_len * 128 * 9 + shortlist * 8
        self.Q8 = None
        self.rows = None

    def _pack(self, queries: Sequence[np.ndarray]):
        lens = [int(q.shape[0]) for q in queries]
        off = np.zeros(len(lens) + 1, np.int64)
        off[1:] = np.cumsum(lens)
        vecs = np.concatenate(queries, 0).astype(np.float32) if queries else np.zeros((0, 128), np.float32)
        v = torch.from_numpy(vecs).pin_memory().to(self.device, non_blocking=True)
        o = torch.from_numpy(off).pin_memory().to(self.device, non_blocking=True)
        return self._gem.Sets(v, o, "f32", max(lens) if lens else 0)

    def set_batch(self, slots, queries):
        Q = self._pack(queries)
        self.Q8 = self._gem.quantize_fp8(Q, stream=self.stream)
        self.rows = torch.tensor(list(slots), dtype=torch.int32).pin_memory().to(self.device, non_blocking=True)

    def score_chunk(self, chunk: int) -> None:
        a, b = self.bounds[chunk], self.bounds[chunk + 1]
        if b <= a:
            return
        Dc = self.D8.view(a, b)
        out = self.est[:, a:]
        self._gem.score_quant(self.Q8, Dc, scores=out, ld=self.n_docs, rows=self.rows, stream=self.stream)

    def finish(self, slots, queries):
        g = self._gem
        rows = torch.tensor(list(slots), dtype=torch.int32).pin_memory().to(self.device, non_blocking=True)
        sl = min(self.shortlist, self.n_docs)
        _, short_i = g.topk(self.est, sl, seg_rows=rows, stream=self.stream)
        Q = self._pack(queries)
        C = g.Cands(short_i.reshape(-1), stride=sl, n_lists=len(slots))
        ts, ti = g.score_exact(Q, self.D32, cands=C, compute="f32", k=self.k, stream=self.stream)
        return ts.cpu().numpy(), ti.cpu().numpy()
