"""Serving loop for multi-vector queries: memory-admitted continuous batching.

The corpus stays resident on the device as FP8 codes (for the estimate) and
float32 rows (for the exact rerank). It is split into `n_chunks` document
chunks. Every iteration scores one chunk -- the next one in round-robin order
-- for every active request at once (the quantized Chamfer estimate of all
active queries against that chunk, one launch). A request that arrives while
others are running is admitted at the next iteration, whatever chunk comes
next, as soon as a slot and device memory are free; it has seen the whole
corpus after `n_chunks` chunks (an iteration may score several consecutive
chunks when the active batch is light: `chunk_work`). It then finishes: the
top `shortlist` documents of its estimate row are reranked with exact float32
Chamfer scores and the top k are returned (the rerank of GEM's search, Alg. 5
final step).

Because a (query, document) score does not depend on which other queries
share a launch, a request's result is bitwise the same alone and in any mix.

The engine only schedules. Device work goes through an executor (admit,
set_batch, score_chunk, finish_async / ready / results); `DeviceExecutor` runs
them with the library's kernels. A request's query vectors are uploaded and
quantized once, at admission, into a device slot; a batch is gathered from the
slots on the device; finished requests' results come back through an
asynchronous copy that the engine polls, so the host never waits for the
device inside the loop.
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

    def admit(self, slots: Sequence[int], queries: Sequence[np.ndarray]) -> None:
        """New requests take these slots (upload their queries)."""

    def set_batch(self, slots: Sequence[int], queries: Sequence[np.ndarray]) -> None:
        raise NotImplementedError

    def score_chunk(self, chunk: int) -> None:
        raise NotImplementedError

    def score_chunks(self, chunk: int, span: int) -> None:
        """Chunks chunk, chunk + 1, ... (span of them, wrapping around the corpus)."""
        for i in range(span):
            self.score_chunk((chunk + i) % self.n_chunks)

    def finish(self, slots: Sequence[int], queries: Sequence[np.ndarray]):
        """-> (top_scores [n, k], top_ids [n, k]) numpy arrays, results on the host."""
        raise NotImplementedError

    # asynchronous completion (default: the synchronous finish, ready at once)
    def finish_async(self, slots: Sequence[int], queries: Sequence[np.ndarray]):
        return self.finish(slots, queries)

    def ready(self, handle) -> bool:
        return True

    def results(self, handle):
        return handle


class ServingEngine:
    """Admission, round-robin chunk schedule and completion bookkeeping."""

    def __init__(self, executor: Executor, max_slots: int, mem_budget_bytes: Optional[int] = None,
                 clock: Optional[Callable[[], float]] = None, chunk_work: int = 0):
        """mem_budget_bytes: device memory for request state (None: the
        executor's own budget, `device_budget`, which it derives from the
        device's free memory). A request is admitted only while the state of
        the active requests plus its own fits the budget.

        chunk_work: if > 0, an iteration scores as many consecutive chunks as
        fit chunk_work (query vectors x chunks) for the active batch, at least
        one: a light batch then takes the corpus in fewer, fuller iterations
        (less per-iteration host time in each request's latency), a heavy one
        keeps one chunk per iteration. 0: always one chunk."""
        self.ex = executor
        self.chunk_work = int(chunk_work)
        self.max_slots = min(int(max_slots), int(getattr(executor, "max_slots", max_slots)))
        self.mem_budget = int(mem_budget_bytes if mem_budget_bytes is not None else executor.device_budget)
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
        self.pending: List[tuple] = []    # (handle, finished requests) awaiting their results
        self._batch_key = None
        # requests completed while the executor waited for the device
        self._early: List[Request] = []

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
        new = []
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
            new.append(r)
        if new:
            self.ex.admit([r.slot for r in new], [r.vecs for r in new])
        return len(new)

    def poll(self) -> List[Request]:
        """Complete the finished requests whose results have reached the host."""
        out, keep = [], []
        for handle, reqs in self.pending:
            if self.ex.ready(handle):
                ts, ti = self.ex.results(handle)
                t = self.now()
                for i, r in enumerate(reqs):
                    r.top_scores, r.top_ids, r.t_done = ts[i], ti[i], t
                self.done.extend(reqs)
                out.extend(reqs)
            else:
                keep.append((handle, reqs))
        self.pending = keep
        return out

    def _poll_waiting(self) -> None:
        if self.pending:
            self._early.extend(self.poll())

    def _take_early(self) -> List[Request]:
        out, self._early = self._early, []
        return out

    # -- one iteration: one corpus chunk for every active request
    def step(self) -> List[Request]:
        """One iteration; returns the requests completed (results on the host) during it."""
        if hasattr(self.ex, "on_wait"):
            self.ex.on_wait = self._poll_waiting                 # (the executor may serve several engines)
        completed = self._take_early() + self.poll()
        self.admit()
        if not self.active:
            return completed + self._take_early()
        key = tuple(r.slot for r in self.active)
        if key != self._batch_key:
            self.ex.set_batch([r.slot for r in self.active], [r.vecs for r in self.active])
            self._batch_key = key
        span = self.span()
        self.ex.score_chunks(self.chunk, span)
        self.active_sum += len(self.active)
        for r in self.active:
            r.chunks_done += span
        # (a request whose revolution ends inside the span scores a few of its
        # chunks twice; a score does not depend on the batch, so the repeat
        # writes the same values)
        finished = [r for r in self.active if r.chunks_done >= self.ex.n_chunks]
        if finished:
            # the slots are free at once: later work on them is ordered after
            # this request's on the device stream
            handle = self.ex.finish_async([r.slot for r in finished], [r.vecs for r in finished])
            self.pending.append((handle, finished))
            for r in finished:
                self.free_slots.append(r.slot)
            self.active = [r for r in self.active if r.chunks_done < self.ex.n_chunks]
        self.chunk = (self.chunk + span) % self.ex.n_chunks
        self.iteration += 1
        return completed + self._take_early() + self.poll()

    def span(self) -> int:
        """Chunks the next iteration scores."""
        if self.chunk_work <= 0:
            return 1
        qv = sum(r.vecs.shape[0] for r in self.active)
        return max(1, min(self.ex.n_chunks, self.chunk_work // max(1, qv)))

    def run(self, requests: Sequence[Request], idle_sleep: float = 0.0) -> List[Request]:
        """Serve requests (sorted by arrival) until all are done."""
        for r in sorted(requests, key=lambda r: r.t_arrival):
            self.submit(r)
        if self._clock is None:
            self.start_clock()
        while self.waiting or self.active or self.pending:
            if not self.active and self.waiting and not self.pending:
                t = self.now()
                wait = self.waiting[0].t_arrival - t
                if wait > 0:
                    if self._clock is not None:
                        # a simulated clock advances as it is read
                        if self.now() <= t:
                            raise RuntimeError("a simulated clock must advance by itself")
                        continue
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
    """Executor on the library's kernels: FP8 estimate per chunk, float32 rerank at the end.

    Each slot holds one request's query vectors on the device (float32 for the
    rerank, FP8 codes and scales for the estimate), written once at admission.
    max_ahead: iterations the host may issue before the device has finished
    the oldest of them (1 keeps a new request behind at most one iteration;
    at most the result ring's length minus 2).
    mem_budget_bytes: device memory for request state; None takes half of
    the device's free memory at construction. The slots (and their score
    rows) are sized to it: at most budget // bytes_per_request requests are
    resident, and the engine admits by the same budget.
    """

    RESULT_RING = 16

    def __init__(self, D8, D32, n_chunks: int, max_slots: int, shortlist: int = 1000, k: int = 100,
                 max_query_len: int = 64, stream=None, copy_stream: bool = False, max_ahead: int = 1,
                 mem_budget_bytes: Optional[int] = None):
        import importlib
        self._gem = importlib.import_module(__package__)
        self.D8, self.D32 = D8, D32
        self.n_docs = D8.n_sets
        self.n_chunks = int(n_chunks)
        bounds = np.linspace(0, self.n_docs, self.n_chunks + 1).round().astype(np.int64)
        self.bounds = [int(b) for b in bounds]
        self.shortlist, self.k = int(shortlist), int(k)
        self.L = int(max_query_len)
        self.max_ahead = max(1, int(max_ahead))
        if self.max_ahead > self.RESULT_RING - 2:
            raise ValueError(f"max_ahead {max_ahead} exceeds {self.RESULT_RING - 2} (the result ring's length - 2)")
        self.device = D8.device
        self.stream = stream
        # device state per request: its estimate row, its query slot (float32
        # and FP8 rows) and its shortlist
        self.bytes_per_request = self.n_docs * 4 + max_query_len * 128 * 9 + shortlist * 8
        if mem_budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.device)
            mem_budget_bytes = free // 2
        self.device_budget = int(mem_budget_bytes)
        self.max_slots = max(1, min(int(max_slots), self.device_budget // self.bytes_per_request))
        max_slots = self.max_slots
        self.est = torch.empty(max_slots, self.n_docs, dtype=torch.float32, device=self.device)
        # slot storage: slot s owns rows [s L, s L + len)
        n_rows = self.max_slots * self.L
        self.q32 = torch.zeros(n_rows, 128, dtype=torch.float32, device=self.device)
        self.q8 = torch.zeros(n_rows, 128, dtype=torch.uint8, device=self.device)
        self.q8s = torch.ones(n_rows, dtype=torch.float32, device=self.device)
        self.lens = np.zeros(self.max_slots, np.int64)
        # packed batches, gathered from the slots into fixed buffers (no
        # allocation per membership change): the estimate batch and the
        # finishing requests' float32 queries
        self.pk8 = torch.empty(n_rows, 128, dtype=torch.uint8, device=self.device)
        self.pk8s = torch.empty(n_rows, dtype=torch.float32, device=self.device)
        self.pk32 = torch.empty(n_rows, 128, dtype=torch.float32, device=self.device)
        # pinned staging for uploads, which run on a copy stream of their own
        # (so that they never queue behind the scoring work); the staging is
        # reused once the previous upload is done
        # a ring of staging buffers: one is reused only after the upload issued
        # from it several uploads ago has completed, which is almost never a wait
        # (admission vectors and index lists have rings of their own; an
        # iteration takes up to one vector and three index buffers)
        self._rings = {
            "v": [torch.empty(n_rows, 128, dtype=torch.float32).pin_memory() for _ in range(4)],
            "i": [torch.empty(2 * n_rows + 2 * self.max_slots + 2, dtype=torch.int64).pin_memory()
                  for _ in range(12)]}
        self._ring_evt = {k: [None] * len(v) for k, v in self._rings.items()}
        self._ring_at = {"v": 0, "i": 0}
        self._copy = torch.cuda.Stream(device=self.device) if copy_stream else None
        # admission vectors uploaded on the compute stream land in device
        # buffers of their own, one per staging buffer, reused in stream order
        # (admit consumes them at once; index uploads stay fresh tensors, since
        # the packed batch keeps views of them across iterations)
        self._dev_rings = None if copy_stream else {
            "v": [torch.empty_like(h, device=self.device) for h in self._rings["v"]]}
        # ring of pinned result buffers for finished requests: entry j holds
        # [device copy event, results read by the host]
        self._ring = [(torch.empty(self.max_slots, self.k, dtype=torch.float32).pin_memory(),
                       torch.empty(self.max_slots, self.k, dtype=torch.int32).pin_memory(), [None, True])
                      for _ in range(self.RESULT_RING)]
        self._ring_pos = 0
        self._off2 = torch.zeros(2, dtype=torch.int64, device=self.device)
        # one workspace for the loop's scoring calls (they run in order on the
        # executor's stream), grown only when a call needs more: a batch size
        # the loop has not met before then allocates nothing
        self._wsbuf = torch.empty(16 << 20, dtype=torch.uint8, device=self.device)
        self._iter_evts = []
        self.Q8 = None
        self.rows = None
        # called over and over while the host waits for the device (the
        # engine collects finished results then, not only between iterations)
        self.on_wait: Optional[Callable[[], None]] = None

    def _stream(self):
        return self.stream if self.stream is not None else torch.cuda.current_stream(self.device)

    def autotune(self, sample: Sequence[np.ndarray], max_batch: Optional[int] = None, reps: int = 3,
                 chunk_work: int = 0) -> dict:
        """Tune the library's schedules for the shapes this loop launches, on
        sample queries of the serving mix: the FP8 scorer for batches of 1, 2,
        4, ... requests (up to max_batch) against the chunks an iteration of
        that batch scores (one, or as many as fit chunk_work query vectors x
        chunks: ServingEngine's rule), and the float32 rerank for finishing
        batches of up to 64 requests. The schedules are installed in the
        device's context for each shape class (a schedule changes the launch,
        never a score). Returns {shape: schedule}."""
        g = self._gem
        cs = self._stream()
        max_batch = min(len(sample), self.max_slots if max_batch is None else int(max_batch))
        out = {}
        with torch.cuda.stream(cs):
            n = 1
            while n <= max_batch:
                qs = sorted(sample[:n], key=lambda q: -q.shape[0])
                lens = np.array([q.shape[0] for q in qs], np.int64)
                off = torch.from_numpy(np.concatenate([[0], np.cumsum(lens)])).to(self.device)
                Q32 = g.Sets(torch.from_numpy(np.concatenate(qs, 0)).to(self.device), off, "f32", int(lens.max()))
                Q8 = g.quantize_fp8(Q32, stream=cs)
                span = 1 if chunk_work <= 0 else max(1, min(self.n_chunks, int(chunk_work) // int(lens.sum())))
                chunk = self.D8.view(self.bounds[0], self.bounds[span])
                sched, _ = g.autotune_dense(Q8, chunk, reps=reps, scores=self.est[:n], ld=self.n_docs, stream=cs)
                out[f"score_fp8_{n}"] = sched
                if n <= 64:
                    # finishing batch: its shortlists come from its own estimate rows
                    for c0 in range(self.n_chunks):
                        Dc = self.D8.view(self.bounds[c0], self.bounds[c0 + 1])
                        g.score_quant(Q8, Dc, scores=self.est[:n, self.bounds[c0]:], ld=self.n_docs, stream=cs)
                    sl = min(self.shortlist, self.n_docs)
                    _, short_i = g.topk(self.est[:n], sl, stream=cs)
                    C = g.Cands(short_i.reshape(-1), stride=sl, n_lists=n)
                    gs, _ = g.autotune_gather(Q32, self.D32, C, compute="f32", reps=reps, stream=cs)
                    out[f"rerank_f32_{n}"] = gs
                n *= 2
        cs.synchronize()
        return out

    def _stage(self, kind: str):
        """The next staging buffer of a ring, once its last upload is done; -> (buffer, ring index)."""
        j = self._ring_at[kind]
        self._ring_at[kind] = (j + 1) % len(self._rings[kind])
        evt = self._ring_evt[kind][j]
        if evt is not None:
            evt.synchronize()
        return self._rings[kind][j], j

    def _upload(self, host: torch.Tensor, kind: str, j: int) -> torch.Tensor:
        """Copy pinned `host` (ring `kind`, buffer j) to the device: on the
        compute stream, or on the copy stream with the compute stream waiting
        for it on the device."""
        cs = self._stream()
        st = cs if self._copy is None else self._copy
        with torch.cuda.stream(st):
            if self._dev_rings is not None and kind in self._dev_rings:
                dev = self._dev_rings[kind][j].view(-1)[: host.numel()].view(host.shape)
                dev.copy_(host, non_blocking=True)
            else:
                dev = host.to(self.device, non_blocking=True)
            evt = torch.cuda.Event()
            evt.record(st)
        self._ring_evt[kind][j] = evt
        if self._copy is not None:
            cs.wait_event(evt)
            dev.record_stream(cs)
        return dev

    def _rows_of(self, slots) -> np.ndarray:
        slots = np.asarray(slots, np.int64)
        lens = self.lens[slots]
        starts = slots * self.L
        tot = int(lens.sum())
        idx = np.repeat(starts - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens) + np.arange(tot)
        return idx, lens

    def admit(self, slots, queries):
        g = self._gem
        lens = np.array([q.shape[0] for q in queries], np.int64)
        if (lens > self.L).any():
            raise ValueError(f"query longer than {self.L} vectors")
        for s, m in zip(slots, lens):
            self.lens[s] = m
        tot = int(lens.sum())
        if tot == 0:
            return
        hv, jv = self._stage("v")
        hi, ji = self._stage("i")
        sv = hv[:tot].numpy()
        np.concatenate(queries, 0, out=sv) if len(queries) > 1 else np.copyto(sv, queries[0])
        idx, _ = self._rows_of(slots)
        hi.numpy()[:tot] = idx
        v = self._upload(hv[:tot], "v", jv)
        ri = self._upload(hi[:tot], "i", ji)
        cs = self._stream()
        with torch.cuda.stream(cs):
            g.copy_rows(v, self.q32, dst_idx=ri, n=tot, stream=cs)
            # (the quantizer reads rows only; the offsets just complete the view)
            q8 = g.quantize_fp8(g.Sets(v, self._off2, "f32", int(lens.max())), stream=cs)
            g.copy_rows(q8.vecs, self.q8, dst_idx=ri, n=tot, stream=cs)
            g.copy_rows(q8.scales, self.q8s, dst_idx=ri, n=tot, stream=cs)

    def _gather(self, slots, fp8: bool):
        """Packed sets of the slots' queries, gathered on the device."""
        g = self._gem
        idx, lens = self._rows_of(slots)
        n = len(slots)
        off = np.zeros(n + 1, np.int64)
        off[1:] = np.cumsum(lens)
        hi, ji = self._stage("i")
        # one upload: row indices and offsets (int64), then the slots as int32
        # (the row map of the scores), packed two to an int64 word
        st = hi.numpy()
        st[:idx.size] = idx
        st[idx.size:idx.size + n + 1] = off
        n_w = (n + 1) // 2
        st[idx.size + n + 1:idx.size + n + 1 + n_w].view(np.int32)[:n] = slots
        dev = self._upload(hi[:idx.size + n + 1 + n_w], "i", ji)
        with torch.cuda.stream(self._stream()):
            ri, o = dev[:idx.size], dev[idx.size:idx.size + n + 1]
            rows32 = dev[idx.size + n + 1:].view(torch.int32)[:n]
            mx = int(lens.max()) if n else 0
            r = idx.size
            cs = self._stream()
            if fp8:
                g.copy_rows(self.q8, self.pk8, src_idx=ri, n=r, stream=cs)
                g.copy_rows(self.q8s, self.pk8s, src_idx=ri, n=r, stream=cs)
                S = g.Sets(self.pk8[:r], o, "fp8", mx, scales=self.pk8s[:r])
            else:
                g.copy_rows(self.q32, self.pk32, src_idx=ri, n=r, stream=cs)
                S = g.Sets(self.pk32[:r], o, "f32", mx)
        return S, rows32

    def set_batch(self, slots, queries):
        # longest queries first: the scorer packs queries, in order, into
        # blocks of a fixed column count, and decreasing lengths leave the
        # least padding at the block ends (the row map keeps each score in
        # its request's row, so the order changes no result)
        slots = np.asarray(slots, np.int64)
        order = np.argsort(-self.lens[slots], kind="stable")
        self.Q8, self.rows = self._gather(slots[order], fp8=True)

    def _workspace(self, need: int) -> Optional[torch.Tensor]:
        if need > self._wsbuf.numel():
            self._wsbuf = torch.empty(2 * need, dtype=torch.uint8, device=self.device)
        return self._wsbuf

    def _wait(self, evt) -> None:
        if self.on_wait is not None:
            while not evt.query():
                self.on_wait()
        evt.synchronize()

    def score_chunk(self, chunk: int) -> None:
        self.score_chunks(chunk, 1)

    def score_chunks(self, chunk: int, span: int) -> None:
        # the host runs at most max_ahead iterations ahead of the device:
        # deeper queues add their whole backlog to a new request's latency
        # (the next iteration's admission and gather are issued before this
        # wait, so they still overlap the previous iteration's scoring)
        if len(self._iter_evts) >= self.max_ahead:
            self._wait(self._iter_evts.pop(0))
        end = chunk + span
        ranges = [(chunk, min(end, self.n_chunks))]
        if end > self.n_chunks:
            ranges.append((0, end - self.n_chunks))             # wrapped around the corpus
        for c0, c1 in ranges:
            a, b = self.bounds[c0], self.bounds[c1]
            if b > a:
                Dc = self.D8.view(a, b)
                out = self.est[:, a:]
                ws = self._workspace(self._gem.score_workspace_bytes(self.Q8, Dc, scores_given=True))
                self._gem.score_quant(self.Q8, Dc, scores=out, ld=self.n_docs, rows=self.rows, stream=self.stream,
                                      ws=ws)
        evt = torch.cuda.Event()
        evt.record(self._stream())
        self._iter_evts.append(evt)

    def finish_async(self, slots, queries):
        g = self._gem
        Q, rows = self._gather(slots, fp8=False)
        sl = min(self.shortlist, self.n_docs)
        with torch.cuda.stream(self._stream()):
            _, short_i = g.topk(self.est, sl, seg_rows=rows, stream=self.stream)
            C = g.Cands(short_i.reshape(-1), stride=sl, n_lists=len(slots))
            ws = self._workspace(g.score_workspace_bytes(Q, self.D32, cands=C, k=self.k, compute="f32"))
            ts, ti = g.score_exact(Q, self.D32, cands=C, compute="f32", k=self.k, stream=self.stream, ws=ws)
            hs_full, hi_full, slot_evt = self._ring[self._ring_pos]
            self._ring_pos = (self._ring_pos + 1) % len(self._ring)
            if not slot_evt[1]:
                # (max_ahead < ring length - 1 keeps every pending result's
                # buffer out of reach; this guards that bound)
                raise RuntimeError("result ring overrun: a finished batch's results were not read yet")
            if slot_evt[0] is not None:
                slot_evt[0].synchronize()                       # the buffer's previous device copy is done
            n = len(slots)
            hs, hi = hs_full[:n], hi_full[:n]
            hs.copy_(ts, non_blocking=True)
            hi.copy_(ti, non_blocking=True)
            evt = torch.cuda.Event()
            evt.record(self._stream())
            slot_evt[0] = evt
            slot_evt[1] = False
        return (evt, hs, hi, ts, ti, slot_evt)

    def ready(self, handle) -> bool:
        return handle[0].query()

    def results(self, handle):
        evt, hs, hi = handle[0], handle[1], handle[2]
        evt.synchronize()
        out = hs.numpy().copy(), hi.numpy().copy()
        handle[5][1] = True                                     # the ring entry may be reused
        return out

    def finish(self, slots, queries):
        h = self.finish_async(slots, queries)
        return self.results(h)
