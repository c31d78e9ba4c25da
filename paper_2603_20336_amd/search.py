"""Batched beam expansion captured in a HIP graph.

Each step of GEM's cluster-guided beam search (Alg. 5, neighbour loop) scores
the candidates every query reaches with the quantized Chamfer estimate and
inserts them into the query's bounded result set R (at most ef entries, the
worst evicted). Here a step is one gem_expand_batch call for all queries at
once, and a run of steps -- with candidate lists fixed in device memory -- is
recorded once into a graph and replayed, so the host issues one launch per
run instead of two kernels per step.

The second half runs the whole of Alg. 5 on a graph of the document sets:
set-level clusters (Sec. 4.1), the C Q^T cluster filter, one entry per
selected cluster, and search steps whose candidates are the unvisited,
unpruned neighbours of the best unexpanded results (GraphSearch).
"""
from __future__ import annotations

import contextlib
import ctypes
from typing import List, Optional, Sequence

import torch

from . import GEM_FP8_E4M3, GEM_MXFP4, GEM_MXFP6, Beam, Cands, Sets, expand_batch, expand_workspace_bytes, score_exact


def _on_stream(stream):
    """Make `stream` current for a block (no change when it is None)."""
    return contextlib.nullcontext() if stream is None else torch.cuda.stream(stream)


class ExpansionGraph:
    """`steps` beam-expansion steps over fixed candidate lists, recorded into a graph."""

    def __init__(self, Q8: Sets, D8: Sets, steps: Sequence[Cands], ef: int, stream=None):
        if Q8.dtype != D8.dtype or D8.dtype not in (GEM_FP8_E4M3, GEM_MXFP4, GEM_MXFP6):
            raise TypeError("Q8 and D8 must share one quantized format, FP8, MXFP4 or MXFP6 (quantize the queries "
                            "once, outside the graph)")
        self.Q8, self.D8, self.steps = Q8, D8, list(steps)
        self.device = D8.device
        self.beam = Beam(Q8.n_sets, ef, self.device)
        n = max((c.ids.numel() for c in self.steps), default=0)
        self.cand_scores = torch.empty(max(n, 1), dtype=torch.float32, device=self.device)
        # one workspace for every step (large steps sort their lists there),
        # allocated before any capture
        ws = max((expand_workspace_bytes(Q8, D8, c, True) for c in self.steps), default=0)
        self.ws = torch.empty(ws, dtype=torch.uint8, device=self.device) if ws > 0 else None
        self.graph: Optional[torch.cuda.CUDAGraph] = None

    def run_eager(self, stream=None) -> None:
        self.beam.reset(stream)
        for c in self.steps:
            expand_batch(self.Q8, self.D8, c, self.beam, cand_scores=self.cand_scores[: c.ids.numel()],
                         stream=stream, ws=self.ws)

    def capture(self) -> None:
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(s):
            self.run_eager(s)                     # warm-up outside the graph
        torch.cuda.current_stream(self.device).wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            self.run_eager(s)
        self.graph = g

    def replay(self, stream=None) -> None:
        """Replay the recorded steps on `stream` (default: the current stream);
        a graph replays on the stream that is current when it is launched."""
        if self.graph is None:
            self.capture()
        with _on_stream(stream):
            self.graph.replay()

    def rerank(self, Q32: Sets, D32: Sets, k: int):
        """Exact float32 Chamfer rerank of the beam (Alg. 5 final step) -> (scores, ids) [n_q, k]."""
        C = Cands(self.beam.ids.reshape(-1), stride=self.beam.ef, n_lists=Q32.n_sets)
        return score_exact(Q32, D32, cands=C, compute="f32", k=k)


# ---------------------------------------------------------------------------
# Cluster-guided beam search (Alg. 5) over a graph of the document sets.

def _lib_ctx(device):
    from . import _ctx, _stream, library
    return library(), _ctx(torch.device(device)), _stream


def set_clusters(vec_clusters: torch.Tensor, set_offsets: torch.Tensor, k2: int, r: int, stream=None):
    """Set-level clusters of Sec. 4.1 (TF-IDF pruning): (masks [N, words] int32 bit
    patterns, member offsets [k2 + 1], members) from each vector's cluster."""
    from . import _abi, _ptr
    dev = vec_clusters.device
    lib, ctx, _stream = _lib_ctx(dev)
    n = int(set_offsets.numel() - 1)
    words = (k2 + 31) // 32
    masks = torch.empty(n, words, dtype=torch.int32, device=dev)
    moff = torch.empty(k2 + 1, dtype=torch.int64, device=dev)
    members = torch.empty(max(1, n * r), dtype=torch.int32, device=dev)
    ws = torch.empty(_abi.GEM_SEARCH_CLUSTER_WS, dtype=torch.uint8, device=dev)
    _abi.check(lib.gem_set_clusters(ctx, _ptr(vec_clusters), _ptr(set_offsets), n, int(k2), int(r), _ptr(masks),
                                    _ptr(moff), _ptr(members), _ptr(ws), ws.numel(), _stream(stream)))
    return masks, moff, members


def query_clusters(Q32: Sets, centroids: torch.Tensor, t: int, stream=None) -> torch.Tensor:
    """C_query masks [n_q, words] (S = C Q^T, top-t per query vector, Sec. 4.5)."""
    from . import _abi, _ptr
    dev = Q32.device
    lib, ctx, _stream = _lib_ctx(dev)
    k2 = int(centroids.shape[0])
    masks = torch.empty(Q32.n_sets, (k2 + 31) // 32, dtype=torch.int32, device=dev)
    qs = Q32.struct()
    _abi.check(lib.gem_query_clusters(ctx, ctypes.byref(qs), _ptr(centroids), k2, int(t), _ptr(masks),
                                      _stream(stream)))
    return masks


def _score_any(Q: Sets, D: Sets, **kw):
    from . import score_exact, score_quant, _QUANT
    if D.dtype in _QUANT:
        return score_quant(Q, D, **kw)
    return score_exact(Q, D, compute=D.dtype, **kw)


def knn_graph(D_as_queries: Sets, D: Sets, degree: int, candidates: int = 64, batch: int = 2000,
              forward: Optional[int] = None, stream=None) -> torch.Tensor:
    """A kNN graph of the document sets (scores in D's dtype): row p lists
    `forward` sets by CH(P, .), then the best of the rest of P's `candidates`
    by the symmetric Chamfer similarity CH(P, P') / |P| + CH(P', P) / |P'|,
    P itself left out (default: half and half). CH of one direction favours
    long targets (a max over more vectors), as queries do; alone it makes the
    same long sets everyone's neighbours, and the symmetric half keeps the
    rest of the neighbourhood reachable. D_as_queries holds the same sets in a
    query-side dtype."""
    forward = degree // 2 if forward is None else int(forward)
    from . import topk
    n, dev = D.n_sets, D.device
    cand = torch.empty(n, candidates, dtype=torch.int32, device=dev)
    fwd = torch.empty(n, candidates, dtype=torch.float32, device=dev)
    scores = torch.empty(min(batch, n), n, dtype=torch.float32, device=dev)
    for a in range(0, n, batch):
        b = min(n, a + batch)
        sc = scores[: b - a]
        _score_any(D_as_queries.view(a, b), D, scores=sc, stream=stream)
        s, ids = topk(sc, candidates, stream=stream)
        fwd[a:b], cand[a:b] = s, ids
    # reverse direction: CH(P', P) for every listed pair, the pairs grouped by P'
    src = torch.arange(n, device=dev, dtype=torch.int64).repeat_interleave(candidates)
    dst = cand.reshape(-1).long()
    order = torch.argsort(dst, stable=True)
    counts = torch.bincount(dst, minlength=n)
    off = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    off[1:] = torch.cumsum(counts, 0)
    rc = Cands(src[order].to(torch.int32).contiguous(), off, max_list_len=int(counts.max().item()))
    rev_sorted = _score_any(D_as_queries, D, cands=rc, stream=stream)
    rev = torch.empty_like(rev_sorted)
    rev[order] = rev_sorted
    lens = (D.offsets[1:] - D.offsets[:-1]).to(torch.float32)
    sym = fwd / lens[:, None] + rev.reshape(n, candidates) / lens[cand.long()]
    own = cand.long() == torch.arange(n, device=dev)[:, None]
    # forward part: the best by CH(P, .) (candidates are sorted), P left out
    rank = torch.cumsum((~own).to(torch.int32), 1) - 1
    take_fwd = (~own) & (rank < forward)
    sym = torch.where(own | take_fwd, torch.full_like(sym, float("-inf")), sym)
    _, pos = topk(sym, degree - forward, stream=stream)
    fwd_ids = cand.masked_select(take_fwd).reshape(n, forward)
    return torch.cat([fwd_ids, torch.gather(cand, 1, pos.long())], 1).contiguous()


class ClusterIndex:
    """The searchable index: neighbour lists and set clusters (device tensors)."""

    def __init__(self, neighbors: torch.Tensor, set_masks: torch.Tensor, member_offsets: torch.Tensor,
                 members: torch.Tensor, centroids: torch.Tensor):
        self.neighbors, self.set_masks = neighbors.contiguous(), set_masks.contiguous()
        self.member_offsets, self.members, self.centroids = member_offsets, members, centroids
        self.k2 = int(centroids.shape[0])

    def struct(self):
        from . import _abi, _ptr
        g = _abi.gem_graph()
        g.n_sets, g.k2, g.degree = int(self.neighbors.shape[0]), self.k2, int(self.neighbors.shape[1])
        g.neighbors, g.set_masks = _ptr(self.neighbors), _ptr(self.set_masks)
        g.member_offsets, g.members = _ptr(self.member_offsets), _ptr(self.members)
        return g


class GraphSearch:
    """One batch of queries searched together (Alg. 5, every path of every query
    advancing per step): R in `beam`, the visited / expanded maps and the
    candidate rows in device buffers allocated once."""

    def __init__(self, Q: Sets, D: Sets, index: ClusterIndex, query_masks: torch.Tensor, ef: int, width: int = 4):
        from . import _abi, _ptr
        self.Q, self.D, self.index = Q, D, index
        dev = self.device = D.device
        n_q, n = Q.n_sets, D.n_sets
        deg = int(index.neighbors.shape[1])
        self.row = max(index.k2, width * deg)
        bw = (n + 31) // 32
        self.visited = torch.empty(n_q, bw, dtype=torch.int32, device=dev)
        self.expanded = torch.empty(n_q, bw, dtype=torch.int32, device=dev)
        self.frontier = torch.empty(n_q, width, dtype=torch.int32, device=dev)
        self.cand_ids = torch.empty(n_q, self.row, dtype=torch.int32, device=dev)
        self.cand_scores = torch.empty(n_q, self.row, dtype=torch.float32, device=dev)
        self.active = torch.zeros(1, dtype=torch.int32, device=dev)
        self.query_masks = query_masks.contiguous()
        self.beam = Beam(n_q, ef, dev)
        st = _abi.gem_search_state()
        st.width, st.reserved = int(width), 0
        st.query_masks, st.visited, st.expanded = _ptr(self.query_masks), _ptr(self.visited), _ptr(self.expanded)
        st.frontier, st.cand_ids, st.cand_scores = _ptr(self.frontier), _ptr(self.cand_ids), _ptr(self.cand_scores)
        st.active = _ptr(self.active)
        self._state, self._graph = st, index.struct()
        self._qs, self._ds = Q.struct(), D.struct()
        self.steps = 0
        self._hip_graph: Optional[torch.cuda.CUDAGraph] = None
        self._hip_graph_steps = 0

    def begin(self, random_words: torch.Tensor, stream=None) -> None:
        """random_words: [n_q, k2] uint32 (int32 bit patterns) drawn by the caller."""
        from . import _abi, _ptr
        lib, ctx, _stream = _lib_ctx(self.D.device)
        _abi.check(lib.gem_search_begin(ctx, ctypes.byref(self._qs), ctypes.byref(self._ds), ctypes.byref(self._graph),
                                        ctypes.byref(self._state), _ptr(random_words), ctypes.byref(self.beam.struct()),
                                        _stream(stream)))
        self.steps = 0

    def step(self, stream=None) -> None:
        from . import _abi
        lib, ctx, _stream = _lib_ctx(self.D.device)
        _abi.check(lib.gem_search_step(ctx, ctypes.byref(self._qs), ctypes.byref(self._ds), ctypes.byref(self._graph),
                                       ctypes.byref(self._state), ctypes.byref(self.beam.struct()), _stream(stream)))
        self.steps += 1

    def capture(self, n_steps: int) -> None:
        """Record n_steps search steps into one HIP graph. Every step reads and
        writes only this object's device buffers, so the graph replays on any
        state that begin() left there (recording runs nothing)."""
        s = torch.cuda.Stream(device=self.device)
        s.wait_stream(torch.cuda.current_stream(self.device))
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            for _ in range(n_steps):
                self.step(s)
        torch.cuda.current_stream(self.device).wait_stream(s)
        self.steps = 0
        self._hip_graph, self._hip_graph_steps = g, n_steps

    def run(self, random_words: torch.Tensor, max_steps: int = 10000, check_every: int = 4, graph: bool = True,
            stream=None) -> int:
        """Search until no query has anything left to expand, checking every
        `check_every` steps (a finished query's extra steps change nothing).
        With graph=True the block of steps between checks is one replay of a
        captured HIP graph."""
        if graph and (self._hip_graph is None or self._hip_graph_steps != check_every):
            self.capture(check_every)
        self.begin(random_words, stream)
        # Replays and the reads of the active count are ordered on `stream`,
        # behind begin() and every step before them.
        with _on_stream(stream):
            while self.steps < max_steps:
                if graph:
                    self._hip_graph.replay()
                    self.steps += check_every
                else:
                    for _ in range(check_every):
                        self.step(stream)
                if int(self.active.item()) == 0:
                    break
        return self.steps

    def rerank(self, Q32: Sets, D32: Sets, k: int):
        """Exact float32 Chamfer rerank of R (Alg. 5, last line) -> (scores, ids) [n_q, k]."""
        C = Cands(self.beam.ids.reshape(-1), stride=self.beam.ef, n_lists=Q32.n_sets)
        return score_exact(Q32, D32, cands=C, compute="f32", k=k)
