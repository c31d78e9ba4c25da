"""Batched beam expansion captured in a HIP graph.

Each step of GEM's cluster-guided beam search (Alg. 5, neighbour loop) scores
the candidates every query reaches with the quantized Chamfer estimate and
inserts them into the query's bounded result set R (at most ef entries, the
worst evicted). Here a step is one gem_expand_batch call for all queries at
once, and a run of steps -- with candidate lists fixed in device memory -- is
recorded once into a graph and replayed, so the host issues one launch per
run instead of two kernels per step.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import torch

from . import Beam, Cands, Sets, expand_batch, expand_workspace_bytes, score_exact


class ExpansionGraph:
    """`steps` beam-expansion steps over fixed candidate lists, recorded into a graph."""

    def __init__(self, Q8: Sets, D8: Sets, steps: Sequence[Cands], ef: int, stream=None):
        if Q8.dtype != 2:
            raise TypeError("Q8 must hold FP8 query sets (quantize them once, outside the graph)")
        self.Q8, self.D8, self.steps = Q8, D8, list(steps)
        self.device = D8.device
        self.beam = Beam(Q8.n_sets, ef, self.device)
        n = max((c.ids.numel() for c in self.steps), default=0)
        self.cand_scores = torch.empty(max(n, 1), dtype=torch.float32, device=self.device)
        for c in self.steps:
            if expand_workspace_bytes(Q8, D8, c, True) != 0:
                raise RuntimeError("expansion with FP8 queries and a score buffer needs no workspace")
        self.graph: Optional[torch.cuda.CUDAGraph] = None

    def run_eager(self, stream=None) -> None:
        self.beam.reset(stream)
        for c in self.steps:
            expand_batch(self.Q8, self.D8, c, self.beam, cand_scores=self.cand_scores[: c.ids.numel()],
                         stream=stream)

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

    def replay(self) -> None:
        if self.graph is None:
            self.capture()
        self.graph.replay()

    def rerank(self, Q32: Sets, D32: Sets, k: int):
        """Exact float32 Chamfer rerank of the beam (Alg. 5 final step) -> (scores, ids) [n_q, k]."""
        C = Cands(self.beam.ids.reshape(-1), stride=self.beam.ef, n_lists=Q32.n_sets)
        return score_exact(Q32, D32, cands=C, compute="f32", k=k)
