"""MI355X (gfx950) set-to-set scoring for multi-vector retrieval (GEM, arXiv 2603.20336).

Thin Python binding of libgem.so (C ABI in include/gem.h). Every step of the
scoring path runs in the library's HIP kernels; this module only marshals
torch tensors (device memory) and the current torch stream into the C calls,
and allocates outputs and workspaces with torch's allocator.

    Q = Sets.from_batch(queries, device)                # float32 CSR sets
    D = Sets.from_batch(corpus, device).to_bf16()       # corpus conversion, once
    top_s, top_i = score_exact(Q, D, k=100, compute="bf16")
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

import torch

from . import _abi
from ._abi import (GEM_BF16, GEM_BF16X3, GEM_F32, GEM_FP8_E4M3, GEM_MAX_K, GEM_MAX_QUERY_LEN, GEM_MXFP4, GEM_MXFP6,
                   GemError)

__all__ = ["Sets", "Cands", "Beam", "GemError", "convert_bf16", "quantize_fp8", "score_exact",
           "score_quant", "topk", "expand_batch", "beam_merge", "beam_reset", "validate_sets", "validate_cands",
           "library", "GEM_F32", "GEM_BF16", "GEM_FP8_E4M3", "GEM_MXFP4", "quantize_mxfp4", "GEM_MXFP6", "quantize_mxfp6", "GEM_MAX_K", "GEM_MAX_QUERY_LEN", "dense_schedule",
           "set_dense_schedule", "autotune_dense", "copy_rows", "nearest_centroid", "centroid_update",
           "kmeans", "encode", "codebook_size",
           "emd_sinkhorn", "set_topk_fusion", "topk_fusion", "set_gather_order", "get_gather_order", "score_workspace_bytes", "gather_schedule",
           "set_check", "check_status", "set_gather_schedule", "autotune_gather", "save_tune_cache", "load_tune_cache",
           "GEM_BF16X3", "split_bf16x3"]

_DTYPES = {"f32": GEM_F32, "bf16": GEM_BF16, "fp8": GEM_FP8_E4M3, "mxfp4": GEM_MXFP4, "mxfp6": GEM_MXFP6,
           "bf16x3": GEM_BF16X3, GEM_F32: GEM_F32, GEM_BF16: GEM_BF16, GEM_FP8_E4M3: GEM_FP8_E4M3,
           GEM_MXFP4: GEM_MXFP4, GEM_MXFP6: GEM_MXFP6, GEM_BF16X3: GEM_BF16X3}
_ROW_TORCH = {GEM_F32: torch.float32, GEM_BF16: torch.uint16, GEM_FP8_E4M3: torch.uint8, GEM_MXFP4: torch.uint8,
              GEM_MXFP6: torch.uint8, GEM_BF16X3: torch.uint16}
_ROW_WIDTH = {GEM_F32: 128, GEM_BF16: 128, GEM_FP8_E4M3: 128, GEM_MXFP4: 64, GEM_MXFP6: 96,
              GEM_BF16X3: 256}   # tensor columns per row
_QUANT = (GEM_FP8_E4M3, GEM_MXFP4, GEM_MXFP6)


def library():
    """The loaded libgem.so (raises ImportError if it was not built)."""
    return _abi.load()


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class _Context:
    """One library context per device; GEM_TUNE_CACHE names a tune cache to load."""

    def __init__(self, device: int):
        lib = library()
        h = ctypes.c_void_p()
        cache = os.environ.get("GEM_TUNE_CACHE")
        _abi.check(lib.gem_create(ctypes.byref(h), device, cache.encode() if cache else None))
        self.handle = h
        self.device = device


_contexts: dict = {}


def _ctx(device: torch.device) -> ctypes.c_void_p:
    idx = device.index if device.index is not None else torch.cuda.current_device()
    c = _contexts.get(idx)
    if c is None:
        c = _contexts[idx] = _Context(idx)
    return c.handle


class Sets:
    """A ragged batch of 128-d vector sets on the device (CSR).

    vecs: [n_vecs, 128] float32 / uint16 (bf16 bits) / uint8 (E4M3 codes), or
        [n_vecs, 64] uint8 (MXFP4: two E2M1 codes a byte), or [n_vecs, 96] uint8
        (MXFP6: 6-bit E2M3 codes, 24 bytes per 32-element block)
    offsets: [n_sets + 1] int64 absolute row indices
    scales: FP8: [n_vecs] float32 powers of two; MXFP4, MXFP6: [n_vecs, 4] uint8
        E8M0 block exponents
    max_len: host-side bound of the set lengths
    codes: code sets only, [n_vecs] int32: entry r stands for row codes[r] of
        vecs, which then holds the codebook (its nearest centroid, Sec. 4.2);
        CH over code sets is the quantized estimate qCH of Sec. 4.5
    """

    def __init__(self, vecs: torch.Tensor, offsets: torch.Tensor, dtype, max_len: int,
                 scales: Optional[torch.Tensor] = None, n_sets: Optional[int] = None,
                 codes: Optional[torch.Tensor] = None):
        self.dtype = _DTYPES[dtype]
        if vecs.dtype != _ROW_TORCH[self.dtype]:
            raise TypeError(f"vecs dtype {vecs.dtype} does not match gem dtype {self.dtype}")
        if vecs.dim() != 2 or vecs.shape[1] != _ROW_WIDTH[self.dtype] or not vecs.is_contiguous():
            raise ValueError(f"vecs must be a contiguous [n, {_ROW_WIDTH[self.dtype]}] tensor")
        if offsets.dtype != torch.int64 or not offsets.is_contiguous():
            raise TypeError("offsets must be contiguous int64")
        if codes is not None and (codes.dtype != torch.int32 or codes.dim() != 1 or not codes.is_contiguous()):
            raise TypeError("codes must be a contiguous 1-d int32 tensor")
        self.vecs, self.offsets, self.scales, self.codes = vecs, offsets, scales, codes
        self.max_len = int(max_len)
        self.n_sets = int(offsets.numel() - 1) if n_sets is None else int(n_sets)

    @property
    def device(self) -> torch.device:
        return self.vecs.device

    @property
    def n_vecs(self) -> int:
        return int(self.codes.numel() if self.codes is not None else self.vecs.shape[0])

    @classmethod
    def from_batch(cls, batch, device="cuda") -> "Sets":
        """float32 Sets from a workloads.SetBatch (host or device)."""
        vecs = batch.vecs.to(device=device, dtype=torch.float32).contiguous()
        off = batch.offsets.to(device=device, dtype=torch.int64).contiguous()
        return cls(vecs, off, GEM_F32, batch.max_len())

    def struct(self) -> _abi.gem_sets:
        s = _abi.gem_sets()
        s.dtype, s.dim, s.n_sets, s.n_vecs = self.dtype, _abi.GEM_DIM, self.n_sets, self.n_vecs
        s.max_set_len, s.reserved = self.max_len, 0
        s.offsets, s.vecs, s.scales = _ptr(self.offsets), _ptr(self.vecs), _ptr(self.scales)
        s.codebook_rows = int(self.vecs.shape[0]) if self.codes is not None else 0
        s.codes = _ptr(self.codes)
        return s

    def view(self, a: int, b: int) -> "Sets":
        """Sets a..b-1 as a batch of their own (no copy; ids become relative to a)."""
        return Sets(self.vecs, self.offsets[a:b + 1], self.dtype, self.max_len, self.scales, codes=self.codes)

    def to_bf16(self, stream=None) -> "Sets":
        return convert_bf16(self, stream)

    def to_bf16x3(self, stream=None) -> "Sets":
        return split_bf16x3(self, stream)

    def to_fp8(self, stream=None) -> "Sets":
        return quantize_fp8(self, stream)

    def to_mxfp4(self, stream=None) -> "Sets":
        return quantize_mxfp4(self, stream)

    def to_mxfp6(self, stream=None) -> "Sets":
        return quantize_mxfp6(self, stream)


class Cands:
    """Candidate-id lists, one per query: CSR (offsets) or fixed-length rows (stride)."""

    def __init__(self, ids: torch.Tensor, offsets: Optional[torch.Tensor] = None, stride: int = 0,
                 max_list_len: Optional[int] = None, n_lists: Optional[int] = None):
        if ids.dtype != torch.int32 or not ids.is_contiguous():
            raise TypeError("ids must be contiguous int32")
        self.ids, self.offsets, self.stride = ids, offsets, int(stride)
        if offsets is not None:
            self.n_lists = int(offsets.numel() - 1)
            self.max_list_len = int(max_list_len) if max_list_len is not None else \
                int((offsets[1:] - offsets[:-1]).max().item()) if self.n_lists else 0
        else:
            self.n_lists = int(n_lists) if n_lists is not None else (ids.numel() // max(self.stride, 1))
            self.max_list_len = self.stride

    def struct(self) -> _abi.gem_cands:
        c = _abi.gem_cands()
        c.n_lists, c.n_entries = self.n_lists, int(self.ids.numel())
        c.stride, c.max_list_len = self.stride, self.max_list_len
        c.offsets, c.ids = _ptr(self.offsets), _ptr(self.ids)
        return c


class Beam:
    """The bounded per-query result set R (Alg. 5): [n_queries, ef] scores and ids."""

    def __init__(self, n_queries: int, ef: int, device="cuda", stream=None):
        self.ef = int(ef)
        self.scores = torch.empty(n_queries, ef, dtype=torch.float32, device=device)
        self.ids = torch.empty(n_queries, ef, dtype=torch.int32, device=device)
        self.reset(stream)

    @property
    def n_queries(self) -> int:
        return int(self.scores.shape[0])

    def struct(self) -> _abi.gem_beam:
        b = _abi.gem_beam()
        b.ef, b.reserved, b.scores, b.ids = self.ef, 0, _ptr(self.scores), _ptr(self.ids)
        return b

    def reset(self, stream=None) -> None:
        beam_reset(self, stream)


def _ws(n: int, device) -> Optional[torch.Tensor]:
    return torch.empty(n, dtype=torch.uint8, device=device) if n > 0 else None


def convert_bf16(S: Sets, stream=None) -> Sets:
    """float32 sets -> bfloat16 sets (round to nearest even)."""
    if S.dtype != GEM_F32:
        raise TypeError("convert_bf16 takes float32 sets")
    n = int(S.vecs.shape[0])                       # (a code set converts its codebook)
    out = torch.empty(n, _abi.GEM_DIM, dtype=torch.uint16, device=S.device)
    _abi.check(library().gem_convert_bf16(_ctx(S.device), _ptr(S.vecs), n, _abi.GEM_DIM,
                                          _ptr(out), _stream(stream)))
    return Sets(out, S.offsets, GEM_BF16, S.max_len, n_sets=S.n_sets, codes=S.codes)


def split_bf16x3(S: Sets, stream=None) -> Sets:
    """float32 sets -> bfloat16 (hi, lo) pairs, the operands of the exact mode
    that runs float32 products as three bfloat16 products (GEM_BF16X3)."""
    if S.dtype != GEM_F32:
        raise TypeError("split_bf16x3 takes float32 sets")
    n = int(S.vecs.shape[0])                       # (a code set converts its codebook)
    out = torch.empty(n, 2 * _abi.GEM_DIM, dtype=torch.uint16, device=S.device)
    _abi.check(library().gem_split_bf16x3(_ctx(S.device), _ptr(S.vecs), n, _abi.GEM_DIM,
                                          _ptr(out), _stream(stream)))
    return Sets(out, S.offsets, GEM_BF16X3, S.max_len, n_sets=S.n_sets, codes=S.codes)


def quantize_fp8(S: Sets, stream=None) -> Sets:
    """float32 sets -> E4M3 codes + one power-of-two scale per vector."""
    if S.dtype != GEM_F32:
        raise TypeError("quantize_fp8 takes float32 sets")
    n = int(S.vecs.shape[0])                       # (a code set converts its codebook)
    out = torch.empty(n, _abi.GEM_DIM, dtype=torch.uint8, device=S.device)
    sc = torch.empty(n, dtype=torch.float32, device=S.device)
    _abi.check(library().gem_quantize_fp8(_ctx(S.device), _ptr(S.vecs), n, _abi.GEM_DIM,
                                          _ptr(out), _ptr(sc), _stream(stream)))
    return Sets(out, S.offsets, GEM_FP8_E4M3, S.max_len, scales=sc, n_sets=S.n_sets, codes=S.codes)


def quantize_mxfp4(S: Sets, stream=None) -> Sets:
    """float32 sets -> MXFP4: E2M1 codes with one power-of-two scale per 32-element block."""
    if S.dtype != GEM_F32:
        raise TypeError("quantize_mxfp4 takes float32 sets")
    n = int(S.vecs.shape[0])                       # (a code set converts its codebook)
    out = torch.empty(n, 64, dtype=torch.uint8, device=S.device)
    ex = torch.empty(n, 4, dtype=torch.uint8, device=S.device)
    _abi.check(library().gem_quantize_mxfp4(_ctx(S.device), _ptr(S.vecs), n, _abi.GEM_DIM, _ptr(out), _ptr(ex),
                                            _stream(stream)))
    return Sets(out, S.offsets, GEM_MXFP4, S.max_len, scales=ex, n_sets=S.n_sets, codes=S.codes)


def quantize_mxfp6(S: Sets, stream=None) -> Sets:
    """float32 sets -> MXFP6: E2M3 codes with one power-of-two scale per 32-element block."""
    if S.dtype != GEM_F32:
        raise TypeError("quantize_mxfp6 takes float32 sets")
    n = int(S.vecs.shape[0])                       # (a code set converts its codebook)
    out = torch.empty(n, 96, dtype=torch.uint8, device=S.device)
    ex = torch.empty(n, 4, dtype=torch.uint8, device=S.device)
    _abi.check(library().gem_quantize_mxfp6(_ctx(S.device), _ptr(S.vecs), n, _abi.GEM_DIM, _ptr(out), _ptr(ex),
                                            _stream(stream)))
    return Sets(out, S.offsets, GEM_MXFP6, S.max_len, scales=ex, n_sets=S.n_sets, codes=S.codes)


def _score(fn_exact: bool, Q: Sets, D: Sets, cands: Optional[Cands], k: int, compute: int,
           scores: Optional[torch.Tensor], ld: int, rows: Optional[torch.Tensor], want_scores: bool,
           stream, ws: Optional[torch.Tensor]):
    lib = library()
    dev = D.device
    qs, ds = Q.struct(), D.struct()
    cs = cands.struct() if cands is not None else None
    pc = ctypes.byref(cs) if cs is not None else None
    if scores is None and (want_scores or k == 0):
        n = cands.ids.numel() if cands is not None else Q.n_sets * D.n_sets
        shape = (n,) if cands is not None else (Q.n_sets, D.n_sets)
        scores = torch.empty(shape, dtype=torch.float32, device=dev)
    op = _abi.GEM_OP_SCORE_EXACT if fn_exact else _abi.GEM_OP_SCORE_QUANT
    need = lib.gem_workspace_bytes(_ctx(dev), op, ctypes.byref(qs), ctypes.byref(ds), pc, compute, k,
                                   int(scores is not None))
    if ws is None or ws.numel() < need:
        ws = _ws(need, dev)
    top_s = torch.empty(Q.n_sets, k, dtype=torch.float32, device=dev) if k > 0 else None
    top_i = torch.empty(Q.n_sets, k, dtype=torch.int32, device=dev) if k > 0 else None
    args = (ctypes.byref(qs), ctypes.byref(ds), pc)
    tail = (_ptr(scores), int(ld), _ptr(rows), _ptr(top_s), _ptr(top_i), _ptr(ws),
            0 if ws is None else ws.numel(), _stream(stream))
    if fn_exact:
        st = lib.gem_score_exact(_ctx(dev), *args, compute, k, *tail)
    else:
        st = lib.gem_score_quant(_ctx(dev), *args, k, *tail)
    _abi.check(st)
    if k == 0:
        return scores
    return (top_s, top_i, scores) if want_scores else (top_s, top_i)


_TOPK_MODES = {"auto": _abi.GEM_TOPK_AUTO, "fused": _abi.GEM_TOPK_FUSED, "staged": _abi.GEM_TOPK_STAGED}


def set_topk_fusion(mode: str, device="cuda") -> None:
    """How exhaustive calls with k > 0 and no score buffer find the top-k:
    "auto" (fused into the scorer when that needs less workspace than staging
    the score rows), "fused" or "staged". Every mode gives the same result."""
    _abi.check(library().gem_set_option(_ctx(torch.device(device)), _abi.GEM_OPT_TOPK_FUSION, _TOPK_MODES[mode]))


_GATHER_ORDERS = {"auto": _abi.GEM_GATHER_AUTO, "query": _abi.GEM_GATHER_BY_QUERY,
                  "document": _abi.GEM_GATHER_BY_DOCUMENT}


def set_gather_order(mode: str, device="cuda") -> None:
    """How candidate-list calls walk their entries: "query" (one wave per run of
    a query's entries, documents streamed), "document" (entries grouped by
    document, each document staged once in LDS and scored against all of its
    queries) or "auto" (once the lists hold two or more entries per corpus
    document in f32 and bf16x3, four in the other formats: a document whose listings times 16-row tiles reach a threshold
    of the format by document, the rest by query). Every order gives bitwise
    the same scores."""
    _abi.check(library().gem_set_option(_ctx(torch.device(device)), _abi.GEM_OPT_GATHER_ORDER,
                                        _GATHER_ORDERS[mode]))


def get_gather_order(device="cuda") -> str:
    v = ctypes.c_int64(0)
    _abi.check(library().gem_get_option(_ctx(torch.device(device)), _abi.GEM_OPT_GATHER_ORDER, ctypes.byref(v)))
    return {b: a for a, b in _GATHER_ORDERS.items()}[int(v.value)]


def set_check(on: bool, device="cuda") -> None:
    """GEM_CHECK mode: every call validates its device inputs first (synchronizing)."""
    _abi.check(library().gem_set_option(_ctx(torch.device(device)), _abi.GEM_OPT_CHECK, int(bool(on))))


def check_status(stream=None, device="cuda") -> None:
    """Synchronize the stream and raise GemError if a kernel failed or checked calls found bad data."""
    _abi.check(library().gem_check_status(_ctx(torch.device(device)), _stream(stream)))


def topk_fusion(device="cuda") -> str:
    v = ctypes.c_int64(0)
    _abi.check(library().gem_get_option(_ctx(torch.device(device)), _abi.GEM_OPT_TOPK_FUSION, ctypes.byref(v)))
    return {b: a for a, b in _TOPK_MODES.items()}[int(v.value)]


def score_workspace_bytes(Q: Sets, D: Sets, cands: Optional[Cands] = None, k: int = 0, compute=None,
                          scores_given: bool = False) -> int:
    """Workspace bytes of a scoring call with these arguments (gem_workspace_bytes)."""
    compute = D.dtype if compute is None else _DTYPES[compute]
    qs, ds = Q.struct(), D.struct()
    cs = cands.struct() if cands is not None else None
    op = _abi.GEM_OP_SCORE_QUANT if compute in _QUANT else _abi.GEM_OP_SCORE_EXACT
    return int(library().gem_workspace_bytes(_ctx(D.device), op, ctypes.byref(qs), ctypes.byref(ds),
                                             ctypes.byref(cs) if cs is not None else None, compute, int(k),
                                             int(scores_given)))


def score_exact(Q: Sets, D: Sets, cands: Optional[Cands] = None, k: int = 0, compute="f32",
                scores: Optional[torch.Tensor] = None, ld: int = 0, rows: Optional[torch.Tensor] = None,
                want_scores: bool = False, stream=None, ws: Optional[torch.Tensor] = None):
    """Exact Chamfer scores (Def. 1): compute "f32" (float32 products), "bf16x3"
    (each float32 product as three bfloat16 products, D split by split_bf16x3)
    or "bf16" (products of bfloat16-rounded operands).

    cands None: every query against every document -> [n_q, n_docs] (or into
    `scores` with row stride `ld` and optional row map `rows`). With cands:
    one score per candidate entry. k > 0 returns (top_scores, top_ids) (and
    the scores when want_scores)."""
    return _score(True, Q, D, cands, k, _DTYPES[compute], scores, ld, rows, want_scores, stream, ws)


def copy_rows(src: torch.Tensor, dst: torch.Tensor, src_idx: Optional[torch.Tensor] = None,
              dst_idx: Optional[torch.Tensor] = None, n: Optional[int] = None, stream=None) -> None:
    """dst[dst_idx[i]] = src[src_idx[i]] for i < n (rows of the leading dimension;
    an index of None is the identity). Rows of src and dst must have the same size."""
    rb = src[0].numel() * src.element_size() if src.dim() > 1 else src.element_size()
    rbd = dst[0].numel() * dst.element_size() if dst.dim() > 1 else dst.element_size()
    if rb != rbd or not src.is_contiguous() or not dst.is_contiguous():
        raise ValueError("copy_rows needs contiguous tensors with equal row sizes")
    for t in (src_idx, dst_idx):
        if t is not None and (t.dtype != torch.int64 or not t.is_contiguous()):
            raise TypeError("row indices must be contiguous int64")
    if n is None:
        n = (src_idx if src_idx is not None else dst_idx if dst_idx is not None else src).shape[0]
    _abi.check(library().gem_copy_rows(_ctx(dst.device), _ptr(src), _ptr(src_idx), _ptr(dst), _ptr(dst_idx), int(n),
                                       int(rb), _stream(stream)))


def _rows(x: torch.Tensor, what: str) -> int:
    if x.dim() != 2 or x.shape[1] != _abi.GEM_DIM or not x.is_contiguous():
        raise ValueError(f"{what} must be a contiguous [n, 128] tensor")
    return int(x.shape[0])


def codebook_size(n_vectors: int) -> int:
    """|C_quant| of Sec. 5.1: the power of two 2^floor(log2(16 sqrt(n_vectors)))."""
    return 1 << int(math.floor(math.log2(16.0 * math.sqrt(max(1, n_vectors)))))


def nearest_centroid(x: torch.Tensor, centroids: torch.Tensor, stream=None) -> torch.Tensor:
    """NN(x) of Sec. 4.2 as int32 centroid indices: argmin_j ||x_i - c_j||^2, ties to
    the smallest j. x and centroids are float32 rows (float32 products) or bfloat16
    bit patterns (uint16; bf16 products), both of the same type."""
    dt = {torch.float32: GEM_F32, torch.uint16: GEM_BF16}.get(x.dtype)
    if dt is None or centroids.dtype != x.dtype:
        raise TypeError("x and centroids must both be float32 or both bfloat16 bit patterns (uint16)")
    n, k = _rows(x, "x"), _rows(centroids, "centroids")
    lib = library()
    codes = torch.empty(n, dtype=torch.int32, device=x.device)
    need = lib.gem_codebook_workspace_bytes(_abi.GEM_OP_NEAREST_CENTROID, n, k)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
    _abi.check(lib.gem_nearest_centroid(_ctx(x.device), _ptr(x), n, _ptr(centroids), k, _abi.GEM_DIM, dt,
                                        _ptr(codes), _ptr(ws), need, _stream(stream)))
    return codes


def centroid_update(x: torch.Tensor, codes: torch.Tensor, centroids: torch.Tensor,
                    out: Optional[torch.Tensor] = None, stream=None):
    """One k-means update (Sec. 4.1): each centroid moves to the mean of its rows;
    one without rows stays. Returns (new centroids, rows per centroid)."""
    if x.dtype != torch.float32 or centroids.dtype != torch.float32:
        raise TypeError("centroid_update takes float32 rows and centroids")
    if codes.dtype != torch.int32 or not codes.is_contiguous() or codes.numel() != x.shape[0]:
        raise TypeError("codes must be contiguous int32, one per row")
    n, k = _rows(x, "x"), _rows(centroids, "centroids")
    out = torch.empty_like(centroids) if out is None else out
    counts = torch.empty(k, dtype=torch.int32, device=x.device)
    lib = library()
    need = lib.gem_codebook_workspace_bytes(_abi.GEM_OP_CENTROID_UPDATE, n, k)
    ws = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
    _abi.check(lib.gem_centroid_update(_ctx(x.device), _ptr(x), n, _abi.GEM_DIM, _ptr(codes), _ptr(centroids), k,
                                       _ptr(out), _ptr(counts), _ptr(ws), need, _stream(stream)))
    return out, counts


def _bf16_rows(x: torch.Tensor, stream=None) -> torch.Tensor:
    out = torch.empty(x.shape[0], _abi.GEM_DIM, dtype=torch.uint16, device=x.device)
    _abi.check(library().gem_convert_bf16(_ctx(x.device), _ptr(x), int(x.shape[0]), _abi.GEM_DIM, _ptr(out),
                                          _stream(stream)))
    return out


def kmeans(x: torch.Tensor, init_rows: torch.Tensor, n_iter: int, assign: str = "f32", stream=None) -> torch.Tensor:
    """The k-means vocabulary C_quant of Sec. 4.1: Lloyd's algorithm on the float32
    rows x from the centroids x[init_rows] (the caller draws init_rows), n_iter
    rounds of (nearest centroid, update). `assign` is the precision of the
    nearest-centroid step ("f32" or "bf16"); the update is always float32."""
    if init_rows.dtype != torch.int64:
        raise TypeError("init_rows must be int64")
    k = int(init_rows.numel())
    C = torch.empty(k, _abi.GEM_DIM, dtype=torch.float32, device=x.device)
    copy_rows(x, C, src_idx=init_rows.to(x.device).contiguous(), n=k, stream=stream)
    xa = _bf16_rows(x, stream) if assign == "bf16" else x
    for _ in range(n_iter):
        Ca = _bf16_rows(C, stream) if assign == "bf16" else C
        codes = nearest_centroid(xa, Ca, stream)
        C, _ = centroid_update(x, codes, C, out=C, stream=stream)
    return C


def encode(S: Sets, centroids: torch.Tensor, assign: str = "f32", stream=None) -> Sets:
    """The code set of float32 sets S over a float32 codebook: every vector is
    replaced by the index of its nearest centroid (Sec. 4.2)."""
    if S.dtype != GEM_F32 or S.codes is not None:
        raise TypeError("encode takes float32 sets of vectors")
    if assign == "bf16":
        codes = nearest_centroid(_bf16_rows(S.vecs, stream), _bf16_rows(centroids, stream), stream)
    else:
        codes = nearest_centroid(S.vecs, centroids, stream)
    return Sets(centroids, S.offsets, GEM_F32, S.max_len, n_sets=S.n_sets, codes=codes)


def emd_sinkhorn(A: Sets, B: Sets, a_idx: torch.Tensor, b_idx: torch.Tensor, eps: float = 0.05, n_iter: int = 100,
                 stream=None) -> torch.Tensor:
    """Entropic EMD (Sec. 4.2; Sinkhorn in the log domain) of the set pairs
    (A[a_idx[p]], B[b_idx[p]]); float32 sets, or code sets over float32
    codebooks for qEMD. Returns [n_pairs] float32 (NaN for an empty set)."""
    for t in (a_idx, b_idx):
        if t.dtype != torch.int32 or not t.is_contiguous():
            raise TypeError("pair indices must be contiguous int32")
    n = int(a_idx.numel())
    out = torch.empty(n, dtype=torch.float32, device=A.device)
    sa, sb = A.struct(), B.struct()
    lib = library()
    need = lib.gem_emd_workspace_bytes(n)
    ws = _ws(need, A.device)
    _abi.check(lib.gem_emd_sinkhorn(_ctx(A.device), ctypes.byref(sa), ctypes.byref(sb), _ptr(a_idx), _ptr(b_idx),
                                    n, float(eps), int(n_iter), _ptr(out), _ptr(ws), need, _stream(stream)))
    return out


def _sched_dict(s) -> dict:
    return {"chunk_docs": int(s.chunk_docs), "items_per_slot": int(s.items_per_slot),
            "slots_per_xcd": int(s.slots_per_xcd)}


def dense_schedule(dtype, q_rows: int, n_docs: int, device="cuda") -> dict:
    """The dense-scorer schedule a call of this shape class uses."""
    s = _abi.gem_dense_schedule()
    _abi.check(library().gem_get_dense_schedule(_ctx(torch.device(device)), _DTYPES[dtype], int(q_rows),
                                                int(n_docs), ctypes.byref(s)))
    return _sched_dict(s)


def set_dense_schedule(dtype, q_rows: int, n_docs: int, schedule: Optional[dict], device="cuda") -> None:
    """Install a schedule for the shape class (None: back to the library default)."""
    p = None
    if schedule is not None:
        s = _abi.gem_dense_schedule(int(schedule["chunk_docs"]), int(schedule["items_per_slot"]),
                                    int(schedule["slots_per_xcd"]), 0)
        p = ctypes.byref(s)
    _abi.check(library().gem_set_dense_schedule(_ctx(torch.device(device)), _DTYPES[dtype], int(q_rows),
                                                int(n_docs), p))


def autotune_dense(Q: Sets, D: Sets, compute=None, reps: int = 2, scores: Optional[torch.Tensor] = None,
                   ld: int = 0, stream=None):
    """Time the candidate schedules of the dense scorer on this call, install the
    fastest for its shape class and return (schedule, ms per call)."""
    compute = D.dtype if compute is None else _DTYPES[compute]
    dev = D.device
    if scores is None:
        scores = torch.empty(Q.n_sets, D.n_sets, dtype=torch.float32, device=dev)
    qs, ds = Q.struct(), D.struct()
    op = _abi.GEM_OP_SCORE_QUANT if compute in _QUANT else _abi.GEM_OP_SCORE_EXACT
    need = library().gem_workspace_bytes(_ctx(dev), op, ctypes.byref(qs), ctypes.byref(ds), None, compute, 0, 1)
    ws = _ws(need, dev)
    best = _abi.gem_dense_schedule()
    ms = ctypes.c_float(0.0)
    _abi.check(library().gem_autotune_dense(_ctx(dev), ctypes.byref(qs), ctypes.byref(ds), compute, _ptr(scores),
                                            int(ld), _ptr(ws), 0 if ws is None else ws.numel(), _stream(stream),
                                            int(reps), ctypes.byref(best), ctypes.byref(ms)))
    return _sched_dict(best), float(ms.value)


def _gather_dict(g) -> dict:
    return {"entries_per_wave": int(g.entries_per_wave), "depth": int(g.depth)}


def gather_schedule(dtype, n_lists: int, max_list_len: int, device="cuda") -> dict:
    """The gathered-scorer schedule a call of this shape class uses (entries_per_wave 0: the library's rule)."""
    g = _abi.gem_gather_schedule()
    _abi.check(library().gem_get_gather_schedule(_ctx(torch.device(device)), _DTYPES[dtype], int(n_lists),
                                                 int(max_list_len), ctypes.byref(g)))
    return _gather_dict(g)


def set_gather_schedule(dtype, n_lists: int, max_list_len: int, schedule: Optional[dict], device="cuda") -> None:
    """Install a gathered-scorer schedule for the shape class (None: back to the library's rule)."""
    p = None
    if schedule is not None:
        g = _abi.gem_gather_schedule(int(schedule["entries_per_wave"]), int(schedule["depth"]))
        p = ctypes.byref(g)
    _abi.check(library().gem_set_gather_schedule(_ctx(torch.device(device)), _DTYPES[dtype], int(n_lists),
                                                 int(max_list_len), p))


def autotune_gather(Q: Sets, D: Sets, cands: Cands, compute=None, reps: int = 2,
                    scores: Optional[torch.Tensor] = None, stream=None):
    """Time the gathered scorer's candidate schedules on this call (scoring the
    candidate lists), install the fastest for its shape class and return
    (schedule, ms per call)."""
    compute = D.dtype if compute is None else _DTYPES[compute]
    dev = D.device
    if scores is None:
        scores = torch.empty(cands.ids.numel(), dtype=torch.float32, device=dev)
    qs, ds, cs = Q.struct(), D.struct(), cands.struct()
    op = _abi.GEM_OP_SCORE_QUANT if compute in _QUANT else _abi.GEM_OP_SCORE_EXACT
    need = library().gem_workspace_bytes(_ctx(dev), op, ctypes.byref(qs), ctypes.byref(ds), ctypes.byref(cs),
                                         compute, 0, 1)
    ws = _ws(need, dev)
    best = _abi.gem_gather_schedule()
    ms = ctypes.c_float(0.0)
    _abi.check(library().gem_autotune_gather(_ctx(dev), ctypes.byref(qs), ctypes.byref(ds), ctypes.byref(cs), compute,
                                             _ptr(scores), _ptr(ws), 0 if ws is None else ws.numel(), _stream(stream),
                                             int(reps), ctypes.byref(best), ctypes.byref(ms)))
    return _gather_dict(best), float(ms.value)


def save_tune_cache(path: str, device="cuda") -> None:
    """Write every installed dense and gathered schedule to a JSON tune cache."""
    _abi.check(library().gem_save_tune_cache(_ctx(torch.device(device)), str(path).encode()))


def load_tune_cache(path: str, device="cuda") -> None:
    """Install the schedules of a JSON tune cache for this GPU's architecture."""
    _abi.check(library().gem_load_tune_cache(_ctx(torch.device(device)), str(path).encode()))


def score_quant(Q: Sets, D8: Sets, cands: Optional[Cands] = None, k: int = 0,
                scores: Optional[torch.Tensor] = None, ld: int = 0, rows: Optional[torch.Tensor] = None,
                want_scores: bool = False, stream=None, ws: Optional[torch.Tensor] = None):
    """Quantized estimate in D8's format, FP8 E4M3, MXFP4 or MXFP6 (same conventions as score_exact)."""
    if D8.dtype not in _QUANT:
        raise TypeError("score_quant takes FP8, MXFP4 or MXFP6 documents")
    return _score(False, Q, D8, cands, k, D8.dtype, scores, ld, rows, want_scores, stream, ws)


def topk(scores: torch.Tensor, k: int, seg_offsets: Optional[torch.Tensor] = None,
         seg_ids: Optional[torch.Tensor] = None, seg_rows: Optional[torch.Tensor] = None,
         n_segs: Optional[int] = None, seg_len: Optional[int] = None, seg_ld: int = 0, stream=None):
    """Segmented top-k: CSR segments (seg_offsets [+ seg_ids]) or the rows of a
    [n, L] matrix (optionally the rows listed in seg_rows). Returns (scores, ids) [n_segs, k]."""
    lib = library()
    dev = scores.device
    if seg_offsets is not None:
        n = seg_offsets.numel() - 1
        L, ld = 0, 0
    else:
        if scores.dim() == 2:
            L = scores.shape[1] if seg_len is None else seg_len
            ld = seg_ld or scores.stride(0)
            n = (seg_rows.numel() if seg_rows is not None else scores.shape[0]) if n_segs is None else n_segs
        else:
            L, ld = int(seg_len), int(seg_ld or seg_len)
            n = int(n_segs)
    top_s = torch.empty(n, k, dtype=torch.float32, device=dev)
    top_i = torch.empty(n, k, dtype=torch.int32, device=dev)
    _abi.check(lib.gem_topk(_ctx(dev), _ptr(scores), _ptr(seg_offsets), _ptr(seg_ids), n, L, ld,
                            _ptr(seg_rows), k, _ptr(top_s), _ptr(top_i), None, 0, _stream(stream)))
    return top_s, top_i


def expand_batch(Q8: Sets, D8: Sets, cands: Cands, beam: Beam, cand_scores: Optional[torch.Tensor] = None,
                 stream=None, ws: Optional[torch.Tensor] = None) -> None:
    """One beam-expansion step: FP8-estimate every candidate and merge it into the beam in place."""
    lib = library()
    dev = D8.device
    qs, ds, cs, bs = Q8.struct(), D8.struct(), cands.struct(), beam.struct()
    need = lib.gem_workspace_bytes(_ctx(dev), _abi.GEM_OP_EXPAND, ctypes.byref(qs), ctypes.byref(ds),
                                   ctypes.byref(cs), D8.dtype, 1, int(cand_scores is not None))
    if ws is None or ws.numel() < need:
        ws = _ws(need, dev)
    _abi.check(lib.gem_expand_batch(_ctx(dev), ctypes.byref(qs), ctypes.byref(ds), ctypes.byref(cs),
                                    ctypes.byref(bs), _ptr(cand_scores), _ptr(ws),
                                    0 if ws is None else ws.numel(), _stream(stream)))


def beam_merge(cand_scores: torch.Tensor, cands: Cands, beam: Beam, stream=None) -> None:
    """Merge already-scored candidates into the beam in place (top-ef, ids distinct)."""
    cs, bs = cands.struct(), beam.struct()
    _abi.check(library().gem_beam_merge(_ctx(beam.scores.device), _ptr(cand_scores), ctypes.byref(cs),
                                        ctypes.byref(bs), _stream(stream)))


def expand_workspace_bytes(Q8: Sets, D8: Sets, cands: Cands, with_cand_scores: bool) -> int:
    qs, ds, cs = Q8.struct(), D8.struct(), cands.struct()
    return int(library().gem_workspace_bytes(_ctx(D8.device), _abi.GEM_OP_EXPAND, ctypes.byref(qs),
                                             ctypes.byref(ds), ctypes.byref(cs), D8.dtype, 1,
                                             int(with_cand_scores)))


def beam_reset(beam: Beam, stream=None) -> None:
    b = beam.struct()
    _abi.check(library().gem_beam_reset(_ctx(beam.scores.device), ctypes.byref(b), beam.n_queries,
                                        _stream(stream)))


def validate_sets(S: Sets, stream=None) -> None:
    s = S.struct()
    _abi.check(library().gem_validate_sets(_ctx(S.device), ctypes.byref(s), _stream(stream)))


def validate_cands(C: Cands, n_sets: int, stream=None) -> None:
    c = C.struct()
    _abi.check(library().gem_validate_cands(_ctx(C.ids.device), ctypes.byref(c), int(n_sets), _stream(stream)))
