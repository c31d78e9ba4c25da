"""ctypes declarations of the C ABI in include/gem.h, and the library loader.

torch is imported before the library is loaded so that the process has a
single HIP runtime: libgem.so then binds to the libamdhip64 torch already
loaded, and torch's streams and device pointers are valid in its calls.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must come before the library is loaded)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgem.so")

GEM_OK, GEM_ERR_INVALID, GEM_ERR_WORKSPACE, GEM_ERR_UNSUPPORTED, GEM_ERR_HIP, GEM_ERR_DEVICE_CHECK = range(6)
GEM_F32, GEM_BF16, GEM_FP8_E4M3, GEM_MXFP4, GEM_MXFP6, GEM_BF16X3 = 0, 1, 2, 3, 4, 5
GEM_OP_SCORE_EXACT, GEM_OP_SCORE_QUANT, GEM_OP_TOPK, GEM_OP_EXPAND = 0, 1, 2, 3
GEM_OP_NEAREST_CENTROID, GEM_OP_CENTROID_UPDATE = 4, 5
GEM_OPT_TOPK_FUSION, GEM_OPT_CHECK, GEM_OPT_GATHER_ORDER = 0, 1, 2
GEM_TOPK_AUTO, GEM_TOPK_FUSED, GEM_TOPK_STAGED = 0, 1, 2
GEM_GATHER_AUTO, GEM_GATHER_BY_QUERY, GEM_GATHER_BY_DOCUMENT = 0, 1, 2
GEM_STATIC_SCRATCH_BYTES = 64 << 20
GEM_MAX_QUERY_LEN = 256
GEM_MAX_K = 2048
GEM_MAX_EF = 1024
GEM_DIM = 128
BEAM_MAX_ENTRIES = 4096

# every function the header declares, with (restype, argtypes)
c_p = ctypes.c_void_p
i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t


class gem_sets(ctypes.Structure):
    _fields_ = [("dtype", i32), ("dim", i32), ("n_sets", i64), ("n_vecs", i64),
                ("max_set_len", i32), ("reserved", i32),
                ("offsets", c_p), ("vecs", c_p), ("scales", c_p),
                ("codebook_rows", i64), ("codes", c_p)]


class gem_cands(ctypes.Structure):
    _fields_ = [("n_lists", i64), ("n_entries", i64), ("stride", i32), ("max_list_len", i32),
                ("offsets", c_p), ("ids", c_p)]


class gem_beam(ctypes.Structure):
    _fields_ = [("ef", i32), ("reserved", i32), ("scores", c_p), ("ids", c_p)]


class gem_dense_schedule(ctypes.Structure):
    _fields_ = [("chunk_docs", i32), ("items_per_slot", i32), ("slots_per_xcd", i32), ("reserved", i32)]


class gem_gather_schedule(ctypes.Structure):
    _fields_ = [("entries_per_wave", i32), ("depth", i32), ("reserved", i32 * 2)]


class gem_graph(ctypes.Structure):
    _fields_ = [("n_sets", i64), ("k2", i32), ("degree", i32), ("neighbors", c_p), ("set_masks", c_p),
                ("member_offsets", c_p), ("members", c_p)]


class gem_search_state(ctypes.Structure):
    _fields_ = [("width", i32), ("reserved", i32), ("query_masks", c_p), ("visited", c_p), ("expanded", c_p),
                ("frontier", c_p), ("cand_ids", c_p), ("cand_scores", c_p), ("active", c_p)]


GEM_SEARCH_CLUSTER_WS = 8192

P_SETS = ctypes.POINTER(gem_sets)
P_CANDS = ctypes.POINTER(gem_cands)
P_BEAM = ctypes.POINTER(gem_beam)

SIGNATURES = {
    "gem_create": (i32, [ctypes.POINTER(c_p), ctypes.c_int, ctypes.c_char_p]),
    "gem_destroy": (i32, [c_p]),
    "gem_status_string": (ctypes.c_char_p, [i32]),
    "gem_last_error": (ctypes.c_char_p, []),
    "gem_version": (ctypes.c_char_p, []),
    "gem_workspace_bytes": (sz, [c_p, i32, P_SETS, P_SETS, P_CANDS, i32, i32, i32]),
    "gem_set_option": (i32, [c_p, i32, i64]),
    "gem_get_option": (i32, [c_p, i32, ctypes.POINTER(i64)]),
    "gem_check_status": (i32, [c_p, c_p]),
    "gem_convert_bf16": (i32, [c_p, c_p, i64, i32, c_p, c_p]),
    "gem_split_bf16x3": (i32, [c_p, c_p, i64, i32, c_p, c_p]),
    "gem_quantize_fp8": (i32, [c_p, c_p, i64, i32, c_p, c_p, c_p]),
    "gem_quantize_mxfp4": (i32, [c_p, c_p, i64, i32, c_p, c_p, c_p]),
    "gem_quantize_mxfp6": (i32, [c_p, c_p, i64, i32, c_p, c_p, c_p]),
    "gem_score_exact": (i32, [c_p, P_SETS, P_SETS, P_CANDS, i32, i32, c_p, i64, c_p, c_p, c_p, c_p, sz, c_p]),
    "gem_score_quant": (i32, [c_p, P_SETS, P_SETS, P_CANDS, i32, c_p, i64, c_p, c_p, c_p, c_p, sz, c_p]),
    "gem_score_quant_static": (i32, [c_p, P_SETS, P_SETS, P_CANDS, i32, c_p, i64, c_p, c_p, c_p, c_p]),
    "gem_topk": (i32, [c_p, c_p, c_p, c_p, i64, i64, i64, c_p, i32, c_p, c_p, c_p, sz, c_p]),
    "gem_expand_batch": (i32, [c_p, P_SETS, P_SETS, P_CANDS, P_BEAM, c_p, c_p, sz, c_p]),
    "gem_beam_merge": (i32, [c_p, c_p, P_CANDS, P_BEAM, c_p]),
    "gem_beam_reset": (i32, [c_p, P_BEAM, i64, c_p]),
    "gem_validate_sets": (i32, [c_p, P_SETS, c_p]),
    "gem_validate_cands": (i32, [c_p, P_CANDS, i64, c_p]),
    "gem_copy_rows": (i32, [c_p, c_p, c_p, c_p, c_p, i64, i64, c_p]),
    "gem_nearest_centroid": (i32, [c_p, c_p, i64, c_p, i64, i32, i32, c_p, c_p, sz, c_p]),
    "gem_centroid_update": (i32, [c_p, c_p, i64, i32, c_p, c_p, i64, c_p, c_p, c_p, sz, c_p]),
    "gem_codebook_workspace_bytes": (sz, [i32, i64, i64]),
    "gem_emd_sinkhorn": (i32, [c_p, P_SETS, P_SETS, c_p, c_p, i64, ctypes.c_float, i32, c_p, c_p, sz, c_p]),
    "gem_emd_workspace_bytes": (sz, [i64]),
    "gem_set_clusters": (i32, [c_p, c_p, c_p, i64, i32, i32, c_p, c_p, c_p, c_p, sz, c_p]),
    "gem_query_clusters": (i32, [c_p, P_SETS, c_p, i32, i32, c_p, c_p]),
    "gem_search_begin": (i32, [c_p, P_SETS, P_SETS, ctypes.POINTER(gem_graph), ctypes.POINTER(gem_search_state),
                               c_p, P_BEAM, c_p]),
    "gem_search_step": (i32, [c_p, P_SETS, P_SETS, ctypes.POINTER(gem_graph), ctypes.POINTER(gem_search_state),
                              P_BEAM, c_p]),
    "gem_get_dense_schedule": (i32, [c_p, i32, i64, i64, ctypes.POINTER(gem_dense_schedule)]),
    "gem_set_dense_schedule": (i32, [c_p, i32, i64, i64, ctypes.POINTER(gem_dense_schedule)]),
    "gem_autotune_dense": (i32, [c_p, P_SETS, P_SETS, i32, c_p, i64, c_p, sz, c_p, i32,
                                 ctypes.POINTER(gem_dense_schedule), ctypes.POINTER(ctypes.c_float)]),
    "gem_get_gather_schedule": (i32, [c_p, i32, i64, i64, ctypes.POINTER(gem_gather_schedule)]),
    "gem_set_gather_schedule": (i32, [c_p, i32, i64, i64, ctypes.POINTER(gem_gather_schedule)]),
    "gem_autotune_gather": (i32, [c_p, P_SETS, P_SETS, P_CANDS, i32, c_p, c_p, sz, c_p, i32,
                                  ctypes.POINTER(gem_gather_schedule), ctypes.POINTER(ctypes.c_float)]),
    "gem_save_tune_cache": (i32, [c_p, ctypes.c_char_p]),
    "gem_load_tune_cache": (i32, [c_p, ctypes.c_char_p]),
}

_lib = None


class GemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{status_name(status)}: {msg}")
        self.status = status


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libgem.so (built by paper_2603_20336_amd.build); fails loudly if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2603_20336_amd.build` "
                          "(the scoring path has no fallback)")
    lib = ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_name(status: int) -> str:
    return ["GEM_OK", "GEM_ERR_INVALID", "GEM_ERR_WORKSPACE", "GEM_ERR_UNSUPPORTED",
            "GEM_ERR_HIP", "GEM_ERR_DEVICE_CHECK"][status] if 0 <= status <= 5 else f"status {status}"


def check(status: int) -> None:
    if status != GEM_OK:
        msg = load().gem_last_error()
        raise GemError(status, msg.decode() if msg else "")
