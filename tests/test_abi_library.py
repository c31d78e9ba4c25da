"""The C-ABI library loads and exports every entry point that include/gem.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gem.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gem_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("gem_score_exact", "gem_score_quant", "gem_topk", "gem_expand_batch",
              "gem_convert_bf16", "gem_quantize_fp8", "gem_workspace_bytes", "gem_beam_merge"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2603_20336_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.fail("libgem.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_abi.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    # the binding declares exactly the header's functions
    assert sorted(_abi.SIGNATURES) == _declared()


def test_status_strings_without_gpu():
    from paper_2603_20336_amd import _abi
    lib = _abi.load()
    assert lib.gem_status_string(0) == b"GEM_OK"
    assert lib.gem_status_string(2) == b"GEM_ERR_WORKSPACE"
    assert b"gfx950" in lib.gem_version()


def test_host_side_argument_errors_without_gpu():
    """Invalid arguments are rejected on the host before anything is enqueued."""
    from paper_2603_20336_amd import _abi
    lib = _abi.load()
    # a NULL context fails before any HIP call
    st = lib.gem_topk(None, None, None, None, 1, 10, 10, None, 5, None, None, None, 0, None)
    assert st == _abi.GEM_ERR_INVALID
    q = _abi.gem_sets()
    q.dtype, q.dim, q.n_sets = 0, 64, 1
    st = lib.gem_score_exact(ctypes.c_void_p(1), ctypes.byref(q), ctypes.byref(q), None, 0, 0,
                             None, 0, None, None, None, None, 0, None)
    assert st == _abi.GEM_ERR_UNSUPPORTED        # dim != 128
    assert b"dim" in lib.gem_last_error()
