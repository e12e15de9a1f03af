"""The C-ABI library loads on the host and exports every symbol include/bm25.h declares.

No compute call is made here (no GPU is needed).
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bm25.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bm25_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib_path():
    from paper_2407_03618_amd import bm25
    if not os.path.exists(bm25.LIB_PATH):
        from paper_2407_03618_amd.build import build
        build()
    return bm25.LIB_PATH


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("bm25_index_build", "bm25_search_batch", "bm25_serve_submit", "bm25_serve_poll"):
        assert want in names


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\bT (bm25_[a-z_]+)\b", out))
    assert set(_declared()) <= exported


def test_binding_lists_every_declared_symbol(lib_path):
    from paper_2407_03618_amd import bm25
    assert sorted(bm25.EXPORTED) == _declared()
    lib = bm25.load_library()
    assert lib.bm25_last_error() == b""


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2407_03618_amd import bm25
    monkeypatch.setattr(bm25, "_lib", None)
    monkeypatch.setattr(bm25, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        bm25.load_library()


def test_null_index_is_rejected_without_device_work(lib_path):
    """Entry points taking an index reject NULL with BM25_E_INVAL and a message, before any
    device call (runs on a host without a GPU)."""
    from paper_2407_03618_amd import bm25
    lib = bm25.load_library()
    b = ctypes.c_int64()
    u = ctypes.c_int64()
    assert lib.bm25_search_set_graphs(None, 1) == bm25.E_INVAL
    assert b"NULL" in lib.bm25_last_error()
    assert lib.bm25_search_graph_stats(None, ctypes.byref(b), ctypes.byref(u)) == bm25.E_INVAL
    assert lib.bm25_search_set_plan(None, None) == bm25.E_INVAL
    assert lib.bm25_kernel_timing(None, 1) == bm25.E_INVAL
