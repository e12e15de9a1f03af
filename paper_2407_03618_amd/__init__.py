"""MI355X (gfx950) implementation of BM25S eager sparse scoring (arXiv 2407.03618).

The hot path lives in hand-written HIP kernels compiled into ``libbm25_mi355x.so`` (C ABI in
``include/bm25.h``); ``bm25`` is the thin ctypes binding. Build with
``python -m paper_2407_03618_amd.build``.
"""
from .bm25 import (  # noqa: F401
    BM25Error, Index, Server, Vocab, copy_bytes, load_library, LIB_PATH, VARIANTS, DTYPES, EXPORTED,
)
