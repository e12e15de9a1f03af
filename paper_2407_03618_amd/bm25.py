"""Python binding of the gfx950 BM25S library (``libbm25_mi355x.so``) through ctypes.

Argument marshalling only: every step of index build and search runs in the library's HIP
kernels. PyTorch supplies device memory (tensors, and by default the index's own arrays and
scratch through a ``bm25_allocator`` backed by PyTorch's caching allocator) and streams
(``torch.cuda.current_stream()``). Importing this module does not need a GPU; creating an index
does, and fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
import sys
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbm25_mi355x.so")

LUCENE, BM25L, BM25PLUS, ROBERTSON, ATIRE, TFLDP = range(6)
VARIANTS = {"lucene": LUCENE, "bm25l": BM25L, "bm25plus": BM25PLUS, "robertson": ROBERTSON,
            "atire": ATIRE, "tfldp": TFLDP}
F32, F16, BF16 = range(3)
DTYPES = {"f32": F32, "f16": F16, "bf16": BF16}
MAX_K = 1024
MAX_QUERY_LEN = 2048

OK, E_INVAL, E_RANGE, E_NOMEM, E_BUSY, E_HIP, E_STATE, E_TIMEOUT = 0, -1, -2, -3, -4, -5, -6, -7

# every symbol include/bm25.h declares
EXPORTED = (
    "bm25_index_build", "bm25_index_info", "bm25_index_export", "bm25_index_device_bytes",
    "bm25_index_range_stats", "bm25_index_free", "bm25_search_batch",
    "bm25_search_batch_noalloc", "bm25_search_plain", "bm25_search_set_plan",
    "bm25_search_get_plan", "bm25_search_set_graphs", "bm25_search_graph_stats",
    "bm25_autotune", "bm25_kernel_timing", "bm25_kernel_time_read",
    "bm25_serve_create", "bm25_serve_submit", "bm25_serve_poll", "bm25_serve_stats",
    "bm25_serve_replay", "bm25_serve_destroy", "bm25_copy_bytes", "bm25_last_error",
    "bm25_tokenize_corpus", "bm25_vocab_info", "bm25_vocab_corpus", "bm25_vocab_words",
    "bm25_vocab_map", "bm25_vocab_free",
)
TOK_LOWERCASE = 1


class Params(ctypes.Structure):
    _fields_ = [("k1", ctypes.c_double), ("b", ctypes.c_double), ("delta", ctypes.c_double),
                ("variant", ctypes.c_int32), ("store_dtype", ctypes.c_int32)]


class TilePlan(ctypes.Structure):
    _fields_ = [("q_tile", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("doc_tile", ctypes.c_int32), ("doc_groups", ctypes.c_int32),
                ("query_order", ctypes.c_int32), ("sparse_only", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class ServeConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("max_k", ctypes.c_int32),
                ("n_streams", ctypes.c_int32)]


class ServeCounters(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("rejected_busy", ctypes.c_int64),
                ("rejected_nomem", ctypes.c_int64), ("max_batch_seen", ctypes.c_int32),
                ("waiting", ctypes.c_int32), ("lanes_busy", ctypes.c_int32),
                ("max_lanes_busy", ctypes.c_int32), ("lane_busy_s", ctypes.c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


class TorchAllocator:
    """bm25_allocator backed by PyTorch's caching allocator on one device: the library's device
    memory shows up in torch.cuda.memory_allocated() and is reused by PyTorch once freed."""

    def __init__(self, device: int):
        self.device = int(device)
        self._alloc = ALLOC_FN(self._alloc_cb)
        self._free = FREE_FN(self._free_cb)
        self.struct = Allocator(self._alloc, self._free, None)
        self.live = {}  # pointer -> bytes of the allocations the library holds

    def _alloc_cb(self, nbytes, stream, ctx):
        # the raw stream handle (0 = null stream) is the stream the library uses the memory on
        try:
            torch = _torch()
            p = int(torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                       int(stream or 0)))
        except Exception:  # out of memory: the library reports BM25_E_NOMEM
            return None
        self.live[p] = int(nbytes)
        return p

    def _free_cb(self, ptr, stream, ctx):
        if ptr:
            self.live.pop(int(ptr), None)
            _torch().cuda.caching_allocator_delete(int(ptr))


class BM25Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bm25 error {code}: {msg}")
        self.code = code


_lib = None


def load_library() -> ctypes.CDLL:
    """Loads the built library (raises if it is missing) and declares the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2407_03618_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.bm25_index_build.argtypes = [vp, i64, vp, i64, i32, P(Params), P(Allocator), vp, P(vp)]
    L.bm25_index_range_stats.argtypes = [vp, P(i64), P(i64), P(i64)]
    L.bm25_index_info.argtypes = [vp, P(i64), P(i32), P(i64), P(i64), P(dbl), P(Params)]
    L.bm25_index_export.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.bm25_index_device_bytes.argtypes = [vp]
    L.bm25_index_device_bytes.restype = i64
    L.bm25_index_free.argtypes = [vp]
    L.bm25_index_free.restype = None
    for fn in (L.bm25_search_batch, L.bm25_search_plain, L.bm25_search_batch_noalloc):
        fn.argtypes = [vp, vp, vp, i32, vp, i32, vp, vp, vp, vp]
    L.bm25_search_set_plan.argtypes = [vp, P(TilePlan)]
    L.bm25_search_get_plan.argtypes = [vp, i32, i32, i32, P(TilePlan)]
    L.bm25_search_set_graphs.argtypes = [vp, i32]
    L.bm25_search_graph_stats.argtypes = [vp, P(i64), P(i64)]
    L.bm25_autotune.argtypes = [vp, vp, vp, i32, vp, i32, vp, vp, vp, vp, P(TilePlan)]
    L.bm25_kernel_timing.argtypes = [vp, i32]
    L.bm25_kernel_time_read.argtypes = [vp, P(dbl), P(i64)]
    L.bm25_serve_create.argtypes = [vp, P(ServeConfig), P(vp)]
    L.bm25_serve_submit.argtypes = [vp, vp, i32, i32, P(ctypes.c_uint64)]
    L.bm25_serve_poll.argtypes = [vp, vp, vp, vp, vp, i32, i32, i64]
    L.bm25_serve_stats.argtypes = [vp, P(ServeCounters)]
    L.bm25_serve_replay.argtypes = [vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, i32]
    L.bm25_serve_destroy.argtypes = [vp]
    L.bm25_copy_bytes.argtypes = [vp, vp, i64, vp]
    L.bm25_last_error.argtypes = []
    L.bm25_last_error.restype = ctypes.c_char_p
    L.bm25_tokenize_corpus.argtypes = [vp, i64, vp, i64, i32, P(Allocator), vp, P(vp), P(i64),
                                       P(i32)]
    L.bm25_vocab_info.argtypes = [vp, P(i64), P(i64), P(i32), P(i64), P(i32)]
    L.bm25_vocab_corpus.argtypes = [vp, vp, vp, vp]
    L.bm25_vocab_words.argtypes = [vp, vp, vp, vp]
    L.bm25_vocab_map.argtypes = [vp, vp, i64, vp, i64, vp, i64, vp, P(i64), vp]
    L.bm25_vocab_free.argtypes = [vp]
    L.bm25_vocab_free.restype = None
    _lib = L
    return L


def _check(rc: int) -> int:
    if rc < 0:
        msg = load_library().bm25_last_error().decode(errors="replace")
        raise BM25Error(rc, msg)
    return rc


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _host_i64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int64))


def _host_i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def copy_bytes(dst, src, n_bytes: int, stream=None) -> None:
    """Device copy of n_bytes through the library's plain copy kernel (calibration)."""
    _check(load_library().bm25_copy_bytes(_ptr(dst), _ptr(src), int(n_bytes),
                                          _stream_ptr(stream)))


class Index:
    """A BM25S index resident in device memory, built by the library's HIP kernels."""

    def __init__(self, token_ids, doc_offsets, vocab: int, k1: float = 1.5, b: float = 0.75,
                 delta: float = 0.0, variant="lucene", dtype="f32", stream=None,
                 allocator: str = "torch"):
        """allocator: "torch" (the index's device memory comes from PyTorch's caching allocator)
        or None (the library calls hipMalloc)."""
        torch = _torch()
        L = load_library()
        if not (token_ids.is_cuda and doc_offsets.is_cuda):
            raise ValueError("token_ids and doc_offsets must be device tensors")
        if token_ids.dtype != torch.int32 or doc_offsets.dtype != torch.int64:
            raise ValueError("token_ids must be int32 and doc_offsets int64")
        token_ids = token_ids.contiguous()
        doc_offsets = doc_offsets.contiguous()
        var = VARIANTS[variant] if isinstance(variant, str) else int(variant)
        dt = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        self.params = Params(float(k1), float(b), float(delta), var, dt)
        if allocator not in ("torch", None):
            raise ValueError("allocator must be 'torch' or None")
        # the callbacks must outlive the index: they are called again by free()
        self._allocator = TorchAllocator(token_ids.device.index) if allocator else None
        h = ctypes.c_void_p()
        rc = L.bm25_index_build(_ptr(token_ids), token_ids.numel(), _ptr(doc_offsets),
                                doc_offsets.numel() - 1, int(vocab), ctypes.byref(self.params),
                                ctypes.byref(self._allocator.struct) if self._allocator else None,
                                _stream_ptr(stream), ctypes.byref(h))
        _check(rc)
        self._h = h
        self.vocab = int(vocab)
        self.dtype = dt
        self.variant = var
        n = ctypes.c_int64()
        nnz = ctypes.c_int64()
        sl = ctypes.c_int64()
        la = ctypes.c_double()
        _check(L.bm25_index_info(self._h, ctypes.byref(n), None, ctypes.byref(nnz),
                                 ctypes.byref(sl), ctypes.byref(la), None))
        self.n_docs, self.nnz, self.sum_len, self.l_avg = n.value, nnz.value, sl.value, la.value

    @property
    def handle(self):
        return self._h

    def free(self) -> None:
        if getattr(self, "_h", None):
            load_library().bm25_index_free(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit the allocator callbacks can no longer run: leave the memory to
        # the process teardown (the check is bound here: module globals may be gone by then)
        if _finalizing():
            return
        try:
            self.free()
        except Exception:
            pass

    def device_bytes(self) -> int:
        return int(load_library().bm25_index_device_bytes(self._h))

    def range_stats(self) -> dict:
        """Stored values rounded to a subnormal, from non-zero to zero, and to infinity."""
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(load_library().bm25_index_range_stats(self._h, ctypes.byref(a), ctypes.byref(b),
                                                     ctypes.byref(c)))
        return {"subnormal": a.value, "flushed_to_zero": b.value, "overflow": c.value}

    def export(self, stream=None) -> dict:
        """Device copies of indptr, indices, tf, df, idf, theta and data."""
        torch = _torch()
        dev = torch.device("cuda")
        V, nnz = self.vocab, self.nnz
        out = {
            "indptr": torch.empty(V + 1, dtype=torch.int64, device=dev),
            "indices": torch.empty(max(nnz, 1), dtype=torch.int32, device=dev),
            "tf": torch.empty(max(nnz, 1), dtype=torch.int32, device=dev),
            "df": torch.empty(V, dtype=torch.int32, device=dev),
            "idf": torch.empty(V, dtype=torch.float64, device=dev),
            "theta": torch.empty(V, dtype=torch.float64, device=dev),
        }
        if self.dtype == F32:
            out["data"] = torch.empty(max(nnz, 1), dtype=torch.float32, device=dev)
        elif self.dtype == F16:
            out["data"] = torch.empty(max(nnz, 1), dtype=torch.float16, device=dev)
        else:
            out["data"] = torch.empty(max(nnz, 1), dtype=torch.bfloat16, device=dev)
        _check(load_library().bm25_index_export(
            self._h, _ptr(out["indptr"]), _ptr(out["indices"]), _ptr(out["tf"]),
            _ptr(out["df"]), _ptr(out["idf"]), _ptr(out["theta"]), _ptr(out["data"]),
            _stream_ptr(stream)))
        for key in ("indices", "tf", "data"):
            out[key] = out[key][:nnz]
        return out

    def _outputs(self, n: int, k_max: int, out=None):
        torch = _torch()
        if out is not None:
            return out
        dev = torch.device("cuda")
        return (torch.empty((n, k_max), dtype=torch.int32, device=dev),
                torch.empty((n, k_max), dtype=torch.float32, device=dev),
                torch.empty(n, dtype=torch.int32, device=dev))

    def _search(self, fn, q_ids, q_offsets, k, k_max, out, stream):
        q_off = _host_i64(q_offsets)
        n = q_off.shape[0] - 1
        if k is None:
            k_arr = None
        elif np.isscalar(k):
            k_arr = np.full(n, int(k), dtype=np.int32)
        else:
            k_arr = _host_i32(k)
        if k_max is None:
            k_max = int(k_arr.max()) if (k_arr is not None and n > 0) else 10
        ids, scores, count = self._outputs(n, k_max, out)
        rc = fn(self._h, _ptr(q_ids), q_off.ctypes.data, n,
                None if k_arr is None else k_arr.ctypes.data, int(k_max), _ptr(ids),
                _ptr(scores), _ptr(count), _stream_ptr(stream))
        _check(rc)
        return ids, scores, count

    def search_batch(self, q_ids, q_offsets, k=None, k_max=None, out=None, stream=None):
        """Batched form. q_ids: device int32; q_offsets: host int64[n+1]; k: int or int32[n]."""
        return self._search(load_library().bm25_search_batch, q_ids, q_offsets, k, k_max, out,
                            stream)

    def search_batch_noalloc(self, q_ids, q_offsets, k=None, k_max=None, out=None,
                             stream=None):
        """Batched form on the library's fixed scratch: allocates nothing (pass `out` to keep
        the call itself free of allocations)."""
        return self._search(load_library().bm25_search_batch_noalloc, q_ids, q_offsets, k, k_max,
                            out, stream)

    def search_plain(self, q_ids, q_offsets, k=None, k_max=None, out=None, stream=None):
        """Per-query form (one sweep launch per query)."""
        return self._search(load_library().bm25_search_plain, q_ids, q_offsets, k, k_max, out,
                            stream)

    def set_plan(self, plan: Optional[dict]) -> None:
        L = load_library()
        if plan is None:
            _check(L.bm25_search_set_plan(self._h, None))
            return
        p = TilePlan(int(plan.get("q_tile", 0)), int(plan.get("waves", 0)),
                     int(plan.get("doc_tile", 0)), int(plan.get("doc_groups", 0)),
                     int(plan.get("query_order", 0)), int(plan.get("sparse_only", 0)))
        _check(L.bm25_search_set_plan(self._h, ctypes.byref(p)))

    def get_plan(self, n_queries: int, max_query_len: int, k_max: int) -> dict:
        p = TilePlan()
        _check(load_library().bm25_search_get_plan(self._h, int(n_queries), int(max_query_len),
                                                   int(k_max), ctypes.byref(p)))
        return p.as_dict()

    def autotune(self, q_ids, q_offsets, k=None, k_max=None, stream=None) -> dict:
        q_off = _host_i64(q_offsets)
        n = q_off.shape[0] - 1
        k_arr = None if k is None else (np.full(n, int(k), np.int32) if np.isscalar(k)
                                        else _host_i32(k))
        if k_max is None:
            k_max = int(k_arr.max()) if k_arr is not None else 10
        ids, scores, count = self._outputs(n, k_max)
        best = TilePlan()
        _check(load_library().bm25_autotune(
            self._h, _ptr(q_ids), q_off.ctypes.data, n,
            None if k_arr is None else k_arr.ctypes.data, int(k_max), _ptr(ids), _ptr(scores),
            _ptr(count), _stream_ptr(stream), ctypes.byref(best)))
        return best.as_dict()

    def set_graphs(self, enable: bool) -> None:
        """Graph mode: each later batched search (and server micro-batch) is one HIP graph
        launch."""
        _check(load_library().bm25_search_set_graphs(self._h, 1 if enable else 0))

    def graph_stats(self) -> dict:
        b = ctypes.c_int64()
        u = ctypes.c_int64()
        _check(load_library().bm25_search_graph_stats(self._h, ctypes.byref(b), ctypes.byref(u)))
        return {"builds": b.value, "updates": u.value}

    def kernel_timing(self, enable: bool) -> None:
        _check(load_library().bm25_kernel_timing(self._h, 1 if enable else 0))

    def kernel_time_read(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(load_library().bm25_kernel_time_read(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


class Server:
    """Continuous-batching server over a resident index (host-side requests)."""

    def __init__(self, index: Index, hbm_budget_bytes: int = 1 << 30, max_slots: int = 65536,
                 max_batch: int = 4096, max_k: int = 1000, n_streams: int = 2):
        self.index = index
        self.cfg = ServeConfig(int(hbm_budget_bytes), int(max_slots), int(max_batch), int(max_k),
                               int(n_streams))
        self.max_k = int(max_k)
        h = ctypes.c_void_p()
        _check(load_library().bm25_serve_create(index.handle, ctypes.byref(self.cfg),
                                                ctypes.byref(h)))
        self._h = h

    def submit(self, ids, k: int) -> int:
        a = _host_i32(ids)
        t = ctypes.c_uint64()
        _check(load_library().bm25_serve_submit(self._h, a.ctypes.data if a.size else None,
                                                a.size, int(k), ctypes.byref(t)))
        return int(t.value)

    def poll(self, max_results: int = 256, timeout_us: int = 0, k_stride: Optional[int] = None):
        """List of (ticket, count, ids[k_stride], scores[k_stride]); empty on timeout."""
        ks = int(k_stride or self.max_k)
        tickets = np.zeros(max_results, np.uint64)
        counts = np.zeros(max_results, np.int32)
        ids = np.zeros((max_results, ks), np.int32)
        scores = np.zeros((max_results, ks), np.float32)
        rc = load_library().bm25_serve_poll(self._h, tickets.ctypes.data, ids.ctypes.data,
                                            scores.ctypes.data, counts.ctypes.data, max_results,
                                            ks, int(timeout_us))
        if rc == E_TIMEOUT:
            return []
        _check(rc)
        return [(int(tickets[i]), int(counts[i]), ids[i], scores[i]) for i in range(rc)]

    def stats(self) -> dict:
        c = ServeCounters()
        _check(load_library().bm25_serve_stats(self._h, ctypes.byref(c)))
        return {f: getattr(c, f) for f, _ in ServeCounters._fields_}

    def replay(self, q_ids, q_offsets, k, arrival_us, k_stride: Optional[int] = None,
               keep_results: bool = True):
        """Open-loop replay; returns (latency_us[n], queue_us[n], ids[n, k_stride], scores,
        counts). queue_us is the wait before admission into a micro-batch. With
        keep_results=False the result rows are not kept (ids and scores are None)."""
        q = _host_i32(q_ids)
        off = _host_i64(q_offsets)
        n = off.shape[0] - 1
        kk = _host_i32(np.broadcast_to(np.asarray(k), (n,)))
        arr = np.ascontiguousarray(np.asarray(arrival_us, dtype=np.float64))
        ks = int(k_stride or self.max_k)
        lat = np.full(n, np.nan)
        queue = np.full(n, np.nan)
        ids = np.zeros((n, ks), np.int32) if keep_results else None
        scores = np.zeros((n, ks), np.float32) if keep_results else None
        counts = np.zeros(n, np.int32)
        rc = load_library().bm25_serve_replay(
            self._h, q.ctypes.data if q.size else None, off.ctypes.data, kk.ctypes.data,
            arr.ctypes.data, n, lat.ctypes.data, queue.ctypes.data,
            ids.ctypes.data if keep_results else None,
            scores.ctypes.data if keep_results else None, counts.ctypes.data, ks)
        _check(rc)
        return lat, queue, ids, scores, counts

    def close(self) -> None:
        if getattr(self, "_h", None):
            _check(load_library().bm25_serve_destroy(self._h))
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Vocab:
    """Tokenized corpus and its word dictionary, built by the library's kernels from device
    UTF-8 text (Section 2, "Tokenization")."""

    def __init__(self, text, doc_offsets, lowercase: bool = False, stream=None,
                 allocator: str = "torch"):
        torch = _torch()
        L = load_library()
        if not (text.is_cuda and doc_offsets.is_cuda):
            raise ValueError("text and doc_offsets must be device tensors")
        if text.dtype != torch.uint8 or doc_offsets.dtype != torch.int64:
            raise ValueError("text must be uint8 and doc_offsets int64")
        text = text.contiguous()
        doc_offsets = doc_offsets.contiguous()
        self._allocator = TorchAllocator(text.device.index) if allocator else None
        h = ctypes.c_void_p()
        nt = ctypes.c_int64()
        nv = ctypes.c_int32()
        _check(L.bm25_tokenize_corpus(
            _ptr(text), text.numel(), _ptr(doc_offsets), doc_offsets.numel() - 1,
            TOK_LOWERCASE if lowercase else 0,
            ctypes.byref(self._allocator.struct) if self._allocator else None,
            _stream_ptr(stream), ctypes.byref(h), ctypes.byref(nt), ctypes.byref(nv)))
        self._h = h
        self.n_docs = doc_offsets.numel() - 1
        self.n_tokens = nt.value
        self.vocab_size = nv.value
        self.lowercase = bool(lowercase)

    def corpus(self, stream=None):
        """(token_ids int32[n_tokens], doc_offsets int64[n_docs + 1]) on the device."""
        torch = _torch()
        ids = torch.empty(max(self.n_tokens, 1), dtype=torch.int32, device="cuda")
        off = torch.empty(self.n_docs + 1, dtype=torch.int64, device="cuda")
        _check(load_library().bm25_vocab_corpus(self._h, _ptr(ids), _ptr(off),
                                                _stream_ptr(stream)))
        return ids[:self.n_tokens], off

    def words(self, stream=None) -> list:
        """The words by id (host strings)."""
        torch = _torch()
        nb = ctypes.c_int64()
        _check(load_library().bm25_vocab_info(self._h, None, None, None, ctypes.byref(nb), None))
        off = torch.empty(self.vocab_size + 1, dtype=torch.int32, device="cuda")
        data = torch.empty(max(nb.value, 1), dtype=torch.uint8, device="cuda")
        _check(load_library().bm25_vocab_words(self._h, _ptr(off), _ptr(data),
                                               _stream_ptr(stream)))
        torch.cuda.synchronize()
        o = off.cpu().numpy().view(np.uint32).astype(np.int64)
        b = data.cpu().numpy().tobytes()
        return [b[o[i]:o[i + 1]].decode("utf-8") for i in range(self.vocab_size)]

    def map(self, text, offsets, stream=None):
        """Ids of the texts' words (device int32) and per-text offsets (device int64[n+1])."""
        torch = _torch()
        L = load_library()
        n = offsets.numel() - 1
        id_off = torch.empty(n + 1, dtype=torch.int64, device="cuda")
        cnt = ctypes.c_int64()
        cap = max(1, text.numel() // 2 + 1)  # a word takes at least two bytes
        ids = torch.empty(cap, dtype=torch.int32, device="cuda")
        _check(L.bm25_vocab_map(self._h, _ptr(text), text.numel(), _ptr(offsets), n, _ptr(ids),
                                cap, _ptr(id_off), ctypes.byref(cnt), _stream_ptr(stream)))
        return ids[:cnt.value], id_off

    def free(self) -> None:
        if getattr(self, "_h", None):
            load_library().bm25_vocab_free(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.free()
        except Exception:
            pass
