"""The allocation-free batched search (bm25_search_batch_noalloc), called through the C ABI, against
bm25_search_batch on the same batches: two calls in a row, the second smaller, and a batch too
large for its fixed scratch."""
import ctypes

import numpy as np
import pytest

from workloads import make_corpus, make_queries

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _call(fn, idx, qd, q_off, k, k_max, out):
    import torch
    q_off = np.ascontiguousarray(q_off, dtype=np.int64)
    n = q_off.shape[0] - 1
    kk = np.ascontiguousarray(np.broadcast_to(np.asarray(k, dtype=np.int32), (n,)))
    rc = fn(idx.handle, qd.data_ptr(), q_off.ctypes.data, n, kk.ctypes.data, k_max,
            out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(),
            torch.cuda.current_stream().cuda_stream)
    return rc


def _agree(got, ref, rtol=1e-6):
    """Same counts; scores equal up to the summation order of the LDS float atomics; ids equal
    except among scores that tie within that tolerance."""
    gi, gs, gc = (t.cpu().numpy() for t in got)
    ri, rs, rc = (t.cpu().numpy() for t in ref)
    np.testing.assert_array_equal(gc, rc)
    np.testing.assert_allclose(gs, rs, rtol=rtol, atol=0)
    for q in range(gc.shape[0]):
        n = int(gc[q])
        for p in np.flatnonzero(gi[q, :n] != ri[q, :n]):
            s = rs[q, :n]
            assert np.sum(np.abs(s - s[p]) <= rtol * abs(s[p])) >= 2, (q, p)
    assert np.all(gi[:, :][gs == -np.inf] == -1)


def test_noalloc_matches_batched_search_twice_then_smaller():
    import torch
    from paper_2407_03618_amd import Index, bm25
    lib = bm25.load_library()
    c = make_corpus(2, n_docs=200_000)
    q = make_queries(2, n_queries=1024, vocab=c.vocab)
    idx = Index(_dev(c.tokens), _dev(c.doc_offsets), c.vocab, 1.5, 0.75, 0.0, "lucene", "f16")
    qd = _dev(q.q_ids)
    rng = np.random.default_rng(5)
    ks = rng.choice([10, 100], size=q.n).astype(np.int32)
    # first the smaller call's reference, so the index's own arena is already sized
    for n, k_max in ((1024, 100), (300, 64)):
        off = q.q_offsets[:n + 1]
        kk = np.minimum(ks[:n], k_max)
        ref = [torch.empty((n, k_max), dtype=torch.int32, device="cuda"),
               torch.empty((n, k_max), dtype=torch.float32, device="cuda"),
               torch.empty(n, dtype=torch.int32, device="cuda")]
        assert _call(lib.bm25_search_batch, idx, qd, off, kk, k_max, ref) == 0
    del ref
    import gc
    gc.collect()  # earlier tests' cyclic garbage must not be freed inside the measured span
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated()
    idx_bytes = idx.device_bytes()
    for n, k_max in ((1024, 100), (300, 64)):   # two calls in a row, the second smaller
        off = q.q_offsets[:n + 1]
        kk = np.minimum(ks[:n], k_max)
        ref = [torch.empty((n, k_max), dtype=torch.int32, device="cuda"),
               torch.empty((n, k_max), dtype=torch.float32, device="cuda"),
               torch.empty(n, dtype=torch.int32, device="cuda")]
        got = [torch.full_like(t, 7) for t in ref]
        base = torch.cuda.memory_allocated()
        assert _call(lib.bm25_search_batch_noalloc, idx, qd, off, kk, k_max, got) == 0, \
            lib.bm25_last_error()
        assert _call(lib.bm25_search_batch, idx, qd, off, kk, k_max, ref) == 0
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == base
        _agree(got, ref)
        assert int(got[2].min()) > 0
        del ref, got
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == held
    assert idx.device_bytes() == idx_bytes
    idx.free()


def test_noalloc_refuses_a_batch_past_its_scratch():
    import torch
    from paper_2407_03618_amd import Index, bm25
    lib = bm25.load_library()
    c = make_corpus(2, n_docs=50_000)
    q = make_queries(2, n_queries=4096, vocab=c.vocab)
    idx = Index(_dev(c.tokens), _dev(c.doc_offsets), c.vocab, 1.5, 0.75, 0.0, "lucene", "f16")
    qd = _dev(q.q_ids)
    out = [torch.empty((q.n, 1000), dtype=torch.int32, device="cuda"),
           torch.empty((q.n, 1000), dtype=torch.float32, device="cuda"),
           torch.empty(q.n, dtype=torch.int32, device="cuda")]
    # 4096 queries with lists of 1024 keys need far more candidate-list scratch than 64 MiB
    rc = _call(lib.bm25_search_batch_noalloc, idx, qd, q.q_offsets, 1000, 1000, out)
    assert rc == bm25.E_NOMEM
    assert b"scratch" in lib.bm25_last_error()
    idx.free()
