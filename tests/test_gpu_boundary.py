"""Boundary behaviour: device memory through the caller's allocator, calls on several streams,
and the stored-score range counters."""
import numpy as np
import pytest

from oracle import eager
from tests.helpers import RTOL, check_batch
from workloads import make_corpus, make_queries

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _settled_allocated():
    """PyTorch's allocated bytes once earlier tests' garbage (tensors held by reference cycles,
    e.g. through exception tracebacks) is collected, so that only this test moves the count."""
    import gc
    import torch
    gc.collect()
    torch.cuda.synchronize()
    return torch.cuda.memory_allocated()


def test_torch_allocator_holds_the_index_memory():
    """With the default allocator every device byte of the index (arrays, then the search arena
    the first batch grows) comes from PyTorch's caching allocator, and free gives it back."""
    import torch
    from paper_2407_03618_amd import Index
    c = make_corpus(0, n_docs=20_000)
    q = make_queries(0, n_queries=64, vocab=c.vocab)
    tok, off, qd = _dev(c.tokens), _dev(c.doc_offsets), _dev(q.q_ids)
    out = (torch.empty((q.n, 10), dtype=torch.int32, device="cuda"),
           torch.empty((q.n, 10), dtype=torch.float32, device="cuda"),
           torch.empty(q.n, dtype=torch.int32, device="cuda"))
    before = _settled_allocated()
    idx = Index(tok, off, c.vocab, 1.5, 0.75, 0.0, "lucene", "f16")
    torch.cuda.synchronize()

    def held_by_library():
        live = idx._allocator.live
        # the library's live allocations are exactly its device bytes; the caching allocator
        # counts each of them rounded up, and a block whose unsplit remainder is under 1 MiB
        # whole
        assert sum(live.values()) == idx.device_bytes(), (live, idx.device_bytes())
        held = torch.cuda.memory_allocated() - before
        assert idx.device_bytes() <= held <= idx.device_bytes() + len(live) * (1 << 20), held

    held_by_library()
    idx.search_batch(qd, q.q_offsets, 10, 10, out=out)
    idx.search_plain(qd, q.q_offsets, 10, 10, out=out)
    torch.cuda.synchronize()
    held_by_library()
    idx.free()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before


def test_hip_malloc_without_allocator():
    """allocator=None: the library calls hipMalloc, PyTorch's count does not move, and the
    results are those of the default allocator."""
    import torch
    from paper_2407_03618_amd import Index
    c = make_corpus(0, n_docs=5_000)
    q = make_queries(0, n_queries=32, vocab=c.vocab)
    tok, off, qd = _dev(c.tokens), _dev(c.doc_offsets), _dev(q.q_ids)
    before = _settled_allocated()
    a = Index(tok, off, c.vocab, 1.5, 0.75, 0.0, "lucene", "f32", allocator=None)
    assert torch.cuda.memory_allocated() == before
    b = Index(tok, off, c.vocab, 1.5, 0.75, 0.0, "lucene", "f32")
    ea, eb = a.export(), b.export()
    for key in ("indptr", "indices", "tf", "df", "data"):
        assert torch.equal(ea[key], eb[key]), key
    ra = [t.cpu().numpy() for t in a.search_batch(qd, q.q_offsets, 10, 10)]
    rb = [t.cpu().numpy() for t in b.search_batch(qd, q.q_offsets, 10, 10)]
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab, 1.5, 0.75, 0.0, "lucene",
                            token_subset=np.unique(q.q_ids))
    for r, name in ((ra, "hipMalloc"), (rb, "torch")):
        check_batch(ref, q.q_ids, q.q_offsets, np.full(q.n, 10), *r, RTOL["f32"], name)
    a.free()
    b.free()


@pytest.mark.parametrize("form", ["batch", "plain"])
def test_back_to_back_calls_on_two_streams(form):
    """Two calls on different streams with no synchronisation between them share the index's
    scratch: the second waits for the first on the device, so both agree with the oracle and
    with their solo results (up to the summation order of the LDS float atomics, which varies
    from run to run)."""
    import torch
    from paper_2407_03618_amd import Index
    c = make_corpus(0, n_docs=30_000)
    qa = make_queries(0, n_queries=96, vocab=c.vocab)
    qb = make_queries(2, n_queries=40, vocab=c.vocab)
    idx = Index(_dev(c.tokens), _dev(c.doc_offsets), c.vocab, 1.5, 0.75, 0.0, "lucene", "f32")
    fn = idx.search_batch if form == "batch" else idx.search_plain
    da, db = _dev(qa.q_ids), _dev(qb.q_ids)
    solo_a = [t.cpu() for t in fn(da, qa.q_offsets, 10, 10)]
    solo_b = [t.cpu() for t in fn(db, qb.q_offsets, 100, 100)]
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab, 1.5, 0.75, 0.0, "lucene",
                            token_subset=np.unique(np.concatenate([qa.q_ids, qb.q_ids])))
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for rep in range(3):
        with torch.cuda.stream(s1):
            ra = fn(da, qa.q_offsets, 10, 10, stream=s1)
        with torch.cuda.stream(s2):
            rb = fn(db, qb.q_offsets, 100, 100, stream=s2)
        torch.cuda.synchronize()
        for res, solo, q, k, name in ((ra, solo_a, qa, 10, "A"), (rb, solo_b, qb, 100, "B")):
            ids, sc, cnt = (t.cpu() for t in res)
            assert torch.equal(cnt, solo[2])
            torch.testing.assert_close(sc, solo[1], rtol=1e-6, atol=0)
            check_batch(ref, q.q_ids, q.q_offsets, np.full(q.n, k), ids.numpy(), sc.numpy(),
                        cnt.numpy(), RTOL["f32"], f"stream {name} rep {rep}")
    idx.free()


def _range(docs, vocab, k1, b, variant, dtype):
    import torch
    from paper_2407_03618_amd import Index
    tokens = np.array([t for d in docs for t in d], dtype=np.int32)
    off = np.zeros(len(docs) + 1, np.int64)
    off[1:] = np.cumsum([len(d) for d in docs])
    idx = Index(_dev(tokens), _dev(off), vocab, k1, b, 0.0, variant, dtype)
    torch.cuda.synchronize()
    r = idx.range_stats()
    nnz = idx.nnz
    idx.free()
    return r, nnz


def test_range_counters():
    """Stored values below the fp16 normal range, rounded to zero, or above its largest finite
    value are counted at build (the values here sit far from every rounding boundary)."""
    docs = [[0, 1, 0], [1, 2], [0, 3, 3, 3]]
    # k1 = 1e9: every S is about 1e-9 * IDF * TF < 5e-9, below half the smallest fp16 subnormal
    r, nnz = _range(docs, 4, 1e9, 0.75, "lucene", "f16")
    assert r == {"subnormal": 0, "flushed_to_zero": nnz, "overflow": 0}
    # k1 = 1e5, b = 0: S is about 1e-5 * IDF * TF, between 4e-6 and 4.2e-5: fp16 subnormals
    r, nnz = _range(docs, 4, 1e5, 0.0, "lucene", "f16")
    assert r == {"subnormal": nnz, "flushed_to_zero": 0, "overflow": 0}
    # the same values are normal in bf16 and FP32
    for dt in ("bf16", "f32"):
        r, _ = _range(docs, 4, 1e9, 0.75, "lucene", dt)
        assert r == {"subnormal": 0, "flushed_to_zero": 0, "overflow": 0}
    # ATIRE with k1 = 1e6, b = 0: S(0, D0) = ln 3 * (1e6 + 1) * 1e5 / (1e5 + 1e6), about 9.99e4,
    # above 65504; the two other pairs score about 0.41
    r, _ = _range([[0] * 100_000, [1], [1]], 2, 1e6, 0.0, "atire", "f16")
    assert r == {"subnormal": 0, "flushed_to_zero": 0, "overflow": 1}
    r, _ = _range([[0] * 100_000, [1], [1]], 2, 1e6, 0.0, "atire", "bf16")
    assert r == {"subnormal": 0, "flushed_to_zero": 0, "overflow": 0}
