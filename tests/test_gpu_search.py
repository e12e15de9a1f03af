"""GPU search (batched and per-query forms) against the FP64 oracle."""
import numpy as np
import pytest

from oracle import eager
from tests.helpers import RTOL, check_batch
from workloads import make_corpus, make_queries, make_tiny_corpus, make_tiny_queries
from workloads.synth import QueryBatch

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _index(c, variant="lucene", k1=1.5, b=0.75, delta=0.0, dtype="f32"):
    from paper_2407_03618_amd import Index
    return Index(_dev(c.tokens), _dev(c.doc_offsets), c.vocab, k1, b, delta, variant, dtype)


def _run(idx, qb, k_max, form):
    import torch
    fn = idx.search_batch if form == "batch" else idx.search_plain
    ids, scores, counts = fn(_dev(qb.q_ids) if qb.q_ids.size else _dev(np.zeros(1, np.int32)),
                             qb.q_offsets, qb.k, k_max)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), scores.cpu().numpy(), counts.cpu().numpy()


@pytest.fixture(scope="module")
def cfg0():
    c = make_corpus(0)
    q = make_queries(0)
    return c, q


@pytest.mark.parametrize("form", ["batch", "plain"])
@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_config0_all_queries(cfg0, form, dtype):
    c, q = cfg0
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab, 1.5, 0.75, 0.0, "lucene")
    idx = _index(c, dtype=dtype)
    ids, sc, cnt = _run(idx, q, 10, form)
    check_batch(ref, q.q_ids, q.q_offsets, q.k, ids, sc, cnt, RTOL[dtype], f"{form}/{dtype}")


@pytest.mark.parametrize("dtype,reps", [("bf16", 300), ("bf16", 2047), ("f16", 2047),
                                        ("f32", 300)])
def test_repeated_dense_token(cfg0, dtype, reps):
    """A query repeating a dense-row token more often than the bf16 matrix-core operand holds
    exactly (2^8): the planner splits its multiplicity over several entries of the same row. In
    fp16 every multiplicity a query can have (at most 2048 ids) is exact, which the longest query
    checks. Neighbours in the batch share the row with other multiplicities."""
    c, _ = cfg0
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab, 1.5, 0.75, 0.0, "lucene")
    df = np.diff(ref.indptr)
    dense_tok = int(np.argmax(df))  # the most frequent token: a dense row at any threshold
    assert df[dense_tok] * 16 >= c.n_docs
    other = int(np.argsort(df)[-2])
    queries = [np.array([dense_tok] * reps + [other], np.int32),
               np.array([dense_tok, other], np.int32),
               np.array([dense_tok] * 3, np.int32),
               np.array([other] * reps, np.int32)]
    off = np.zeros(len(queries) + 1, np.int64)
    off[1:] = np.cumsum([q.size for q in queries])
    qb = QueryBatch(np.concatenate(queries), off, np.full(len(queries), 10, np.int32))
    idx = _index(c, dtype=dtype)
    ids, sc, cnt = _run(idx, qb, 10, "batch")
    check_batch(ref, qb.q_ids, qb.q_offsets, qb.k, ids, sc, cnt, RTOL[dtype], f"x{reps} {dtype}")
    idx.free()


VARIANTS = [("bm25plus", 1.2, 0.75, 1.0), ("bm25l", 1.2, 0.75, 0.5), ("robertson", 1.2, 0.75, 0.0),
            ("atire", 1.2, 0.75, 0.0), ("tfldp", 1.2, 0.75, 0.5), ("lucene", 0.9, 0.4, 0.0)]


@pytest.mark.parametrize("variant,k1,b,delta", VARIANTS)
@pytest.mark.parametrize("form", ["batch", "plain"])
def test_variants_config0(cfg0, variant, k1, b, delta, form):
    c, q = cfg0
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab, k1, b, delta, variant)
    for dtype in ("f32", "bf16"):
        idx = _index(c, variant, k1, b, delta, dtype)
        ids, sc, cnt = _run(idx, q, 10, form)
        check_batch(ref, q.q_ids, q.q_offsets, q.k, ids, sc, cnt, RTOL[dtype],
                    f"{variant}/{form}/{dtype}")
        idx.free()


@pytest.mark.parametrize("form", ["batch", "plain"])
def test_tiny_corpora_edge_cases(form):
    """Random tiny corpora: k > N, empty queries, repeated and absent tokens, empty documents."""
    for seed in range(30):
        c = make_tiny_corpus(seed)
        qb = make_tiny_queries(seed, c.vocab + 2)  # ids c.vocab.. are absent (DF = 0) ...
        qb.q_ids[:] = np.minimum(qb.q_ids, c.vocab + 1)
        from workloads.synth import Corpus
        cc = Corpus(c.tokens, c.doc_offsets, c.vocab + 2)  # ... but inside the vocabulary
        for variant, k1, b, delta in (("lucene", 1.5, 0.75, 0.0), ("bm25plus", 1.2, 0.75, 1.0)):
            ref = eager.build_index(cc.tokens, cc.doc_offsets, cc.vocab, k1, b, delta, variant)
            idx = _index(cc, variant, k1, b, delta, "f32")
            ids, sc, cnt = _run(idx, qb, 12, form)
            check_batch(ref, qb.q_ids, qb.q_offsets, qb.k, ids, sc, cnt, 1e-5,
                        f"seed {seed} {variant} {form}")
            idx.free()


@pytest.mark.parametrize("form", ["batch", "plain"])
def test_invalid_token_marks_only_that_query(form):
    c = make_corpus(0, n_docs=500)
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab)
    q_ids = np.array([1, 2, c.vocab + 7, 3, -1, 4, 5], np.int32)
    q_off = np.array([0, 2, 4, 5, 7], np.int64)
    qb = QueryBatch(q_ids, q_off, np.full(4, 5, np.int32))
    idx = _index(c)
    ids, sc, cnt = _run(idx, qb, 5, form)
    assert cnt[1] == -2 and cnt[2] == -2
    assert np.all(ids[1] == -1) and np.all(np.isneginf(sc[2]))
    for i in (0, 3):
        check_batch(ref, q_ids, q_off, 5, ids, sc, cnt, 1e-5, form, sample=[i])


def test_search_argument_errors():
    from paper_2407_03618_amd import BM25Error
    c = make_corpus(0, n_docs=300)
    idx = _index(c)
    q = _dev(np.array([1, 2, 3], np.int32))
    with pytest.raises(BM25Error):
        idx.search_batch(q, np.array([0, 3]), 5, 2000)           # k_max above the limit
    with pytest.raises(BM25Error):
        idx.search_batch(q, np.array([0, 3]), np.array([6]), 5)  # k > k_max
    with pytest.raises(BM25Error):
        idx.search_batch(q, np.array([1, 3]), 5, 5)              # offsets must start at 0
    with pytest.raises(BM25Error):
        idx.search_plain(q, np.array([0, 3, 2]), 5, 5)           # decreasing offsets


@pytest.mark.parametrize("form", ["batch", "plain"])
@pytest.mark.parametrize("k", [1, 100, 300, 1000])
def test_scaled_corpus_many_tiles_and_groups(form, k):
    """Recipe of the 8.8M-document workload at 120k documents: many doc tiles and groups with a
    ragged tail, query tiles with a ragged last tile, k from 1 to 1000."""
    c = make_corpus(2, n_docs=120_000)
    q = make_queries(2, n_queries=77 if k >= 300 else 150, vocab=c.vocab, k=k)
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab, token_subset=np.unique(q.q_ids))
    idx = _index(c, dtype="f16")
    ids, sc, cnt = _run(idx, q, k, form)
    sample = range(q.n) if k <= 100 else range(0, q.n, 5)
    check_batch(ref, q.q_ids, q.q_offsets, q.k, ids, sc, cnt, RTOL["f16"], f"{form} k={k}",
                sample=sample)


@pytest.mark.parametrize("groups", [2, 4, 8])
def test_long_lists_over_few_groups(groups):
    """1024-key lists at fp16 (the gather form held to 4 waves per SIMD) over few document groups,
    as the automatic shape gives large top-1000 batches; fewer than 8 groups take the plain
    block-to-group mapping. Per-query k mixes 1000 with shorter lists in the same batch."""
    c = make_corpus(2, n_docs=120_000)
    q0 = make_queries(2, n_queries=77, vocab=c.vocab, k=1000)
    kk = np.array([1000, 10, 100, 999, 1000, 257, 64], dtype=np.int32)[np.arange(q0.n) % 7]
    q = QueryBatch(q0.q_ids, q0.q_offsets, kk)
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab, token_subset=np.unique(q.q_ids))
    idx = _index(c, dtype="f16")
    idx.set_plan(dict(q_tile=4, waves=4, doc_tile=1024, doc_groups=groups))
    ids, sc, cnt = _run(idx, q, 1000, "batch")
    idx.set_plan(None)
    check_batch(ref, q.q_ids, q.q_offsets, q.k, ids, sc, cnt, RTOL["f16"], f"groups={groups}",
                sample=range(0, q.n, 4))


def test_batched_shapes_agree():
    """Every built launch shape, with and without the dense head rows, gives results within
    tolerance; invalid shapes are rejected."""
    import torch
    from paper_2407_03618_amd import BM25Error
    c = make_corpus(2, n_docs=60_000)
    q = make_queries(2, n_queries=90, vocab=c.vocab, k=50)
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab, token_subset=np.unique(q.q_ids))
    idx = _index(c, dtype="f32")
    for waves, dt in ((8, 1024), (4, 1024), (8, 2048)):
        for qt in (waves, 2 * waves, 4 * waves):
            if qt == 4 * waves and waves * dt // (64 * waves) > 16:
                continue
            for g, sparse_only in ((8, 0), (3, 1), (16, 0)):
                plan = dict(q_tile=qt, waves=waves, doc_tile=dt, doc_groups=g,
                            sparse_only=sparse_only)
                idx.set_plan(plan)
                ids, sc, cnt = _run(idx, q, 50, "batch")
                check_batch(ref, q.q_ids, q.q_offsets, q.k, ids, sc, cnt, 1e-5, str(plan),
                            sample=range(0, q.n, 3))
    for bad in (dict(q_tile=16, waves=8, doc_tile=512, doc_groups=8),
                dict(q_tile=12, waves=8, doc_tile=1024, doc_groups=8),
                dict(q_tile=4, waves=8, doc_tile=1024, doc_groups=8),
                dict(q_tile=16, waves=2, doc_tile=1024, doc_groups=8)):
        with pytest.raises(BM25Error) as e:
            idx.set_plan(bad)
        assert e.value.code == -1
    idx.set_plan(None)
    best = idx.autotune(_dev(q.q_ids), q.q_offsets, 50, 50)
    assert best["q_tile"] >= 1
    ids, sc, cnt = _run(idx, q, 50, "batch")
    check_batch(ref, q.q_ids, q.q_offsets, q.k, ids, sc, cnt, 1e-5, "tuned")
    torch.cuda.synchronize()


@pytest.mark.parametrize("form", ["batch", "plain"])
def test_sparse_only_matches_dense_path(form):
    """The dense copies of the head rows and the sparse rows give the same top-k."""
    import torch
    c = make_corpus(0)
    q = make_queries(0)
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab)
    idx = _index(c, dtype="f32")
    plan = idx.get_plan(q.n, int(np.diff(q.q_offsets).max()), 10)
    plan["sparse_only"] = 1
    idx.set_plan(plan)
    ids, sc, cnt = _run(idx, q, 10, form)
    check_batch(ref, q.q_ids, q.q_offsets, q.k, ids, sc, cnt, 1e-5, f"sparse-only {form}")
    torch.cuda.synchronize()


def test_query_order_grouped_matches_given():
    """Grouping the batch by frequent tokens (two sort windows, a ragged last tile, per-query k,
    an empty query, invalid ids) returns every query's own results in the caller's order; a
    batch whose longest query does not fit a grouped tile falls back to the given order."""
    import torch
    c = make_corpus(2, n_docs=60_000)
    q = make_queries(2, n_queries=4096 + 333, vocab=c.vocab, k=40)
    rng = np.random.default_rng(5)
    q.k[:] = rng.integers(1, 41, q.n).astype(np.int32)
    lens = np.diff(q.q_offsets)
    # query 7 empty; queries 11 and 4200 hold an id outside the vocabulary
    parts = [q.query(i) for i in range(q.n)]
    parts[7] = parts[7][:0]
    parts[11] = np.concatenate([parts[11], [c.vocab + 3]]).astype(np.int32)
    parts[4200] = np.concatenate([[-5], parts[4200]]).astype(np.int32)
    q_ids = np.concatenate(parts).astype(np.int32)
    q_off = np.zeros(q.n + 1, np.int64)
    q_off[1:] = np.cumsum([len(p) for p in parts])
    qb = QueryBatch(q_ids, q_off, q.k)
    ok_ids = q_ids[(q_ids >= 0) & (q_ids < c.vocab)]
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab, token_subset=np.unique(ok_ids))
    idx = _index(c, dtype="f16")
    sample = [i for i in range(0, q.n, 29) if i not in (11, 4200)] + [7, q.n - 1]
    out = {}
    for order in (2, 1):
        plan = idx.get_plan(q.n, int(lens.max()) + 1, 40)
        plan["query_order"] = order
        idx.set_plan(plan)
        ids, sc, cnt = _run(idx, qb, 40, "batch")
        assert cnt[11] == -2 and cnt[4200] == -2 and np.all(ids[11] == -1)
        check_batch(ref, q_ids, q_off, q.k, ids, sc, cnt, RTOL["f16"], f"order {order}",
                    sample=sample)
        out[order] = cnt
    assert np.array_equal(out[1], out[2])
    # longest query 600 ids: 8 queries per tile exceed the tile's positions, so no grouping
    long_q = rng.integers(0, c.vocab, 600).astype(np.int32)
    parts2 = [long_q] + [q.query(i) for i in range(1, 200)]
    q_ids2 = np.concatenate(parts2).astype(np.int32)
    q_off2 = np.zeros(201, np.int64)
    q_off2[1:] = np.cumsum([len(p) for p in parts2])
    qb2 = QueryBatch(q_ids2, q_off2, np.full(200, 40, np.int32))
    ref2 = eager.build_index(c.tokens, c.doc_offsets, c.vocab, token_subset=np.unique(q_ids2))
    idx.set_plan(dict(q_tile=8, waves=4, doc_tile=1024, doc_groups=8, query_order=1))
    ids, sc, cnt = _run(idx, qb2, 40, "batch")
    check_batch(ref2, q_ids2, q_off2, qb2.k, ids, sc, cnt, RTOL["f16"], "long query",
                sample=range(0, 200, 7))
    torch.cuda.synchronize()


def test_empty_document_groups():
    """More document groups than the corpus fills: groups past the last document write empty
    lists that the merge skips (10 document tiles over 8 groups of 2 tiles)."""
    import torch
    c = make_corpus(2, n_docs=10_000)
    q = make_queries(2, n_queries=40, vocab=c.vocab, k=30)
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab, token_subset=np.unique(q.q_ids))
    idx = _index(c, dtype="f16")
    for plan in (dict(q_tile=8, waves=4, doc_tile=1024, doc_groups=8),
                 dict(q_tile=16, waves=8, doc_tile=2048, doc_groups=7)):
        idx.set_plan(plan)
        ids, sc, cnt = _run(idx, q, 30, "batch")
        check_batch(ref, q.q_ids, q.q_offsets, q.k, ids, sc, cnt, RTOL["f16"], str(plan))
    torch.cuda.synchronize()


def _sub_batch(q, idx, k=None):
    parts = [q.query(i) for i in idx]
    off = np.zeros(len(idx) + 1, np.int64)
    off[1:] = np.cumsum([len(p) for p in parts])
    kk = q.k[list(idx)].copy() if k is None else np.full(len(idx), k, np.int32)
    return QueryBatch(np.concatenate(parts).astype(np.int32), off, kk)


def test_graph_mode_matches_eager():
    """Graph mode: batches of several sizes, k and tile orders run as one HIP graph launch each,
    interleaved with eager searches and other device work on the same stream; a repeated batch
    replays the kept graph (in-place update). Every graph result matches the oracle and the
    eager result of the same batch."""
    import torch
    c = make_corpus(2, n_docs=60_000)
    q = make_queries(2, n_queries=900, vocab=c.vocab, k=100)
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab, token_subset=np.unique(q.q_ids))
    idx = _index(c, dtype="f16")
    # (queries, k, tile order): grouped 300 / as given 300 / small / large k / ragged 777
    cases = [(range(0, 300), 100, 0), (range(300, 600), 100, 0), (range(300, 600), 100, 0),
             (range(0, 40), 10, 0), (range(100, 400), 100, 2), (range(0, 64), 1000, 0),
             (range(123, 900), 100, 0), (range(123, 900), 100, 0)]
    calls = 0
    try:
        for qs, k, order in cases:
            qb = _sub_batch(q, list(qs), k)
            if order:
                plan = idx.get_plan(qb.n, 64, k)
                plan["query_order"] = order
                idx.set_plan(plan)
            else:
                idx.set_plan(None)
            idx.set_graphs(False)
            e_ids, e_sc, e_cnt = _run(idx, qb, k, "batch")
            idx.set_graphs(True)
            for rep in range(2):
                # other device work between the replays
                x = torch.arange(1 << 20, device="cuda", dtype=torch.float32)
                assert float(x.sum().item()) == float((1 << 20) * ((1 << 20) - 1) // 2)
                ids, sc, cnt = _run(idx, qb, k, "batch")
                calls += 1
                tag = f"graph {len(qs)}q k={k} order={order} rep={rep}"
                check_batch(ref, qb.q_ids, qb.q_offsets, qb.k, ids, sc, cnt, RTOL["f16"], tag,
                            sample=range(0, qb.n, 7))
                assert np.array_equal(cnt, e_cnt), tag
                # same ranked scores as the eager launch, within the storage tolerance
                fin = np.isfinite(e_sc)
                assert np.array_equal(fin, np.isfinite(sc)), tag
                assert np.allclose(sc[fin], e_sc[fin], rtol=RTOL["f16"], atol=1e-6), tag
    finally:
        idx.set_graphs(False)
        idx.set_plan(None)
    st = idx.graph_stats()
    assert st["builds"] + st["updates"] == calls, st
    assert st["updates"] >= 1 and st["builds"] >= 1, st


@pytest.mark.parametrize("n_queries", [9, 4096 * 8 + 100])
def test_tile_order_small_and_past_limit(cfg0, n_queries):
    """Longest-first tile order: a batch of two tiles (ordered) and one of more than 4096 tiles
    (launched in plain tile order) both return every query's own results."""
    c, _ = cfg0
    q = make_queries(0, n_queries=n_queries, vocab=c.vocab, k=10)
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab, 1.5, 0.75, 0.0, "lucene")
    idx = _index(c, dtype="f16")
    ids, sc, cnt = _run(idx, q, 10, "batch")
    step = max(1, n_queries // 300)
    sample = list(range(0, n_queries, step)) + [n_queries - 1]
    check_batch(ref, q.q_ids, q.q_offsets, q.k, ids, sc, cnt, RTOL["f16"], f"{n_queries} queries",
                sample=sample)
