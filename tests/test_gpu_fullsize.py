"""Full-size runs of the benchmarked workloads, checked against the FP64 oracle on sampled queries.

The oracle builds only the rows of the sampled queries' tokens (every row it builds is the full
row), so each case costs tens of seconds of CPU time and about 20 GB of host memory at 8.8M
documents.
"""
import numpy as np
import pytest

from oracle import eager
from tests.helpers import RTOL, check_batch
from workloads import CONFIGS, make_corpus, make_queries
from workloads.synth import QueryBatch

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _sub_batch(q, idx):
    parts = [q.query(i) for i in idx]
    off = np.zeros(len(idx) + 1, np.int64)
    off[1:] = np.cumsum([len(p) for p in parts])
    return QueryBatch(np.concatenate(parts).astype(np.int32), off, q.k[idx].copy())


def test_full_8_8M_docs_batched_top100_fp16():
    """The benchmark's index (8.8M documents, fp16) and launch: one 4096-query batch with the
    automatic plan; 13 queries spread over the batch (every 341st) are checked."""
    import torch
    from paper_2407_03618_amd import Index
    cfg = CONFIGS[2]
    c = make_corpus(2)
    q = make_queries(2, n_queries=4096, vocab=c.vocab)
    idx = Index(_dev(c.tokens), _dev(c.doc_offsets), c.vocab, cfg["k1"], cfg["b"], cfg["delta"],
                cfg["variant"], "f16")
    torch.cuda.empty_cache()
    ids, sc, cnt = idx.search_batch(_dev(q.q_ids), q.q_offsets, 100, 100)
    torch.cuda.synchronize()
    ids, sc, cnt = ids.cpu().numpy(), sc.cpu().numpy(), cnt.cpu().numpy()
    assert np.all(cnt == 100)
    sample = list(range(0, 4096, 341))
    toks = np.unique(np.concatenate([q.query(i) for i in sample]))
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab, cfg["k1"], cfg["b"], cfg["delta"],
                            cfg["variant"], token_subset=toks)
    check_batch(ref, q.q_ids, q.q_offsets, q.k, ids, sc, cnt, RTOL["f16"], "8.8M batched",
                sample=sample)
    idx.free()


def test_full_1M_docs_plain_top100_fp32():
    """The per-query form at its configured scale (1M documents, fp32, top-100)."""
    import torch
    from paper_2407_03618_amd import Index
    cfg = CONFIGS[1]
    c = make_corpus(1)
    q = make_queries(1, n_queries=64, vocab=c.vocab)
    idx = Index(_dev(c.tokens), _dev(c.doc_offsets), c.vocab, cfg["k1"], cfg["b"], cfg["delta"],
                cfg["variant"], "f32")
    ids, sc, cnt = idx.search_plain(_dev(q.q_ids), q.q_offsets, 100, 100)
    torch.cuda.synchronize()
    ids, sc, cnt = ids.cpu().numpy(), sc.cpu().numpy(), cnt.cpu().numpy()
    sample = list(range(0, 64, 4))
    toks = np.unique(np.concatenate([q.query(i) for i in sample]))
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab, cfg["k1"], cfg["b"], cfg["delta"],
                            cfg["variant"], token_subset=toks)
    check_batch(ref, q.q_ids, q.q_offsets, q.k, ids, sc, cnt, RTOL["f32"], "1M plain",
                sample=sample)
    idx.free()


@pytest.mark.parametrize("variant,delta", [("bm25plus", 1.0), ("bm25l", 0.5)])
def test_long_docs_shifted_top1000_bf16(variant, delta):
    """The shifted-variant workload's recipe (long documents, 30-200-token queries, top-1000,
    bf16, k1 = 1.2, b = 0.75) at 400k documents, both forms."""
    import torch
    from paper_2407_03618_amd import Index
    cfg = CONFIGS[3]
    c = make_corpus(3, n_docs=400_000)
    q = make_queries(3, n_queries=24, vocab=c.vocab)
    idx = Index(_dev(c.tokens), _dev(c.doc_offsets), c.vocab, cfg["k1"], cfg["b"], delta,
                variant, "bf16")
    sample = list(range(0, 24, 3))
    toks = np.unique(np.concatenate([q.query(i) for i in sample]))
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab, cfg["k1"], cfg["b"], delta, variant,
                            token_subset=toks)
    ids, sc, cnt = idx.search_batch(_dev(q.q_ids), q.q_offsets, 1000, 1000)
    torch.cuda.synchronize()
    check_batch(ref, q.q_ids, q.q_offsets, q.k, ids.cpu().numpy(), sc.cpu().numpy(),
                cnt.cpu().numpy(), RTOL["bf16"], f"{variant} batched", sample=sample)
    sub = _sub_batch(q, sample[:3])
    ids, sc, cnt = idx.search_plain(_dev(sub.q_ids), sub.q_offsets, 1000, 1000)
    torch.cuda.synchronize()
    check_batch(ref, sub.q_ids, sub.q_offsets, sub.k, ids.cpu().numpy(), sc.cpu().numpy(),
                cnt.cpu().numpy(), RTOL["bf16"], f"{variant} plain")
    idx.free()
