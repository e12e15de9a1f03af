"""Tokenization on the GPU against the plain-Python oracle (Section 2, "Tokenization"): token ids,
per-document offsets and the dictionary bit-exact, query mapping, and the ids feeding the index
build."""
import numpy as np
import pytest

from oracle import eager
from oracle import tokenize as T
from tests.test_oracle_tokenize import CASES
from workloads.text import make_text_corpus, make_text_queries

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _pack(docs):
    off = np.zeros(len(docs) + 1, np.int64)
    off[1:] = np.cumsum([len(d) for d in docs])
    data = np.frombuffer(b"".join(docs), dtype=np.uint8) if off[-1] else np.zeros(0, np.uint8)
    return data, off


def _gpu_vocab(docs, lower):
    from paper_2407_03618_amd import Vocab
    data, off = _pack(docs)
    return Vocab(_dev(data), _dev(off), lowercase=lower)


def _same_as_oracle(docs, lower):
    v = _gpu_vocab(docs, lower)
    ids, off = v.corpus()
    want_ids, want_off, want_words = T.build_vocab(docs, lower)
    np.testing.assert_array_equal(ids.cpu().numpy(), want_ids)
    np.testing.assert_array_equal(off.cpu().numpy(), want_off)
    assert v.words() == want_words
    assert v.vocab_size == len(want_words) and v.n_tokens == want_ids.size
    return v


@pytest.mark.parametrize("lower", [False, True])
def test_hand_cases_as_one_corpus(lower):
    docs = [c[0] for c in CASES]
    _same_as_oracle(docs, lower)


@pytest.mark.parametrize("lower", [False, True])
def test_synthetic_corpus_bit_exact(lower):
    c = make_text_corpus(3000, seed=5, lexicon=4000)
    v = _same_as_oracle(c.docs(), lower)
    v.free()


def test_invalid_utf8_and_document_edges():
    docs = [b"", b"ab", b"\xe2\x82", b"\xe2\x82\xacab", b"x\xed\xa0\x80yz", b"\xf0\x9f\x99",
            b"\xc0\xafab", "é".encode() + b"\xf4\x90\x80\x80cd", b"a" * 5000, b"ab" * 3 + b"!"]
    _same_as_oracle(docs, False)
    _same_as_oracle(docs, True)


@pytest.mark.parametrize("lower", [False, True])
def test_query_mapping(lower):
    c = make_text_corpus(1500, seed=6, lexicon=3000)
    q = make_text_queries(300, seed=7, lexicon=3000, corpus_seed=6)
    v = _gpu_vocab(c.docs(), lower)
    _, _, words = T.build_vocab(c.docs(), lower)
    data, off = _pack(q.docs())
    ids, id_off = v.map(_dev(data), _dev(off))
    want_ids, want_off = T.map_queries(q.docs(), words, lower)
    np.testing.assert_array_equal(ids.cpu().numpy(), want_ids)
    np.testing.assert_array_equal(id_off.cpu().numpy(), want_off)


def test_malformed_offsets_and_empty_corpus():
    from paper_2407_03618_amd import BM25Error, Vocab
    data, off = _pack([b"alpha beta", b"gamma"])
    bad = off.copy()
    bad[1] = bad[2] + 1
    with pytest.raises(BM25Error) as e:
        Vocab(_dev(data), _dev(bad))
    assert e.value.code == -2
    v = _gpu_vocab([b"", b"a ! b"], False)
    assert v.n_tokens == 0 and v.vocab_size == 0
    ids, off = v.corpus()
    assert ids.numel() == 0 and off.cpu().tolist() == [0, 0, 0]


def test_tokenized_corpus_feeds_the_index():
    """Text -> ids on the GPU -> index build -> batched search, against the oracle run on the
    oracle's own tokenization of the same text."""
    import torch
    from paper_2407_03618_amd import Index
    from tests.helpers import RTOL, check_batch
    c = make_text_corpus(4000, seed=8, lexicon=5000)
    q = make_text_queries(64, seed=9, lexicon=5000, corpus_seed=8)
    v = _gpu_vocab(c.docs(), True)
    ids, off = v.corpus()
    idx = Index(ids, off, max(v.vocab_size, 1), 1.5, 0.75, 0.0, "lucene", "f32")
    data, qoff = _pack(q.docs())
    qids, qid_off = v.map(_dev(data), _dev(qoff))
    res = idx.search_batch(qids, qid_off.cpu().numpy(), 10, 10)
    torch.cuda.synchronize()
    t_ids, t_off, words = T.build_vocab(c.docs(), True)
    oq_ids, oq_off = T.map_queries(q.docs(), words, True)
    ref = eager.build_index(t_ids, t_off, len(words), 1.5, 0.75, 0.0, "lucene")
    check_batch(ref, oq_ids, oq_off, np.full(64, 10), *(r.cpu().numpy() for r in res),
                RTOL["f32"], "text corpus")
