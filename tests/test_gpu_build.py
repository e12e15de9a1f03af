"""GPU index build against the FP64 oracle: CSC, TF and DF bit-exact; IDF and S_theta to FP64
rounding; stored scores to the storage type's rounding; error codes."""
import numpy as np
import pytest

from oracle import eager
from workloads import make_corpus, make_tiny_corpus

pytestmark = pytest.mark.gpu

STORE_RTOL = {"f32": 2e-6, "f16": 1e-3, "bf16": 4e-3}
VARIANTS = [("lucene", 1.5, 0.75, 0.0), ("bm25plus", 1.2, 0.75, 1.0), ("bm25l", 1.2, 0.75, 0.5),
            ("robertson", 1.2, 0.75, 0.0), ("atire", 1.2, 0.75, 0.0), ("tfldp", 1.2, 0.75, 0.5)]


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _build(c, variant="lucene", k1=1.5, b=0.75, delta=0.0, dtype="f32"):
    from paper_2407_03618_amd import Index
    return Index(_dev(c.tokens), _dev(c.doc_offsets), c.vocab, k1, b, delta, variant, dtype)


def _compare(idx, ref, dtype, where):
    import torch
    ex = idx.export()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ex["indptr"].cpu().numpy(), ref.indptr, err_msg=where)
    np.testing.assert_array_equal(ex["indices"].cpu().numpy(), ref.indices, err_msg=where)
    np.testing.assert_array_equal(ex["tf"].cpu().numpy(), ref.tf, err_msg=where)
    np.testing.assert_array_equal(ex["df"].cpu().numpy(), ref.df, err_msg=where)
    np.testing.assert_allclose(ex["idf"].cpu().numpy(), ref.idf, rtol=1e-14, atol=1e-300,
                               err_msg=where)
    np.testing.assert_allclose(ex["theta"].cpu().numpy(), ref.theta, rtol=1e-14, atol=1e-300,
                               err_msg=where)
    data = ex["data"].float().cpu().numpy().astype(np.float64)
    # rounding of the stored value is relative to the value itself; S_delta of shifted
    # variants is computed in a cancellation-free form
    np.testing.assert_allclose(data, ref.data, rtol=STORE_RTOL[dtype], atol=1e-30, err_msg=where)
    assert idx.nnz == ref.nnz and idx.sum_len == ref.sum_len
    assert idx.l_avg == ref.l_avg


@pytest.mark.parametrize("variant,k1,b,delta", VARIANTS)
@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_tiny_corpora_bit_exact(variant, k1, b, delta, dtype):
    for seed in range(12):
        c = make_tiny_corpus(seed)
        ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab, k1, b, delta, variant)
        idx = _build(c, variant, k1, b, delta, dtype)
        _compare(idx, ref, dtype, f"seed {seed}")
        idx.free()


def test_config0_corpus():
    c = make_corpus(0)
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab)
    idx = _build(c)
    _compare(idx, ref, "f32", "config 0")


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_scaled_large_vocab_corpus(dtype):
    """Three radix passes (V = 2M), skip-table rows, several thousand documents per token."""
    c = make_corpus(2, n_docs=120_000)
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab)
    idx = _build(c, dtype=dtype)
    _compare(idx, ref, dtype, "scaled config 2")


def test_empty_documents_and_single_token_vocab():
    from workloads.synth import Corpus
    tokens = np.zeros(7, np.int32)
    offsets = np.array([0, 0, 3, 3, 7, 7], np.int64)
    c = Corpus(tokens, offsets, 1)
    ref = eager.build_index(tokens, offsets, 1)
    idx = _build(c)
    _compare(idx, ref, "f32", "single token")


@pytest.mark.parametrize("shape", ["empty_runs", "one_token_docs", "long_docs"])
def test_document_layouts(shape):
    """Documents that are mostly empty (hundreds of document starts inside one 64-position run),
    one token long, or thousands of tokens long, so that the build's position-to-document search
    takes every path; a negative token id is still reported."""
    from workloads.synth import Corpus
    rng = np.random.default_rng({"empty_runs": 1, "one_token_docs": 2, "long_docs": 3}[shape])
    if shape == "empty_runs":
        lens = np.where(rng.random(30_000) < 0.97, 0, rng.integers(1, 40, 30_000))
        lens[:500] = 0
        lens[-700:] = 0
    elif shape == "one_token_docs":
        lens = rng.integers(0, 3, 50_000)
    else:
        lens = rng.integers(1500, 9000, 40)
    off = np.zeros(lens.size + 1, np.int64)
    off[1:] = np.cumsum(lens)
    V = 3000
    tokens = np.minimum(rng.zipf(1.3, int(off[-1])) - 1, V - 1).astype(np.int32)
    c = Corpus(tokens, off, V)
    ref = eager.build_index(tokens, off, V)
    idx = _build(c, dtype="f16")
    _compare(idx, ref, "f16", shape)
    idx.free()


def test_build_errors():
    from paper_2407_03618_amd import BM25Error, Index
    import torch
    tok = _dev(np.array([0, 1, 5], np.int32))
    off = _dev(np.array([0, 2, 3], np.int64))
    with pytest.raises(BM25Error) as e:
        Index(tok, off, 3)
    assert e.value.code == -2
    tok = _dev(np.array([0, 1, 2], np.int32))
    with pytest.raises(BM25Error) as e:
        Index(tok, _dev(np.array([0, 3, 2], np.int64)), 3)
    assert e.value.code == -2
    with pytest.raises(BM25Error) as e:
        Index(tok, _dev(np.array([1, 2, 3], np.int64)), 3)
    assert e.value.code == -2
    with pytest.raises(BM25Error) as e:
        Index(_dev(np.array([0, -1, 2], np.int32)), off.clone(), 3)
    assert e.value.code == -2
    with pytest.raises(BM25Error) as e:
        Index(tok, off.clone(), 3, b=1.5)
    assert e.value.code == -1
    with pytest.raises(BM25Error) as e:
        Index(tok, off.clone(), 3, variant=9)
    assert e.value.code == -1
    with pytest.raises(BM25Error) as e:
        Index(tok[:0], _dev(np.array([0, 0], np.int64)), 3)
    assert e.value.code == -1
    torch.cuda.synchronize()


def test_build_is_deterministic():
    import torch
    c = make_corpus(0, n_docs=1500)
    a = _build(c).export()
    b = _build(c).export()
    torch.cuda.synchronize()
    for key in ("indptr", "indices", "tf", "data"):
        assert torch.equal(a[key], b[key])
