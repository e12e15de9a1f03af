"""Oracle pins beyond the worked example: brute force, library routines, closed forms, invariants.

Each test ties the FP64 oracle to something other than itself:
* the pure-Python brute force on a few hundred random tiny corpora (Section 2: the eager slice-sum
  reaches the directly defined B(Q, D); Section 2.1: the shifted form reaches the unshifted score);
* SciPy's sparse matrix-vector product (the bag-of-words formulation of Section 1's BM25-PT
  comparison reaches the same score vector as slicing and summing rows);
* SciPy's COO-to-CSC conversion (Section 2, "Efficient Matrix Sparsity") for the TF matrix;
* np.argpartition (the paper's top-k routine, Section 2 "Top-k selection") for set equality;
* closed forms and special cases of the score equation.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import brute, eager, formulas as F, scan
from workloads import make_tiny_corpus, make_tiny_queries

VARIANT_PARAMS = [
    ("lucene", 0, 1.5, 0.75, 0.0),
    ("lucene", 0, 0.9, 0.4, 0.0),
    ("lucene", 0, 1.2, 1.0, 0.0),
    ("robertson", 3, 1.2, 0.75, 0.0),
    ("atire", 4, 1.2, 0.75, 0.0),
    ("bm25plus", 2, 1.2, 0.75, 1.0),
    ("bm25l", 1, 1.2, 0.75, 0.5),
    ("bm25l", 1, 1.5, 0.0, 0.5),
    ("tfldp", 5, 1.2, 0.75, 0.5),
]


def _docs(c):
    return [list(map(int, c.doc(d))) for d in range(c.n_docs)]


@pytest.mark.parametrize("name,vid,k1,b,delta", VARIANT_PARAMS)
def test_eager_and_scan_match_brute_force(name, vid, k1, b, delta):
    for seed in range(40):
        c = make_tiny_corpus(seed)
        qb = make_tiny_queries(seed, c.vocab)
        idx = eager.build_index(c.tokens, c.doc_offsets, c.vocab, k1, b, delta, name)
        docs = _docs(c)
        for i in range(qb.n):
            q = list(map(int, qb.query(i)))
            want = np.array(brute.brute_scores(docs, q, k1, b, delta, vid))
            got = eager.scores(idx, q)
            tol = 1e-12 * (1.0 + np.abs(want).max(initial=0.0))
            np.testing.assert_allclose(got, want, rtol=1e-12, atol=tol)
            direct = scan.direct_scores(c.tokens, c.doc_offsets, c.vocab, q, k1, b, delta, name)
            np.testing.assert_allclose(direct, want, rtol=1e-12, atol=tol)
            # top-k under the tie rule: identical when scores are exactly representable alike
            k = int(qb.k[i])
            ids, _ = eager.search(idx, q, k)
            bt = brute.brute_topk(list(got), k)
            assert list(ids) == bt


def test_csc_matches_brute_force_and_scipy():
    for seed in range(60):
        c = make_tiny_corpus(seed)
        idx = eager.build_index(c.tokens, c.doc_offsets, c.vocab)
        ip, ind, tf = brute.brute_csc(_docs(c), c.vocab)
        np.testing.assert_array_equal(idx.indptr, ip)
        np.testing.assert_array_equal(idx.indices, ind)
        np.testing.assert_array_equal(idx.tf, tf)
        # SciPy: duplicates in COO are summed on conversion, giving TF; CSC of the |C| x |V|
        # matrix is the token-major layout
        doc = np.repeat(np.arange(c.n_docs), np.diff(c.doc_offsets))
        m = sp.coo_matrix((np.ones(c.n_tokens, dtype=np.int64), (doc, c.tokens.astype(np.int64))),
                          shape=(c.n_docs, c.vocab)).tocsc()
        m.sum_duplicates()
        m.sort_indices()
        np.testing.assert_array_equal(idx.indptr, m.indptr)
        np.testing.assert_array_equal(idx.indices, m.indices)
        np.testing.assert_array_equal(idx.tf, m.data)


def test_tf_df_invariants():
    for seed in range(60):
        c = make_tiny_corpus(seed)
        idx = eager.build_index(c.tokens, c.doc_offsets, c.vocab)
        # sum_t TF(t, D) = |D|
        per_doc = np.bincount(idx.indices, weights=idx.tf, minlength=c.n_docs)
        np.testing.assert_array_equal(per_doc, np.diff(c.doc_offsets))
        # sum_t DF(t) = nnz, and DF(t) is the segment length
        assert idx.df.sum() == idx.nnz
        np.testing.assert_array_equal(np.diff(idx.indptr), idx.df)
        # document ids strictly ascending inside each segment
        for t in range(c.vocab):
            seg = idx.indices[idx.indptr[t]:idx.indptr[t + 1]]
            assert np.all(np.diff(seg) > 0)
        assert np.all(idx.tf > 0)


@pytest.mark.parametrize("name,vid,k1,b,delta", VARIANT_PARAMS)
def test_slice_sum_equals_sparse_matvec(name, vid, k1, b, delta):
    """Slicing rows and summing them equals (score matrix)^T x bag-of-words(Q), via SciPy."""
    for seed in range(25):
        c = make_tiny_corpus(seed, max_docs=60, max_vocab=40)
        qb = make_tiny_queries(seed, c.vocab, n=4)
        idx = eager.build_index(c.tokens, c.doc_offsets, c.vocab, k1, b, delta, name)
        m = sp.csr_matrix((idx.data, idx.indices, idx.indptr), shape=(c.vocab, c.n_docs))
        for i in range(qb.n):
            q = qb.query(i)
            bow = np.bincount(q, minlength=c.vocab).astype(np.float64)
            want = m.T @ bow
            np.testing.assert_allclose(eager.slice_sum(idx, q), want, rtol=1e-13, atol=1e-14)


def test_shifted_equals_unshifted_and_same_ranking():
    """Section 2.1: sum S_delta + sum S_theta = sum S; the shift does not change the ranking."""
    for name, vid, k1, b, delta in VARIANT_PARAMS:
        if vid not in F.SHIFTED:
            continue
        for seed in range(30):
            c = make_tiny_corpus(seed)
            qb = make_tiny_queries(seed, c.vocab)
            idx = eager.build_index(c.tokens, c.doc_offsets, c.vocab, k1, b, delta, name)
            for i in range(qb.n):
                q = qb.query(i)
                direct = scan.direct_scores(c.tokens, c.doc_offsets, c.vocab, q, k1, b, delta,
                                            name)
                sd = eager.slice_sum(idx, q)
                sh = eager.shift(idx, q)
                np.testing.assert_allclose(sd + sh, direct, rtol=1e-12,
                                           atol=1e-12 * (1 + np.abs(direct).max(initial=0)))
                assert list(eager.topk(sd, 5)) == list(eager.topk(sd + sh, 5)) or \
                    np.allclose(np.sort(sd)[::-1][:5] + sh, np.sort(direct)[::-1][:5])


def test_topk_against_argpartition():
    rng = np.random.default_rng(3)
    for trial in range(50):
        n = int(rng.integers(1, 300))
        s = rng.integers(0, 20, size=n).astype(np.float64) / 7.0  # many exact ties
        k = int(rng.integers(1, n + 5))
        ids = eager.topk(s, k)
        kk = min(k, n)
        assert len(ids) == kk
        # ordered by score desc, id asc
        for a, c in zip(ids[:-1], ids[1:]):
            assert s[a] > s[c] or (s[a] == s[c] and a < c)
        if kk < n:
            part = np.argpartition(-s, kk - 1)[:kk]
            # same multiset of scores; ids may differ only among ties at the k-th score
            np.testing.assert_array_equal(np.sort(s[part]), np.sort(s[ids]))
            kth = s[ids[-1]]
            assert set(np.flatnonzero(s > kth)) <= set(ids)


def test_partitioned_search_agrees_with_the_full_order():
    """The paper's partition-then-sort top-k returns the scores of the definitional full sort;
    ids differ only among ties at the k-th score."""
    for seed in range(20):
        c = make_tiny_corpus(seed)
        if int(np.diff(c.doc_offsets).sum()) == 0:
            continue
        idx = eager.build_index(c.tokens, c.doc_offsets, c.vocab)
        qb = make_tiny_queries(seed, c.vocab, n=8)
        for i in range(qb.n):
            q = qb.query(i)
            b = eager.scores(idx, q)
            for k in (1, 3, c.n_docs, c.n_docs + 2):
                ids_a, s_a = eager.search(idx, q, k)
                ids_b, s_b = eager.search_partitioned(idx, q, k)
                np.testing.assert_array_equal(s_a, s_b)
                assert set(np.flatnonzero(b > s_a[-1])) <= set(ids_b.tolist())
                assert len(set(ids_b.tolist())) == len(ids_b)


def test_lucene_idf_closed_form_and_monotone():
    # ln((N - DF + 0.5)/(DF + 0.5) + 1) = ln((N + 1)/(DF + 0.5))
    for n in (1, 2, 3, 10, 1000, 8_800_000):
        df = np.arange(1, min(n, 5000) + 1)
        got = F.idf(df, n, "lucene")
        np.testing.assert_allclose(got, np.log((n + 1.0) / (df + 0.5)), rtol=1e-14)
        assert np.all(got > 0)
        assert np.all(np.diff(got) < 0)
    np.testing.assert_array_equal(F.idf([0, 0], 10, "lucene"), [0.0, 0.0])


def test_score_special_cases():
    tf = np.array([1, 2, 3, 7, 40])
    dl = np.array([5, 9, 30, 60, 200])
    l_avg = 37.5
    idf_t = 2.0
    # k1 = 0: S = IDF for every TF > 0 (binary)
    np.testing.assert_allclose(F.term_score(idf_t, tf, dl, l_avg, 0.0, 0.75, 0, "lucene"), 2.0)
    # b = 0: independent of |D|: S = IDF * TF / (TF + k1)
    np.testing.assert_allclose(F.term_score(idf_t, tf, dl, l_avg, 1.2, 0.0, 0, "lucene"),
                               idf_t * tf / (tf + 1.2), rtol=1e-15)
    # b = 1 and |D| = L_avg: the normaliser is TF + k1
    np.testing.assert_allclose(F.term_score(idf_t, tf, np.full(5, l_avg), l_avg, 1.2, 1.0, 0,
                                            "lucene"), idf_t * tf / (tf + 1.2), rtol=1e-15)
    # saturation: S < IDF, increasing in TF, decreasing in |D| when b > 0
    s = F.term_score(idf_t, np.arange(1, 50), np.full(49, 20), l_avg, 1.5, 0.75, 0, "lucene")
    assert np.all(s < idf_t) and np.all(np.diff(s) > 0)
    s = F.term_score(idf_t, np.full(49, 3), np.arange(1, 50), l_avg, 1.5, 0.75, 0, "lucene")
    assert np.all(np.diff(s) < 0)


def test_shifted_delta_closed_forms():
    """S - S_theta in closed form: BM25+ gives ATIRE's saturation; BM25L the product form."""
    tf = np.arange(1, 30)
    dl = np.linspace(1, 300, 29)
    l_avg, k1, b = 77.0, 1.2, 0.75
    norm = 1 - b + b * dl / l_avg
    sp_ = F.saturation(tf, dl, l_avg, k1, b, 1.0, "bm25plus") - F.saturation(0 * tf, dl, l_avg,
                                                                            k1, b, 1.0,
                                                                            "bm25plus")
    np.testing.assert_allclose(sp_, F.saturation(tf, dl, l_avg, k1, b, 0, "atire"), rtol=1e-13)
    d = 0.5
    c = tf / norm
    sl = F.saturation(tf, dl, l_avg, k1, b, d, "bm25l") - F.saturation(0 * tf, dl, l_avg, k1, b,
                                                                       d, "bm25l")
    np.testing.assert_allclose(sl, (k1 + 1) * k1 * c / ((k1 + c + d) * (k1 + d)), rtol=1e-13)


def test_absent_query_token_and_errors():
    c = make_tiny_corpus(5)
    v = c.vocab + 3  # ids c.vocab.. are never used by the corpus: DF = 0
    idx = eager.build_index(c.tokens, c.doc_offsets, v, 1.2, 0.75, 1.0, "bm25plus")
    np.testing.assert_array_equal(eager.scores(idx, [v - 1, v - 2]), 0.0)
    with pytest.raises(ValueError):
        eager.build_index(np.array([0, 5], np.int32), np.array([0, 2]), 3)
    with pytest.raises(ValueError):
        eager.build_index(np.zeros(0, np.int32), np.array([0, 0]), 3)


def test_token_subset_index_matches_full_index():
    c = make_tiny_corpus(11, max_docs=40, max_vocab=25)
    full = eager.build_index(c.tokens, c.doc_offsets, c.vocab, 1.5, 0.75, 0.0, "lucene")
    sub = [0, 2, min(3, c.vocab - 1)]
    part = eager.build_index(c.tokens, c.doc_offsets, c.vocab, 1.5, 0.75, 0.0, "lucene",
                             token_subset=sub)
    for q in ([0], [0, 2, 2], sub):
        np.testing.assert_allclose(eager.scores(part, q), eager.scores(full, q), rtol=1e-15)


def test_generator_is_deterministic_and_shaped():
    from workloads import make_corpus, make_queries
    a = make_corpus(0)
    b = make_corpus(0)
    np.testing.assert_array_equal(a.tokens, b.tokens)
    assert a.n_docs == 2000 and a.doc_offsets[-1] == a.n_tokens
    assert np.diff(a.doc_offsets).min() >= 1
    assert 50 < np.diff(a.doc_offsets).mean() < 70
    q = make_queries(0)
    assert q.n == 200 and np.diff(q.q_offsets).min() >= 1 and np.diff(q.q_offsets).max() <= 8
    q2 = make_queries(2, n_queries=5000)
    lens = np.diff(q2.q_offsets)
    assert lens.min() >= 2 and lens.max() <= 30 and 6.0 < lens.mean() < 8.0
    assert math.isclose(float(np.mean(a.tokens == 0)), 1 / np.sum(np.arange(1, 5001) ** -1.1),
                        rel_tol=0.05)
