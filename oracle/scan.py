"""The plain definition B(Q, D) = sum_i S(q_i, D), evaluated per query without a sparse matrix.

Test infrastructure only (see the package docstring).

Section 2 ("Calculation of BM25") defines the score of a query against a document as a sum of
S(q_i, D) over the query's positions. This module evaluates that sum directly for every document:
TF(q, D) and DF(q) are counted from the documents' own token lists (one pass over the corpus per
query), every position's S is evaluated with the TF of that document, including TF = 0 terms, and
nothing is shifted. The paper's claims that the eager slice-and-sum and the shifted form reach the
same numbers are then checked against this by the tests.
"""
from __future__ import annotations

import numpy as np

from . import formulas as F


def doc_of_positions(doc_offsets: np.ndarray, positions: np.ndarray) -> np.ndarray:
    return np.searchsorted(doc_offsets, positions, side="right") - 1


def direct_scores(tokens, doc_offsets, vocab: int, query, k1: float = 1.5, b: float = 0.75,
                  delta: float = 0.0, variant="lucene", doc_of=None) -> np.ndarray:
    """B(Q, D) for every document D in FP64, straight from the definition.

    ``doc_of`` may pass a precomputed document id per token position (int32/int64[T]).
    """
    variant = F.variant_id(variant)
    tokens = np.asarray(tokens)
    doc_offsets = np.asarray(doc_offsets, dtype=np.int64)
    doclen = np.diff(doc_offsets)
    n_docs = doclen.size
    l_avg = int(doclen.sum()) / n_docs
    q = np.asarray(query, dtype=np.int64)
    b_out = np.zeros(n_docs, dtype=np.float64)
    if q.size == 0:
        return b_out
    uq = np.unique(q)
    lut = np.full(vocab, -1, dtype=np.int64)
    lut[uq] = np.arange(uq.size)
    slot = lut[tokens]
    pos = np.flatnonzero(slot >= 0)
    docs = doc_of[pos].astype(np.int64) if doc_of is not None else doc_of_positions(doc_offsets,
                                                                                     pos)
    # TF(q, D) for each distinct query token q, dense over documents
    tf = np.bincount(slot[pos] * n_docs + docs, minlength=uq.size * n_docs)
    tf = tf.reshape(uq.size, n_docs)
    df = np.count_nonzero(tf, axis=1)
    idf_q = F.idf(df, n_docs, variant)
    for t in q:  # every position of the query, repeats included
        j = int(lut[t])
        if df[j] == 0:
            continue  # a token absent from the corpus scores 0 everywhere
        b_out += F.term_score(idf_q[j], tf[j], doclen, l_avg, k1, b, delta, variant)
    return b_out
