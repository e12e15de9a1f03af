"""Pure-Python brute force for tiny corpora: dictionaries and math.log, no NumPy.

Test infrastructure only (see the package docstring). Written separately from ``formulas``,
``eager`` and ``scan`` so that a mistake in one of them shows up as a disagreement.

For a corpus given as a list of token lists, it evaluates B(Q, D) = sum over query positions of
S(q_i, D) directly from each document's token counts (Section 2, "Calculation of BM25"), with the
per-variant IDF and S readings documented in ``formulas``.
"""
from __future__ import annotations

import math
from collections import Counter


def _idf(df: int, n: int, variant: int) -> float:
    if df == 0:
        return 0.0
    if variant == 0:      # Lucene
        return math.log((n - df + 0.5) / (df + 0.5) + 1.0)
    if variant == 3:      # Robertson
        return math.log((n - df + 0.5) / (df + 0.5))
    if variant == 4:      # ATIRE
        return math.log(n / df)
    if variant == 1:      # BM25L
        return math.log((n + 1.0) / (df + 0.5))
    if variant in (2, 5):  # BM25+, TF_ldp
        return math.log((n + 1.0) / df)
    raise ValueError(variant)


def _tf_part(tf: int, dl: int, l_avg: float, k1: float, b: float, delta: float,
             variant: int) -> float:
    if tf == 0:
        # the value at TF = 0 does not depend on the length normaliser
        if variant in (0, 3, 4):
            return 0.0
        if variant == 2:
            return delta
        if variant == 1:
            return (k1 + 1.0) * delta / (k1 + delta)
        return 1.0 + math.log(1.0 + math.log(delta))
    k = k1 * (1.0 - b + b * dl / l_avg)
    if variant in (0, 3):
        return tf / (tf + k)
    if variant == 4:
        return (k1 + 1.0) * tf / (tf + k)
    if variant == 2:
        return (k1 + 1.0) * tf / (k + tf) + delta
    c = tf / (1.0 - b + b * dl / l_avg)
    if variant == 1:
        return (k1 + 1.0) * (c + delta) / (k1 + c + delta)
    return 1.0 + math.log(1.0 + math.log(c + delta))


def brute_scores(docs, query, k1=1.5, b=0.75, delta=0.0, variant=0):
    """List of B(Q, D), one per document, for ``docs`` = list of lists of token ids."""
    n = len(docs)
    lengths = [len(d) for d in docs]
    l_avg = sum(lengths) / n
    counts = [Counter(d) for d in docs]
    df = {}
    for t in set(query):
        df[t] = sum(1 for c in counts if c.get(t, 0) > 0)
    out = []
    for j in range(n):
        total = 0.0
        for t in query:
            if df[t] == 0:
                continue
            total += _idf(df[t], n, variant) * _tf_part(counts[j].get(t, 0), lengths[j], l_avg,
                                                        k1, b, delta, variant)
        out.append(total)
    return out


def brute_topk(scores, k):
    order = sorted(range(len(scores)), key=lambda d: (-scores[d], d))
    return order[:min(k, len(scores))]


def brute_csc(docs, vocab):
    """Token-major (indptr, indices, tf) of the TF matrix, from per-document counts."""
    indptr = [0]
    indices = []
    tfs = []
    counts = [Counter(d) for d in docs]
    for t in range(vocab):
        for j, c in enumerate(counts):
            if c.get(t, 0) > 0:
                indices.append(j)
                tfs.append(c[t])
        indptr.append(len(indices))
    return indptr, indices, tfs
