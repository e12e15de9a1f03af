"""The paper's eager sparse scoring in FP64: index-time scores, query-time slice-and-sum, top-k.

Test infrastructure only (see the package docstring).

Index time (Section 2, "Eager index-time scoring" and "Efficient Matrix Sparsity"): every
(t, D) pair with TF(t, D) > 0 gets S(t, D) computed once and stored in a token-major sparse
matrix. The paper calls it CSC; here the pointer axis is the token axis (one contiguous segment of
(document id, score) per token, document ids ascending), which is the layout that makes "select
the query's rows" a contiguous slice. Pairs with TF = 0 are not stored.

Non-occurrence adjustment (Section 2.1): for the variants whose score is non-zero at TF = 0 the
matrix stores S_delta(t, D) = S(t, D) - S_theta(t); the query adds sum_i S_theta(q_i) back.

Query time (Section 2, "Assigning Query Scores"): slice the rows of the query's tokens and sum them
over the token dimension into one score per document; every query position counts, so a repeated
token is summed once per occurrence (B(Q, D) sums over i = 1..|Q|).

Top-k (Section 2, "Top-k selection"): the k largest scores. The paper partitions and optionally
sorts; the oracle returns the plain definition, the first min(k, N) documents of the full order
(score descending, then document id ascending for equal scores).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import formulas as F


@dataclass
class EagerIndex:
    n_docs: int
    vocab: int
    sum_len: int            # exact sum of |D| (Python int)
    l_avg: float            # sum_len / n_docs in FP64
    doclen: np.ndarray      # int64[N]
    df: np.ndarray          # int64[V]
    idf: np.ndarray         # float64[V]
    theta: np.ndarray       # float64[V], S_theta(t) (zeros for sparse variants)
    indptr: np.ndarray      # int64[V+1]
    indices: np.ndarray     # int64[nnz], document ids, ascending within a token's segment
    tf: np.ndarray          # int64[nnz]
    data: np.ndarray        # float64[nnz], S (sparse variants) or S_delta (shifted variants)
    variant: int
    k1: float
    b: float
    delta: float
    token_subset: np.ndarray | None = None

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])


def _group_pairs(tok: np.ndarray, doc: np.ndarray):
    """Order positions by (token, document); positions arrive in document order."""
    uniq = np.unique(tok)
    if uniq.size <= 65535:
        # dense local ids let NumPy use its stable radix sort; stability keeps document order
        local = np.searchsorted(uniq, tok).astype(np.uint16)
        order = np.argsort(local, kind="stable")
    else:
        order = np.lexsort((doc, tok))
    return tok[order], doc[order]


def build_index(tokens, doc_offsets, vocab: int, k1: float = 1.5, b: float = 0.75,
                delta: float = 0.0, variant="lucene", token_subset=None) -> EagerIndex:
    """Index a corpus given as token ids grouped by document (``doc_offsets`` = CSR offsets).

    ``token_subset`` restricts the stored rows to those tokens (their DF still counts every
    document of the corpus); queries may then only use tokens from the subset.
    """
    variant = F.variant_id(variant)
    tokens = np.asarray(tokens)
    doc_offsets = np.asarray(doc_offsets, dtype=np.int64)
    # |D| in tokens and L_avg (Section 2, definition under the B(Q, D) equation)
    doclen = np.diff(doc_offsets)
    n_docs = int(doclen.size)
    sum_len = int(doclen.sum())
    if n_docs <= 0 or sum_len <= 0:
        raise ValueError("L_avg is undefined: the corpus needs at least one non-empty document")
    if np.any(doclen < 0) or doc_offsets[0] != 0 or doc_offsets[-1] != tokens.size:
        raise ValueError("document offsets must be non-decreasing from 0 to the token count")
    if tokens.size and (tokens.min() < 0 or tokens.max() >= vocab):
        raise ValueError("token id out of range")
    l_avg = sum_len / n_docs

    tok = tokens.astype(np.int64)
    doc = np.repeat(np.arange(n_docs, dtype=np.int64), doclen)
    if token_subset is not None:
        token_subset = np.unique(np.asarray(token_subset, dtype=np.int64))
        keep = np.isin(tok, token_subset)
        tok, doc = tok[keep], doc[keep]

    # TF(t, D): count the positions of each (t, D) pair
    t_s, d_s = _group_pairs(tok, doc)
    if t_s.size:
        new = np.empty(t_s.size, dtype=bool)
        new[0] = True
        new[1:] = (t_s[1:] != t_s[:-1]) | (d_s[1:] != d_s[:-1])
        starts = np.flatnonzero(new)
    else:
        starts = np.zeros(0, dtype=np.int64)
    tf = np.diff(np.append(starts, t_s.size)).astype(np.int64)
    pair_t = t_s[starts]
    pair_d = d_s[starts]

    # DF(t): number of documents with TF(t, D) > 0 (IDF equation)
    df = np.bincount(pair_t, minlength=vocab).astype(np.int64)
    indptr = np.zeros(vocab + 1, dtype=np.int64)
    np.cumsum(df, out=indptr[1:])

    idf_t = F.idf(df, n_docs, variant)
    # S(t, D) for every stored pair (eager index-time scoring)
    s = F.term_score(idf_t[pair_t], tf, doclen[pair_d], l_avg, k1, b, delta, variant)
    theta = F.nonoccurrence(idf_t, k1, b, delta, variant)
    theta = np.where(df > 0, theta, 0.0)
    # S_delta(t, D) = S(t, D) - S_theta(t) (Section 2.1); theta is zero for sparse variants
    data = s - theta[pair_t]
    return EagerIndex(n_docs, int(vocab), sum_len, l_avg, doclen, df, idf_t, theta, indptr,
                      pair_d, tf, data, variant, float(k1), float(b), float(delta),
                      token_subset)


def slice_sum(index: EagerIndex, query) -> np.ndarray:
    """Sum of the query's stored rows: one value per document (Section 2, Assigning Query Scores)."""
    acc = np.zeros(index.n_docs, dtype=np.float64)
    for t in np.asarray(query, dtype=np.int64):
        if index.token_subset is not None and not np.isin(t, index.token_subset):
            raise ValueError(f"token {t} is not in this index's token subset")
        lo, hi = index.indptr[t], index.indptr[t + 1]
        # document ids are unique inside a row, so a fancy-indexed add is exact
        acc[index.indices[lo:hi]] += index.data[lo:hi]
    return acc


def shift(index: EagerIndex, query) -> float:
    """sum_i S_theta(q_i): one scalar per query added to every document (Section 2.1)."""
    q = np.asarray(query, dtype=np.int64)
    return float(index.theta[q].sum()) if q.size else 0.0


def scores(index: EagerIndex, query) -> np.ndarray:
    """B(Q, D) for every document: slice-sum plus the non-occurrence shift."""
    return slice_sum(index, query) + shift(index, query)


def topk(b_scores: np.ndarray, k: int) -> np.ndarray:
    """Ids of the min(k, N) best documents: score descending, then id ascending."""
    n = b_scores.shape[0]
    order = np.lexsort((np.arange(n), -b_scores))
    return order[:min(int(k), n)]


def search(index: EagerIndex, query, k: int):
    """Top-k (ids, B scores) of one query."""
    b = scores(index, query)
    ids = topk(b, k)
    return ids, b[ids]


def search_partitioned(index: EagerIndex, query, k: int):
    """Top-k the way the paper's implementation selects it (Section 2, "Top-k selection"):
    partition the score vector around the k-th largest value, then sort only those k. Among
    documents tied at the k-th score the partition keeps an unspecified subset, so the ids may
    differ from ``search`` only there; the scores are the same. Used to time the paper's method."""
    b = scores(index, query)
    n = b.shape[0]
    kk = min(int(k), n)
    part = np.argpartition(-b, kk - 1)[:kk] if kk < n else np.arange(n)
    order = np.lexsort((part, -b[part]))
    ids = part[order]
    return ids, b[ids]


def search_batch(index: EagerIndex, q_ids, q_offsets, k):
    """Top-k of every query of a batch; ``k`` is a scalar or one value per query."""
    q_offsets = np.asarray(q_offsets, dtype=np.int64)
    n = q_offsets.size - 1
    ks = np.broadcast_to(np.asarray(k, dtype=np.int64), (n,))
    out = []
    for i in range(n):
        out.append(search(index, q_ids[q_offsets[i]:q_offsets[i + 1]], int(ks[i])))
    return out
