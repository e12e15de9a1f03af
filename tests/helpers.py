"""Shared checks of GPU results against the FP64 oracle.

Tolerances: stored FP32 scores 1e-5, FP16 2e-3 and BF16 4e-3, relative to
sum_i (|S_delta(q_i, D)| + |S_theta(q_i)|): the magnitudes of the values that are actually stored,
rounded and summed (Section 2.1's shifted form; S_delta = S and S_theta = 0 for sparse variants).
It equals sum_i |S(q_i, D)| whenever S_delta and S_theta are non-negative, which holds for every
variant except TF_ldp with delta < 1, whose S_theta is negative. For all-positive sparse scores it
is B itself. BF16 keeps 8 significant bits, so rounding one stored score to
nearest costs at most 2^-8 ~ 3.9e-3 of its magnitude; FP16 keeps 11 bits (2^-11 ~ 4.9e-4); FP32
storage plus FP32 accumulation over at most a few hundred positions stays well under 1e-5.

Top-k with ties: let s_k be the oracle's k-th score and tol the tolerance at that rank. Every
returned document must score at least s_k - tol in the oracle, every document scoring more than
s_k + tol must be returned, returned scores must be non-increasing and equal returned scores must
come in ascending id order.
"""
import numpy as np

from oracle import eager

RTOL = {0: 1e-5, 1: 2e-3, 2: 4e-3, "f32": 1e-5, "f16": 2e-3, "bf16": 4e-3}


def oracle_scores(ref: eager.EagerIndex, query):
    """(B, sum_i |S_delta(q_i, D)| + |S_theta(q_i)|) for every document, FP64."""
    q = np.asarray(query, dtype=np.int64)
    b = eager.scores(ref, q)
    th = ref.theta
    absS = np.zeros(ref.n_docs)
    for t in q:
        absS += abs(th[t])
        lo, hi = ref.indptr[t], ref.indptr[t + 1]
        absS[ref.indices[lo:hi]] += np.abs(ref.data[lo:hi])
    return b, absS


def check_query(ids, scores, count, b, absS, k, rtol, where="", all_errors=False):
    """Checks one query's returned rows against the oracle (see the module docstring); returns
    the largest relative error, or with all_errors the relative error of every returned
    document."""
    n = b.shape[0]
    kk = min(int(k), n)
    assert int(count) == kk, f"{where}: count {count} != {kk}"
    top_ids = np.asarray(ids[:kk], dtype=np.int64)
    top_sc = np.asarray(scores[:kk], dtype=np.float64)
    assert np.all(np.asarray(ids[kk:k]) == -1), f"{where}: padding ids"
    assert np.all(np.isneginf(np.asarray(scores[kk:k]))), f"{where}: padding scores"
    assert top_ids.min(initial=0) >= 0 and top_ids.max(initial=0) < n, f"{where}: id range"
    assert len(set(top_ids.tolist())) == kk, f"{where}: duplicate ids"
    tol = rtol * absS[top_ids] + 1e-30
    err = np.abs(top_sc - b[top_ids])
    assert np.all(err <= tol), (f"{where}: score error {err.max():.3e} > tol "
                                f"(worst rel {(err / np.maximum(absS[top_ids], 1e-30)).max():.3e})")
    order = np.lexsort((np.arange(n), -b))
    ref_top = order[:kk]
    s_k = b[ref_top[-1]]
    band = rtol * max(absS[top_ids].max(initial=0.0), absS[ref_top].max(initial=0.0)) + 1e-30
    assert np.all(b[top_ids] >= s_k - 2 * band), f"{where}: returned a doc below the k-th score"
    must = ref_top[b[ref_top] > s_k + 2 * band]
    missing = set(must.tolist()) - set(top_ids.tolist())
    assert not missing, f"{where}: missing clear top-k docs {sorted(missing)[:5]}"
    assert np.all(np.diff(top_sc) <= 0), f"{where}: scores not descending"
    eq = np.flatnonzero(np.diff(top_sc) == 0)
    assert np.all(top_ids[eq] < top_ids[eq + 1]), f"{where}: equal scores not in id order"
    rel = err / np.maximum(absS[top_ids], 1e-30)
    if all_errors:
        return rel
    return float(rel.max(initial=0.0))


def check_batch(ref, q_ids, q_offsets, ks, ids, scores, counts, rtol, where="", sample=None):
    """Checks every query (or the given sample of query indices); returns the max rel error."""
    ids = np.asarray(ids)
    scores = np.asarray(scores)
    counts = np.asarray(counts)
    n = len(q_offsets) - 1
    ks = np.broadcast_to(np.asarray(ks), (n,))
    worst = 0.0
    for i in (range(n) if sample is None else sample):
        q = q_ids[q_offsets[i]:q_offsets[i + 1]]
        b, absS = oracle_scores(ref, q)
        worst = max(worst, check_query(ids[i], scores[i], counts[i], b, absS, int(ks[i]), rtol,
                                       f"{where} query {i}"))
    return worst
