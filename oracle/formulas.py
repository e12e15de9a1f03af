"""Per-variant IDF(t) and term score S(t, D), FP64, vectorised with NumPy.

Test infrastructure only (see the package docstring).

Lucene is the paper's default (Section 2, "Calculation of BM25"): with
  norm(D) = 1 - b + b * |D| / L_avg                      (the length normaliser inside the
                                                         denominator of the S(t, D) equation)
  S(t, D) = IDF(t) * TF(t, D) / (TF(t, D) + k1 * norm(D))
  IDF(t)  = ln((|C| - DF(t) + 0.5) / (DF(t) + 0.5) + 1)  (IDF equation, natural log)

The other variants are named by the paper (Section 2, "Alternative BM25 implementations";
Section 2.1; Table 3) but their formulas are not printed there. The readings used here follow the
BM25 variant study the paper cites, with c(t, D) = TF / norm(D):

  Robertson  IDF = ln((N - DF + 0.5) / (DF + 0.5))   S = IDF * TF / (TF + k1 norm)
  ATIRE      IDF = ln(N / DF)                         S = IDF * (k1 + 1) TF / (TF + k1 norm)
  BM25+      IDF = ln((N + 1) / DF)                   S = IDF * ((k1 + 1) TF / (k1 norm + TF) + delta)
  BM25L      IDF = ln((N + 1) / (DF + 0.5))           S = IDF * (k1 + 1)(c + delta) / (k1 + c + delta)
  TF_ldp     IDF = ln((N + 1) / DF)                   S = IDF * (1 + ln(1 + ln(c + delta)))

Readings where the paper is silent:
  * A token with DF = 0 (absent from the corpus) contributes 0 to every document, for every
    variant, including its non-occurrence score.
  * A term with TF = 0 is scored with norm set to 1. For every variant above the TF = 0 value does
    not depend on norm (Section 2.1 notes that S(t, empty doc) depends on t only through DF), and
    this avoids 0/0 for an empty document when b = 1.
  * BM25L keeps no "c > 0" guard: Section 2.1 states that its score is non-zero at TF = 0.
"""
from __future__ import annotations

import numpy as np

LUCENE, BM25L, BM25PLUS, ROBERTSON, ATIRE, TFLDP = range(6)
VARIANTS = {"lucene": LUCENE, "bm25l": BM25L, "bm25plus": BM25PLUS, "robertson": ROBERTSON,
            "atire": ATIRE, "tfldp": TFLDP}
# Variants whose score is non-zero at TF = 0 (Section 2.1): stored shifted, S_delta = S - S_theta.
SHIFTED = frozenset({BM25L, BM25PLUS, TFLDP})


def variant_id(v) -> int:
    if isinstance(v, str):
        return VARIANTS[v.lower()]
    return int(v)


def idf(df, n_docs: int, variant) -> np.ndarray:
    """IDF(t, C) for each entry of ``df`` (FP64). Lucene: the IDF equation of Section 2."""
    variant = variant_id(variant)
    df = np.asarray(df, dtype=np.float64)
    n = float(n_docs)
    with np.errstate(divide="ignore", invalid="ignore"):
        if variant == LUCENE:
            out = np.log((n - df + 0.5) / (df + 0.5) + 1.0)
        elif variant == ROBERTSON:
            out = np.log((n - df + 0.5) / (df + 0.5))
        elif variant == ATIRE:
            out = np.log(n / df)
        elif variant == BM25L:
            out = np.log((n + 1.0) / (df + 0.5))
        elif variant in (BM25PLUS, TFLDP):
            out = np.log((n + 1.0) / df)
        else:
            raise ValueError(f"unknown variant {variant}")
    out = np.where(df > 0, out, 0.0)
    return out


def saturation(tf, doclen, l_avg: float, k1: float, b: float, delta: float, variant) -> np.ndarray:
    """S(t, D) / IDF(t): the term-frequency part of the score, FP64 (see the module docstring)."""
    variant = variant_id(variant)
    tf = np.asarray(tf, dtype=np.float64)
    doclen = np.asarray(doclen, dtype=np.float64)
    norm = 1.0 - b + b * doclen / float(l_avg)
    norm = np.where(tf > 0, norm, 1.0)
    if variant in (LUCENE, ROBERTSON):
        return tf / (tf + k1 * norm)
    if variant == ATIRE:
        return (k1 + 1.0) * tf / (tf + k1 * norm)
    if variant == BM25PLUS:
        return (k1 + 1.0) * tf / (k1 * norm + tf) + delta
    c = tf / norm
    if variant == BM25L:
        return (k1 + 1.0) * (c + delta) / (k1 + c + delta)
    if variant == TFLDP:
        return 1.0 + np.log(1.0 + np.log(c + delta))
    raise ValueError(f"unknown variant {variant}")


def term_score(idf_t, tf, doclen, l_avg, k1, b, delta, variant) -> np.ndarray:
    """S(t, D) = IDF(t) * saturation (the eager score equation of Section 2)."""
    return np.asarray(idf_t, dtype=np.float64) * saturation(tf, doclen, l_avg, k1, b, delta,
                                                            variant)


def nonoccurrence(idf_t, k1: float, b: float, delta: float, variant) -> np.ndarray:
    """S_theta(t) = S(t, empty document), the non-occurrence score of Section 2.1.

    Zero for the sparse variants (Lucene, Robertson, ATIRE); the TF = 0 value otherwise.
    """
    variant = variant_id(variant)
    idf_t = np.asarray(idf_t, dtype=np.float64)
    if variant not in SHIFTED:
        return np.zeros_like(idf_t)
    zero = np.zeros_like(idf_t)
    return idf_t * saturation(zero, zero, 1.0, k1, b, delta, variant)
