"""Seeded synthetic UTF-8 text corpora for the tokenization step.

The paper's corpora are public retrieval benchmarks, not present here; this generator stands in
with text of a similar shape: documents of Zipf-distributed words from a seeded lexicon, with
log-normal document lengths. The lexicon mixes scripts and character classes so that the word
splitting is exercised across Unicode: lowercase and capitalised ASCII words, accented Latin,
Greek, Cyrillic and CJK words, digits (ASCII and Arabic-Indic), underscores, single-character
words (which the split drops), combining marks (which split a word), the dotted capital I
(U+0130, whose lowercase is two characters), and separators made of spaces, punctuation,
newlines and emoji, with an occasional byte that is not valid UTF-8. No tokenization and no
BM25 arithmetic happens here.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .synth import sample_doc_lengths, sample_zipf, zipf_cdf

_LOWER = [chr(c) for c in range(ord("a"), ord("z") + 1)]
_UPPER = [chr(c) for c in range(ord("A"), ord("Z") + 1)]
_LATIN1 = [chr(c) for c in range(0xE0, 0x100) if c != 0xF7]
_LATIN1_UP = [chr(c) for c in range(0xC0, 0xDF) if c != 0xD7]
_GREEK = [chr(c) for c in range(0x3B1, 0x3CA)]
_GREEK_UP = [chr(c) for c in range(0x391, 0x3AA) if c != 0x3A2]
_CYRILLIC = [chr(c) for c in range(0x430, 0x450)]
_CYRILLIC_UP = [chr(c) for c in range(0x410, 0x430)]
_CJK = [chr(c) for c in range(0x4E00, 0x4E00 + 2000)]
_DIGITS = [chr(c) for c in range(ord("0"), ord("9") + 1)]
_ARABIC_DIGITS = [chr(c) for c in range(0x660, 0x66A)]
_SEPARATORS = [" ", " ", " ", " ", ", ", ". ", " - ", "-", "'", "\n", " (", ") ", "; ", ": ",
               " \U0001F642 ", "/", "\t", " — "]


@dataclass
class TextCorpus:
    data: np.ndarray      # uint8[n_bytes]: the documents' UTF-8 text back to back
    offsets: np.ndarray   # int64[N+1]: document d is data[offsets[d]:offsets[d+1]]

    @property
    def n_docs(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def doc(self, d: int) -> bytes:
        return self.data[self.offsets[d]:self.offsets[d + 1]].tobytes()

    def docs(self):
        return [self.doc(d) for d in range(self.n_docs)]


def _word(rng: np.random.Generator) -> str:
    kind = rng.random()
    n = int(min(12, 1 + rng.geometric(0.22)))
    if kind < 0.55:
        w = "".join(rng.choice(_LOWER, n))
    elif kind < 0.65:
        w = rng.choice(_UPPER) + "".join(rng.choice(_LOWER, max(0, n - 1)))
    elif kind < 0.70:
        w = "".join(rng.choice(_LOWER + _LATIN1, n))
    elif kind < 0.72:
        w = rng.choice(_LATIN1_UP) + "".join(rng.choice(_LATIN1, max(0, n - 1)))
    elif kind < 0.77:
        w = "".join(rng.choice(_GREEK + _GREEK_UP[:4], n))
    elif kind < 0.82:
        w = "".join(rng.choice(_CYRILLIC + _CYRILLIC_UP[:4], n))
    elif kind < 0.86:
        w = "".join(rng.choice(_CJK, max(1, n // 3)))
    elif kind < 0.90:
        w = "".join(rng.choice(_DIGITS, n))
    elif kind < 0.91:
        w = "".join(rng.choice(_ARABIC_DIGITS, n))
    elif kind < 0.94:
        w = "".join(rng.choice(_LOWER, n)) + "_" + "".join(rng.choice(_DIGITS, 2))
    elif kind < 0.95:
        w = "İ" + "".join(rng.choice(_LOWER, n))
    elif kind < 0.96:
        k = int(rng.integers(1, n + 1))
        w = "".join(rng.choice(_LOWER, k)) + "́" + "".join(rng.choice(_LOWER, n))
    else:
        w = "".join(rng.choice(_UPPER, n))
    return w


def make_lexicon(n_words: int, seed: int):
    """(bytes pool uint8, word offsets int64[n+1]) of n seeded word forms."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([60013, seed])))
    enc = [_word(rng).encode("utf-8") for _ in range(n_words)]
    off = np.zeros(n_words + 1, dtype=np.int64)
    np.cumsum([len(e) for e in enc], out=off[1:])
    return np.frombuffer(b"".join(enc), dtype=np.uint8), off


def _separator_pool():
    enc = [s.encode("utf-8") for s in _SEPARATORS] + [b" \xff "]  # one invalid byte
    off = np.zeros(len(enc) + 1, dtype=np.int64)
    np.cumsum([len(e) for e in enc], out=off[1:])
    return np.frombuffer(b"".join(enc), dtype=np.uint8), off


def make_text_corpus(n_docs: int, seed: int = 0, lexicon: int = 50_000, zipf_s: float = 1.05,
                     mean_words: float = 60.0, sigma: float = 0.5) -> TextCorpus:
    """n_docs documents of log-normal word counts (mean `mean_words`, at least 0 words), words
    drawn from a Zipf law over the lexicon, joined by separators."""
    lex, lex_off = make_lexicon(lexicon, seed)
    sep, sep_off = _separator_pool()
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([60017, seed])))
    n_words = sample_doc_lengths(n_docs, mean_words, sigma, 60019 + seed, min_len=0)
    total = int(n_words.sum())
    words = sample_zipf(zipf_cdf(lexicon, zipf_s), total, 60023 + seed).astype(np.int64)
    # separator after every word but the last of its document; invalid bytes are rare
    sep_p = np.ones(len(_SEPARATORS) + 1)
    sep_p[-1] = 0.02
    sep_p /= sep_p.sum()
    seps = rng.choice(len(sep_p), size=total, p=sep_p)
    ends = np.cumsum(n_words)
    last = np.zeros(total, dtype=bool)
    last[ends[n_words > 0] - 1] = True
    w_len = lex_off[words + 1] - lex_off[words]
    s_len = np.where(last, 0, sep_off[seps + 1] - sep_off[seps])
    # pieces in output order: word 0, separator 0, word 1, ...
    p_src = np.empty(2 * total, dtype=np.int64)
    p_len = np.empty(2 * total, dtype=np.int64)
    p_src[0::2] = lex_off[words]
    p_len[0::2] = w_len
    p_src[1::2] = lex.shape[0] + sep_off[seps]
    p_len[1::2] = s_len
    pool = np.concatenate([lex, sep])
    p_out = np.concatenate([[0], np.cumsum(p_len)])
    data = np.empty(int(p_out[-1]), dtype=np.uint8)
    step = 1 << 22
    for lo in range(0, 2 * total, step):
        hi = min(2 * total, lo + step)
        ln = p_len[lo:hi]
        base = p_out[lo:hi]
        idx = np.repeat(p_src[lo:hi] - base, ln) + np.arange(p_out[lo], p_out[hi])
        data[p_out[lo]:p_out[hi]] = pool[idx]
    doc_end_piece = 2 * ends  # piece index one past each document's last separator slot
    offsets = np.zeros(n_docs + 1, dtype=np.int64)
    offsets[1:] = p_out[doc_end_piece]
    return TextCorpus(data, offsets)


def make_text_queries(n: int, seed: int = 1, lexicon: int = 50_000, zipf_s: float = 1.05,
                      corpus_seed: int = 0) -> TextCorpus:
    """Short texts (1-8 words) over the same lexicon as the corpus of `corpus_seed`, with some
    words the corpus may not hold (drawn from the lexicon's tail)."""
    lex, lex_off = make_lexicon(lexicon, corpus_seed)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([60029, seed])))
    cdf = zipf_cdf(lexicon, zipf_s)
    out = []
    for _ in range(n):
        m = int(rng.integers(1, 9))
        ids = np.minimum(np.searchsorted(cdf, rng.random(m), side="right"), lexicon - 1)
        ws = [lex[lex_off[i]:lex_off[i + 1]].tobytes() for i in ids]
        out.append(b" ".join(ws))
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum([len(o) for o in out], out=off[1:])
    return TextCorpus(np.frombuffer(b"".join(out), dtype=np.uint8).copy(), off)
