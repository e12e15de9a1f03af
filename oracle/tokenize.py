"""Tokenization and vocabulary mapping in plain Python (the step in front of the hot path).

Test infrastructure only (see the package docstring).

Section 2 ("Tokenization"): the text is split with the regular expression scikit-learn uses for
its tokenizers, (?u)\\b\\w\\w+\\b, so a token is a maximal run of at least two Unicode word
characters; then a dictionary maps each distinct word to an integer index, and the documents'
words become their indices. Readings where the paper is silent:

* Ids are given in order of first occurrence in the corpus (documents in order, words in order
  inside a document), which is what filling a dictionary while reading the corpus gives.
* Text arrives as UTF-8 bytes, one byte string per document; bytes that are not valid UTF-8 are
  decoded as replacement characters (which are not word characters, so they separate words).
* Lowercasing is optional and is Python's str.lower() of the decoded text, before splitting.
* Stemming and stopword removal are not applied.
* A query word that is not in the corpus dictionary has no index and is dropped (it would score
  0 against every document).
"""
from __future__ import annotations

import re

import numpy as np

TOKEN_PATTERN = re.compile(r"(?u)\b\w\w+\b")


def split(text: bytes, lowercase: bool = False) -> list:
    """The words of one UTF-8 document."""
    s = text.decode("utf-8", errors="replace")
    if lowercase:
        s = s.lower()
    return TOKEN_PATTERN.findall(s)


def build_vocab(docs, lowercase: bool = False):
    """Tokenizes a corpus: returns (token_ids int32[T], doc_offsets int64[N+1], words) where
    words[i] is the word of id i."""
    vocab = {}
    ids = []
    offsets = [0]
    for d in docs:
        for w in split(d, lowercase):
            if w not in vocab:
                vocab[w] = len(vocab)
            ids.append(vocab[w])
        offsets.append(len(ids))
    words = [None] * len(vocab)
    for w, i in vocab.items():
        words[i] = w
    return (np.asarray(ids, dtype=np.int32), np.asarray(offsets, dtype=np.int64), words)


def map_queries(queries, words, lowercase: bool = False):
    """Ids of the queries' words in a corpus dictionary (unknown words dropped): returns
    (ids int32, offsets int64[n+1])."""
    vocab = {w: i for i, w in enumerate(words)}
    ids = []
    offsets = [0]
    for q in queries:
        for w in split(q, lowercase):
            if w in vocab:
                ids.append(vocab[w])
        offsets.append(len(ids))
    return np.asarray(ids, dtype=np.int32), np.asarray(offsets, dtype=np.int64)
