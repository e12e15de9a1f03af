"""Pins of the tokenization oracle (Section 2, "Tokenization"): hand-split examples read off the
definition of the pattern (runs of two or more Unicode word characters), scikit-learn's own
analyzer with the same token pattern (the library the paper takes the pattern from), and the
first-occurrence order of the dictionary."""
import numpy as np
import pytest

from oracle import tokenize as T
from workloads.text import make_text_corpus, make_text_queries

CASES = [
    (b"Hello, world! a b_c 123 x-ray", False, ["Hello", "world", "b_c", "123", "ray"]),
    ("naïve café Ωμέγα 東京 ü".encode(), False, ["naïve", "café", "Ωμέγα", "東京"]),
    # U+0301 (combining acute) is not a word character: it splits "ab" + "cd"
    ("ab\u0301cd e\u0301f \u00e9f".encode(), False, ["ab", "cd", "\u00e9f"]),
    ("٣٤ x٣".encode(), False, ["٣٤", "x٣"]),
    (b"ab\xffcd \xff\xfe", False, ["ab", "cd"]),       # invalid bytes separate words
    (b"", False, []),
    (b"HELLO World", True, ["hello", "world"]),
    # U+0130 lowercases to "i" + U+0307 (not a word character): "i" alone is too short
    ("İstanbul İİ".encode(), True, ["stanbul"]),
    ("İstanbul".encode(), False, ["İstanbul"]),
    (b"__ _ a_", False, ["__", "a_"]),
]


@pytest.mark.parametrize("text,lower,want", CASES)
def test_hand_split_examples(text, lower, want):
    assert T.split(text, lower) == want


@pytest.mark.parametrize("lower", [False, True])
def test_split_matches_scikit_learn_analyzer(lower):
    from sklearn.feature_extraction.text import CountVectorizer
    an = CountVectorizer(token_pattern=r"(?u)\b\w\w+\b", lowercase=lower).build_analyzer()
    c = make_text_corpus(300, seed=3, lexicon=3000)
    for d in range(c.n_docs):
        text = c.doc(d)
        assert T.split(text, lower) == an(text.decode("utf-8", errors="replace")), d


def test_vocabulary_first_occurrence_order_and_round_trip():
    c = make_text_corpus(400, seed=4, lexicon=2000)
    ids, off, words = T.build_vocab(c.docs())
    assert off[0] == 0 and off[-1] == ids.size and np.all(np.diff(off) >= 0)
    assert len(set(words)) == len(words)
    # id i first appears before id i + 1
    first = np.full(len(words), -1)
    for p, i in enumerate(ids.tolist()):
        if first[i] < 0:
            first[i] = p
    assert np.all(np.diff(first) > 0) and first[0] == 0
    for d in range(c.n_docs):
        assert [words[i] for i in ids[off[d]:off[d + 1]]] == T.split(c.doc(d))


def test_query_mapping_drops_unknown_words():
    ids, off, words = T.build_vocab([b"alpha beta", b"gamma alpha"])
    assert words == ["alpha", "beta", "gamma"]
    q_ids, q_off = T.map_queries([b"beta delta alpha", b"", b"zeta"], words)
    assert q_ids.tolist() == [1, 0] and q_off.tolist() == [0, 2, 2, 2]
    q = make_text_queries(50, seed=2, lexicon=2000, corpus_seed=4)
    c = make_text_corpus(400, seed=4, lexicon=2000)
    _, _, words = T.build_vocab(c.docs())
    q_ids, q_off = T.map_queries(q.docs(), words)
    for i in range(q.n_docs):
        want = [words.index(w) for w in T.split(q.doc(i)) if w in words]
        assert q_ids[q_off[i]:q_off[i + 1]].tolist() == want
