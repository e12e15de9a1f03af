"""Oracle pins: the hand-derived worked example (tests/golden/w1_worked_example.json).

The paper prints no worked example, so the fixture holds closed forms derived by hand from the
equations of Section 2 (Lucene) and Section 2.1 (BM25+, BM25L shifting), written as decimals.
"""
import json
import os

import numpy as np
import pytest

from oracle import brute, eager

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "w1_worked_example.json")))


def _corpus():
    docs = GOLD["docs"]
    tokens = np.array([t for d in docs for t in d], dtype=np.int32)
    offsets = np.zeros(len(docs) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([len(d) for d in docs])
    return tokens, offsets


def test_lucene_index_arrays():
    tokens, offsets = _corpus()
    g = GOLD["lucene"]
    idx = eager.build_index(tokens, offsets, GOLD["vocab"], GOLD["k1"], GOLD["b"], 0.0, "lucene")
    assert idx.sum_len == 9 and idx.l_avg == 3.0
    np.testing.assert_array_equal(idx.df, g["df"])
    np.testing.assert_array_equal(idx.indptr, g["indptr"])
    np.testing.assert_array_equal(idx.indices, g["indices"])
    np.testing.assert_array_equal(idx.tf, g["tf"])
    np.testing.assert_allclose(idx.idf, g["idf"], rtol=1e-14)
    np.testing.assert_allclose(idx.data, g["data"], rtol=1e-14)
    np.testing.assert_array_equal(idx.theta, 0.0)


@pytest.mark.parametrize("case", range(len(GOLD["lucene"]["queries"])))
def test_lucene_query_scores_and_order(case):
    tokens, offsets = _corpus()
    g = GOLD["lucene"]["queries"][case]
    idx = eager.build_index(tokens, offsets, GOLD["vocab"], GOLD["k1"], GOLD["b"], 0.0, "lucene")
    b = eager.scores(idx, g["q"])
    np.testing.assert_allclose(b, g["B"], rtol=1e-14, atol=1e-15)
    ids, s = eager.search(idx, g["q"], 3)
    assert list(ids) == g["top3"]
    # the brute force reaches the same numbers and order
    bb = brute.brute_scores(GOLD["docs"], g["q"], GOLD["k1"], GOLD["b"], 0.0, 0)
    np.testing.assert_allclose(bb, g["B"], rtol=1e-14, atol=1e-15)
    assert brute.brute_topk(bb, 3) == g["top3"]


@pytest.mark.parametrize("name,vid", [("bm25plus", 2), ("bm25l", 1)])
def test_shifted_variant_worked_example(name, vid):
    tokens, offsets = _corpus()
    g = GOLD[name]
    idx = eager.build_index(tokens, offsets, GOLD["vocab"], GOLD["k1"], GOLD["b"], g["delta"],
                            name)
    np.testing.assert_allclose(idx.theta, g["theta"], rtol=1e-14)
    np.testing.assert_allclose(eager.shift(idx, g["q"]), g["shift"], rtol=1e-14)
    np.testing.assert_allclose(eager.slice_sum(idx, g["q"]), g["sum_delta"], rtol=1e-13)
    np.testing.assert_allclose(eager.scores(idx, g["q"]), g["B"], rtol=1e-14)
    bb = brute.brute_scores(GOLD["docs"], g["q"], GOLD["k1"], GOLD["b"], g["delta"], vid)
    np.testing.assert_allclose(bb, g["B"], rtol=1e-14)


def test_fixture_closed_forms_match_decimals():
    """The decimals in the fixture are the closed forms written next to them."""
    import math
    ln16, ln83, ln2 = math.log(1.6), math.log(8 / 3), math.log(2)
    lu = GOLD["lucene"]
    want = [ln16 * 4 / 7, ln16 * 8 / 23, ln16 * 2 / 5, ln16 * 8 / 17, ln83 * 8 / 17, ln83 * 8 / 13]
    np.testing.assert_allclose(lu["data"], want, rtol=1e-14)
    np.testing.assert_allclose(GOLD["bm25plus"]["B"], [ln2 * 31 / 7, ln2 * 54 / 17, ln2 * 66 / 23],
                               rtol=1e-14)
    np.testing.assert_allclose(GOLD["bm25l"]["B"], [ln16 * 45 / 16, 2 * ln16, ln16 * 25 / 14],
                               rtol=1e-14)
