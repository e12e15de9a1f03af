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


# -- Robertson, ATIRE and TF_ldp ------------------------------------------------------------------
# Hand-derived on the same corpus (see each fixture section's "_about"). Every decimal is checked
# against its closed form, evaluated by ``_closed`` from the fixture's text alone, and the oracle
# (eager and brute force) against the decimals.

_VID = {"robertson": 3, "atire": 4, "tfldp": 5}


def _closed(expr: str) -> float:
    """Evaluates a closed form of the fixture: numbers, + - * / ( ) and the natural log ln."""
    import math
    import re
    if not re.fullmatch(r"[0-9.+\-*/() ln]*", expr):
        raise ValueError(f"unexpected closed form {expr!r}")
    return float(eval(expr, {"__builtins__": {}}, {"ln": math.log}))  # noqa: S307


def _closed_pairs(sec):
    """(closed form, decimal) pairs of one fixture section, queries included."""
    pairs = []
    for key in ("idf", "theta", "data"):
        if key + "_closed_form" in sec:
            pairs += list(zip(sec[key + "_closed_form"], sec[key]))
    for q in sec.get("queries", []):
        pairs += list(zip(q.get("B_closed_form", []), q["B"]))
        if "shift_closed_form" in q:
            pairs.append((q["shift_closed_form"], q["shift"]))
            pairs += list(zip(q["sum_delta_closed_form"], q["sum_delta"]))
    return pairs


@pytest.mark.parametrize("name", ["robertson", "atire", "tfldp"])
def test_variant_fixture_closed_forms(name):
    pairs = _closed_pairs(GOLD[name])
    assert len(pairs) >= 16
    for form, dec in pairs:
        assert _closed(form) == pytest.approx(dec, rel=1e-14, abs=1e-15), form


@pytest.mark.parametrize("name", ["robertson", "atire", "tfldp"])
def test_variant_worked_example(name):
    tokens, offsets = _corpus()
    g = GOLD[name]
    delta = g.get("delta", 0.0)
    idx = eager.build_index(tokens, offsets, GOLD["vocab"], GOLD["k1"], GOLD["b"], delta, name)
    np.testing.assert_array_equal(idx.df, GOLD["lucene"]["df"])
    np.testing.assert_allclose(idx.idf, g["idf"], rtol=1e-14)
    np.testing.assert_allclose(idx.data, g["data"], rtol=1e-14)
    np.testing.assert_allclose(idx.theta, g.get("theta", np.zeros(4)), rtol=1e-14)
    for q in g["queries"]:
        b = eager.scores(idx, q["q"])
        np.testing.assert_allclose(b, q["B"], rtol=1e-14, atol=1e-15)
        ids, _ = eager.search(idx, q["q"], 3)
        assert list(ids) == q["top3"], q["q"]
        if "shift" in q:
            np.testing.assert_allclose(eager.shift(idx, q["q"]), q["shift"], rtol=1e-14)
            np.testing.assert_allclose(eager.slice_sum(idx, q["q"]), q["sum_delta"], rtol=1e-13,
                                       atol=1e-15)
        bb = brute.brute_scores(GOLD["docs"], q["q"], GOLD["k1"], GOLD["b"], delta, _VID[name])
        np.testing.assert_allclose(bb, q["B"], rtol=1e-14, atol=1e-15)
        assert brute.brute_topk(bb, 3) == q["top3"]


def test_lucene_and_shifted_fixture_closed_forms():
    """The Lucene, BM25+ and BM25L decimals against their closed forms, by the same evaluator."""
    pairs = _closed_pairs(GOLD["lucene"])
    for name in ("bm25plus", "bm25l"):
        g = GOLD[name]
        pairs += list(zip(g["theta_closed_form"], g["theta"]))
        pairs += list(zip(g["B_closed_form"], g["B"]))
        pairs += list(zip(g["sum_delta_closed_form"], g["sum_delta"]))
        pairs.append((g["shift_closed_form"], g["shift"]))
    for form, dec in pairs:
        form = form.replace("ln ", "ln").replace("ln2", "ln(2)").replace("ln4", "ln(4)")
        assert _closed(form) == pytest.approx(dec, rel=1e-14, abs=1e-15), form
