"""FP64 CPU oracle for BM25S eager sparse scoring (arXiv 2407.03618).

TEST INFRASTRUCTURE ONLY. Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import anything in this package. The product path (the HIP library and
its Python binding) never imports, links or calls it, and shares no code with it.

Three independent implementations of what the hot path computes:

* ``eager``  -- the paper's method in FP64: token-major sparse score matrix built at index time,
  query-time slice-and-sum of the query's rows, then top-k (Section 2).
* ``scan``   -- the plain definition B(Q, D) = sum_i S(q_i, D), evaluated per query directly from
  the documents' tokens with no sparse matrix and no score shifting.
* ``brute``  -- pure-Python dictionaries, for tiny corpora; shares no code with the other two.

Readings of passages where the paper is silent or ambiguous are stated in the docstrings of
``formulas``; the variant formulas other than Lucene's are not printed in the paper and their
parity is unpinned by it (their internal consistency is pinned by hand-derived examples).
"""
from .formulas import (  # noqa: F401
    ATIRE, BM25L, BM25PLUS, LUCENE, ROBERTSON, SHIFTED, TFLDP, VARIANTS, idf, nonoccurrence,
    saturation, variant_id,
)
from .eager import EagerIndex, build_index, search, search_batch, topk  # noqa: F401
from .scan import direct_scores  # noqa: F401
