"""Seeded synthetic inputs shared by the oracle-side tests, the GPU tests and the benchmark.

This package generates corpora (pre-tokenized integer ids, grouped by document) and query
batches. It holds none of the BM25 arithmetic: no term frequencies, document frequencies,
IDF or scores are computed here.
"""
from .synth import (  # noqa: F401
    CONFIGS,
    Corpus,
    QueryBatch,
    make_corpus,
    make_queries,
    make_tiny_corpus,
    make_tiny_queries,
    zipf_cdf,
)
