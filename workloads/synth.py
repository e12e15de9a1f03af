"""Seeded synthetic corpora and query batches.

Every array is drawn on the host with NumPy's PCG64 generator. Large arrays are drawn in fixed-size
chunks; chunk ``j`` of stream ``(seed)`` uses ``SeedSequence([seed, j])``, so the result does not
depend on how many threads run the chunks.

Recipes (the paper measures on public retrieval benchmarks; these synthetic inputs stand in for
them with the shapes of the workloads below):

* token ids follow a bounded Zipf law, P(id = r-1) proportional to r**-s for r = 1..V, sampled by
  inverse CDF over an FP64 table, so id 0 is the most frequent token;
* document lengths are max(1, rint(X)) with X log-normal; the log-mean is ln(mean) - sigma**2/2 so
  that ``mean`` is the distribution mean;
* query token ids are drawn from the same Zipf law as the corpus; repeated ids are kept.

Seeds: config ``c`` uses seed ``1000*c + j`` for stream ``j``: 0 document lengths, 1 document
tokens, 2 query lengths, 3 query tokens, 4 arrival times, 5 per-query k.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

CHUNK = 1 << 22  # draws per chunk; fixed so that results do not depend on the thread count

# Workload recipes. "n_docs"/"vocab" may be overridden by callers that need a smaller copy of the
# same distribution (parity tests at oracle-friendly sizes).
CONFIGS = {
    0: dict(name="lucene-2k-docs-top10", n_docs=2_000, vocab=5_000, zipf_s=1.1, len_mean=60.0,
            len_sigma=0.5, n_queries=200, qlen=("uniform", 1, 8), k=10, variant="lucene",
            k1=1.5, b=0.75, delta=0.0, dtype="f32"),
    1: dict(name="lucene-1M-docs-top100-per-query", n_docs=1_000_000, vocab=1_000_000,
            zipf_s=1.07, len_mean=80.0, len_sigma=0.6, n_queries=10_000,
            qlen=("geometric", 1.0 / 6.0, 0, 32), k=100, variant="lucene", k1=1.5, b=0.75,
            delta=0.0, dtype="f32"),
    2: dict(name="lucene-8.8M-docs-top100-batched", n_docs=8_800_000, vocab=2_000_000,
            zipf_s=1.05, len_mean=60.0, len_sigma=0.5, n_queries=100_000,
            qlen=("geometric", 1.0 / 6.0, 1, 30), k=100, variant="lucene", k1=1.5, b=0.75,
            delta=0.0, dtype="f16", batch=4096),
    3: dict(name="shifted-5M-long-docs-top1000", n_docs=5_000_000, vocab=3_000_000,
            zipf_s=1.0, len_mean=300.0, len_sigma=0.7, n_queries=20_000,
            qlen=("uniform", 30, 200), k=1000, variant="bm25plus", k1=1.2, b=0.75, delta=1.0,
            dtype="bf16"),
    4: dict(name="serving-on-8.8M-docs", n_docs=8_800_000, vocab=2_000_000, zipf_s=1.05,
            len_mean=60.0, len_sigma=0.5, n_queries=200_000, qlen=("zipf", 1.1, 64),
            k=(10, 100, 1000), variant="lucene", k1=1.5, b=0.75, delta=0.0, dtype="f16",
            rates=(20_000, 50_000, 100_000)),
}


@dataclass
class Corpus:
    tokens: np.ndarray        # int32[T], documents back to back
    doc_offsets: np.ndarray   # int64[N+1], offsets[0] = 0, offsets[N] = T
    vocab: int                # ids are in [0, vocab)
    recipe: dict = field(default_factory=dict)

    @property
    def n_docs(self) -> int:
        return int(self.doc_offsets.shape[0] - 1)

    @property
    def n_tokens(self) -> int:
        return int(self.tokens.shape[0])

    def doc(self, d: int) -> np.ndarray:
        return self.tokens[self.doc_offsets[d]:self.doc_offsets[d + 1]]


@dataclass
class QueryBatch:
    q_ids: np.ndarray       # int32[sum |Q|]
    q_offsets: np.ndarray   # int64[B+1]
    k: np.ndarray           # int32[B]

    @property
    def n(self) -> int:
        return int(self.q_offsets.shape[0] - 1)

    def query(self, i: int) -> np.ndarray:
        return self.q_ids[self.q_offsets[i]:self.q_offsets[i + 1]]

    def slice(self, lo: int, hi: int) -> "QueryBatch":
        base = self.q_offsets[lo]
        return QueryBatch(self.q_ids[base:self.q_offsets[hi]].copy(),
                          (self.q_offsets[lo:hi + 1] - base).astype(np.int64),
                          self.k[lo:hi].copy())


def _threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(16, n))


def zipf_cdf(vocab: int, s: float) -> np.ndarray:
    """FP64 CDF of the bounded Zipf law P(r) ~ r**-s over r = 1..vocab (last entry exactly 1)."""
    r = np.arange(1, vocab + 1, dtype=np.float64)
    w = r ** (-float(s))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    return cdf


def _chunked(n: int, seed: int, fill) -> None:
    """Run fill(rng, lo, hi) over fixed chunks of [0, n), chunk j seeded by [seed, j]."""
    nchunks = (n + CHUNK - 1) // CHUNK

    def work(j):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, j])))
        lo = j * CHUNK
        fill(rng, lo, min(n, lo + CHUNK))

    if nchunks <= 1:
        for j in range(nchunks):
            work(j)
        return
    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(work, range(nchunks)))


def sample_zipf(cdf: np.ndarray, n: int, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int32)
    last = cdf.shape[0] - 1

    def fill(rng, lo, hi):
        u = rng.random(hi - lo)
        idx = np.searchsorted(cdf, u, side="right")
        np.minimum(idx, last, out=idx)
        out[lo:hi] = idx

    _chunked(n, seed, fill)
    return out


def sample_doc_lengths(n_docs: int, mean: float, sigma: float, seed: int,
                       min_len: int = 1) -> np.ndarray:
    mu = np.log(mean) - 0.5 * sigma * sigma
    out = np.empty(n_docs, dtype=np.int64)

    def fill(rng, lo, hi):
        x = rng.lognormal(mean=mu, sigma=sigma, size=hi - lo)
        out[lo:hi] = np.maximum(min_len, np.rint(x)).astype(np.int64)

    _chunked(n_docs, seed, fill)
    return out


def make_corpus(cfg: int, n_docs: int | None = None, vocab: int | None = None) -> Corpus:
    """Corpus of config ``cfg``; ``n_docs``/``vocab`` override the sizes, not the distributions."""
    r = dict(CONFIGS[cfg])
    if n_docs is not None:
        r["n_docs"] = int(n_docs)
    if vocab is not None:
        r["vocab"] = int(vocab)
    lengths = sample_doc_lengths(r["n_docs"], r["len_mean"], r["len_sigma"], 1000 * cfg + 0)
    offsets = np.zeros(r["n_docs"] + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    cdf = zipf_cdf(r["vocab"], r["zipf_s"])
    tokens = sample_zipf(cdf, int(offsets[-1]), 1000 * cfg + 1)
    return Corpus(tokens, offsets, r["vocab"], r)


def _query_lengths(qlen, n: int, rng: np.random.Generator) -> np.ndarray:
    kind = qlen[0]
    if kind == "uniform":
        return rng.integers(qlen[1], qlen[2] + 1, size=n).astype(np.int64)
    if kind == "geometric":
        # qlen = ("geometric", p, add, cap): min(add + Geom(p), cap), Geom on {1, 2, ...}
        g = rng.geometric(qlen[1], size=n).astype(np.int64) + int(qlen[2])
        return np.minimum(g, int(qlen[3]))
    if kind == "zipf":
        # P(L) ~ L**-a on 1..cap
        a, cap = qlen[1], qlen[2]
        c = zipf_cdf(cap, a)
        return np.searchsorted(c, rng.random(n), side="right").astype(np.int64) + 1
    raise ValueError(kind)


def make_queries(cfg: int, n_queries: int | None = None, vocab: int | None = None,
                 k: int | None = None) -> QueryBatch:
    r = dict(CONFIGS[cfg])
    if vocab is not None:
        r["vocab"] = int(vocab)
    n = int(n_queries if n_queries is not None else r["n_queries"])
    rng_len = np.random.Generator(np.random.PCG64(1000 * cfg + 2))
    lengths = _query_lengths(r["qlen"], n, rng_len)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    cdf = zipf_cdf(r["vocab"], r["zipf_s"])
    ids = sample_zipf(cdf, int(offsets[-1]), 1000 * cfg + 3)
    if k is not None:
        kk = np.full(n, int(k), dtype=np.int32)
    elif isinstance(r["k"], tuple):
        rng_k = np.random.Generator(np.random.PCG64(1000 * cfg + 5))
        kk = np.asarray(r["k"], dtype=np.int32)[rng_k.integers(0, len(r["k"]), size=n)]
    else:
        kk = np.full(n, int(r["k"]), dtype=np.int32)
    return QueryBatch(ids, offsets, kk)


def poisson_arrivals(rate: float, n: int, seed: int) -> np.ndarray:
    """Arrival times in seconds of an open-loop Poisson process with the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def make_tiny_corpus(seed: int, max_docs: int = 40, max_vocab: int = 30, max_len: int = 12,
                     empty_prob: float = 0.1) -> Corpus:
    """Small random corpus with forced repeats, shared tokens and some empty documents."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([7919, seed])))
    n = int(rng.integers(1, max_docs + 1))
    v = int(rng.integers(1, max_vocab + 1))
    skew = bool(rng.integers(0, 2))
    lengths = rng.integers(0, max_len + 1, size=n)
    lengths[rng.random(n) < empty_prob] = 0
    if lengths.sum() == 0:
        lengths[0] = 1
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    if skew:
        cdf = zipf_cdf(v, 1.2)
        tokens = np.searchsorted(cdf, rng.random(int(offsets[-1])), side="right")
        tokens = np.minimum(tokens, v - 1).astype(np.int32)
    else:
        tokens = rng.integers(0, v, size=int(offsets[-1])).astype(np.int32)
    # duplicate some documents exactly, which forces tied scores
    if n >= 4:
        tokens = tokens.copy()
        for _ in range(int(rng.integers(0, 3))):
            a, c = rng.integers(0, n, size=2)
            if lengths[a] == lengths[c] and a != c:
                tokens[offsets[c]:offsets[c + 1]] = tokens[offsets[a]:offsets[a + 1]]
    return Corpus(tokens, offsets, v, dict(name=f"tiny-{seed}"))


def make_tiny_queries(seed: int, vocab: int, n: int = 6, max_len: int = 6) -> QueryBatch:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([104729, seed])))
    lengths = rng.integers(0, max_len + 1, size=n)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    ids = rng.integers(0, vocab, size=int(offsets[-1])).astype(np.int32)
    # repeat a token inside some queries (duplicates count once per position)
    for i in range(n):
        lo, hi = offsets[i], offsets[i + 1]
        if hi - lo >= 2 and rng.random() < 0.5:
            ids[hi - 1] = ids[lo]
    k = rng.integers(1, 12, size=n).astype(np.int32)
    return QueryBatch(ids, offsets, k)
