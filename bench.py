"""Benchmark of the BM25S eager sparse scoring hot path on one MI355X.

Default workload: an 8.8M-document synthetic corpus (vocabulary 2M, Zipf s = 1.05 token ids,
log-normal lengths with mean 60), 4096-query batches (lengths 2-30, geometric, mean 7), top-100,
scores stored in FP16 and accumulated in FP32, batched form with the autotuned launch shape. A
step is one batch through the whole query path (grouping, plan, gather + accumulate, top-k,
merge with the shift); the index is built once, before the timed region, and its build rate is
reported separately.

Printed JSON line (stdout): value = queries/s over the timed steps; the roofline of the dominant
kernel (the batched gather) against every bound that applies to it; the FP64 CPU oracle timed on
a bounded sample of the same queries; sampled parity of every timed configuration against the
oracle with its error statistics; extra legs: batched FP32, the plain per-query FP32 form (on this
index and on the 1M-document workload), the 5M long-document BM25+ / BM25L bf16 top-1000
workload, HIP-graph launches, index build rates with their roofline, and open-loop serving
latency (p50/p99, queue wait and service time) at fixed arrival rates.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "queries/s + HBM GB/s, 8.8M-doc top-100 index; p50/p99 latency at fixed QPS"
HBM_PEAK_GBS = 8000.0
# FP32 VALU lane operations (an FMA, an add or a compare each) per second without packed math:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
KERNEL_SOURCES = ["paper_2407_03618_amd/csrc/search_kernels.hpp",
                  "paper_2407_03618_amd/csrc/device.hpp",
                  "paper_2407_03618_amd/csrc/search_inst.hip",
                  "paper_2407_03618_amd/build.py"]  # its compiler flags shape the kernel too
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_gather_8.8M-docs_4096-query_top100_f16_traffic.json")
DENSE_FRACTION = 16        # rows of tokens in >= N/16 documents also have a dense copy
DENSE_PAD = 4096           # dense rows are padded to a multiple of this many documents
DENSE_MAX_BYTES = 4 << 30  # at most this many bytes of dense rows


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, plan: dict):
    """HBM bytes per gather launch from the committed counter summary, if it was taken with the
    current kernel sources and the same launch shape."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    entry = t.get(workload)
    if not entry or entry.get("kernel_hash") != kernel_source_hash():
        return None
    if entry.get("plan") != plan:
        return None
    return entry.get("bytes_per_launch")


def algorithmic_bytes(df: np.ndarray, q_ids: np.ndarray, q_off: np.ndarray, k: np.ndarray,
                      s_bytes: int) -> np.ndarray:
    """Per query: sum_i DF(q_i) * (4 + s) + 16 |Q| + 8 k (postings read, row bounds, results)."""
    per_pos = df[q_ids].astype(np.int64) * (4 + s_bytes) + 16
    cs = np.concatenate([[0], np.cumsum(per_pos)])
    return (cs[q_off[1:]] - cs[q_off[:-1]]) + 8 * k.astype(np.int64)


def dense_tokens(df: np.ndarray, n_docs: int, s_bytes: int) -> np.ndarray:
    """Tokens whose rows the index also keeps dense (the library's rule: DF >= ceil(N / 16),
    at least 2, most frequent first, within the dense byte cap)."""
    min_df = max(2, -(-n_docs // DENSE_FRACTION))
    n_pad = -(-n_docs // DENSE_PAD) * DENSE_PAD
    cand = np.flatnonzero(df >= min_df)
    cap = DENSE_MAX_BYTES // (n_pad * s_bytes)
    if cand.size > cap:
        order = np.lexsort((cand, -df[cand]))
        cand = np.sort(cand[order[:cap]])
    return cand


def launch_work(df: np.ndarray, q_ids: np.ndarray, q_off: np.ndarray, k: int, n_docs: int,
                s_bytes: int) -> dict:
    """Work of one batched launch over the given queries:
    unique_bytes   every distinct row the batch touches, read once: its postings (4 + s bytes
                   each) for sparse rows, its dense copy (s bytes per padded document) for dense
                   rows; plus 16 bytes per position and 8 per result
    method_adds    sum over queries and positions of DF(q_i): the slice-and-sum additions
    issued_ops     FP32 lane operations the kernel issues: one FMA per document for each
                   (query, distinct dense token), one add per posting for each (query, distinct
                   sparse token), and one compare per (query, document) in the top-k scan
    select_ops     the compares alone"""
    dense = np.zeros(df.shape[0], bool)
    dense[dense_tokens(df, n_docs, s_bytes)] = True
    n_pad = -(-n_docs // DENSE_PAD) * DENSE_PAD
    n = q_off.shape[0] - 1
    uniq = np.unique(q_ids)
    ub = int(np.sum(np.where(dense[uniq], n_pad * s_bytes, df[uniq].astype(np.int64) * (4 + s_bytes))))
    ub += 16 * int(q_off[-1]) + 8 * k * n
    method = int(df[q_ids].astype(np.int64).sum())
    qi = np.repeat(np.arange(n, dtype=np.int64), np.diff(q_off))
    pairs = np.unique(qi * df.shape[0] + q_ids.astype(np.int64))
    tok = pairs % df.shape[0]
    dense_pairs = int(dense[tok].sum())
    sparse_adds = int(df[tok[~dense[tok]]].astype(np.int64).sum())
    select = n * n_docs
    return dict(unique_bytes=ub, method_adds=method, dense_fmas=dense_pairs * n_docs,
                sparse_adds=sparse_adds, select_ops=select,
                issued_ops=dense_pairs * n_docs + sparse_adds + select)


def roofline(work: dict, kernel_ms: float, traffic, no_reuse_bytes: float) -> dict:
    """Bounds of the gather kernel, each as the shortest time the kernel could take; the binding
    one (the longest) sets bound / achieved / peak / frac."""
    t = kernel_ms / 1e3
    bounds = {
        "hbm_unique_rows": dict(time_ms=work["unique_bytes"] / (HBM_PEAK_GBS * 1e9) * 1e3,
                                bytes=work["unique_bytes"]),
        "valu_issued": dict(time_ms=work["issued_ops"] / (VALU_PEAK_TOPS * 1e12) * 1e3,
                            ops=work["issued_ops"]),
        "valu_method": dict(time_ms=(work["method_adds"] + work["select_ops"]) /
                            (VALU_PEAK_TOPS * 1e12) * 1e3,
                            ops=work["method_adds"] + work["select_ops"]),
    }
    if traffic:
        bounds["hbm_traffic"] = dict(time_ms=traffic / (HBM_PEAK_GBS * 1e9) * 1e3, bytes=traffic)
    for b in bounds.values():
        b["frac"] = b["time_ms"] / kernel_ms
    measured = {k: v for k, v in bounds.items() if k != "valu_method"}
    bind = max(measured, key=lambda k: measured[k]["time_ms"])
    if bind.startswith("hbm"):
        achieved = bounds[bind]["bytes"] / t / 1e9
        out = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                   frac=achieved / HBM_PEAK_GBS)
    else:
        achieved = bounds[bind]["ops"] / t / 1e12
        out = dict(bound="alu", achieved=achieved, peak=VALU_PEAK_TOPS, unit="T lane-ops/s",
                   frac=achieved / VALU_PEAK_TOPS)
    out.update(traffic=traffic, binding=bind, kernel="k_gather", kernel_ms=kernel_ms,
               bounds=bounds,
               effective=dict(no_reuse_bytes_per_launch=no_reuse_bytes,
                              GBs=no_reuse_bytes / t / 1e9,
                              note="each query's postings counted once per query; the batched "
                                   "kernel shares rows across the queries of a tile, so this "
                                   "is not a bandwidth the kernel moves"))
    return out


def build_roofline(n_tokens: int, n_docs: int, nnz: int, vocab: int, s_bytes: int,
                   ms: float) -> dict:
    """A_build = 4T + 8(N+1) + nnz(4 + s + 4) + 20V bytes over the build's wall time."""
    a = 4 * n_tokens + 8 * (n_docs + 1) + nnz * (8 + s_bytes) + 20 * vocab
    ach = a / (ms / 1e3) / 1e9
    return dict(ms=ms, nnz_per_s=nnz / (ms / 1e3), algorithmic_bytes=a, achieved_GBs=ach,
                peak_GBs=HBM_PEAK_GBS, frac=ach / HBM_PEAK_GBS)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _spread(lo: int, hi: int, n: int) -> list:
    return sorted(set(np.linspace(lo, hi - 1, num=min(n, hi - lo)).astype(int).tolist()))


# ------------------------------------------------------------------------------------------
# GPU legs

def plain_1m_leg(nq: int, n_check: int) -> dict:
    """The per-query form on its configured workload: 1M documents (V = 1M, Zipf 1.07, mean length
    80), fp32 scores, top-100, one query per launch. Keeps sampled rows for the parity check."""
    import torch
    from paper_2407_03618_amd import Index
    from workloads import CONFIGS, make_corpus, make_queries
    cfg = CONFIGS[1]
    c = make_corpus(1)
    q = make_queries(1, n_queries=nq, vocab=c.vocab)
    dev = torch.device("cuda:0")
    idx = Index(torch.from_numpy(c.tokens).to(dev), torch.from_numpy(c.doc_offsets).to(dev),
                c.vocab, cfg["k1"], cfg["b"], cfg["delta"], cfg["variant"], "f32")
    qd = torch.from_numpy(q.q_ids).to(dev)
    out = idx._outputs(nq, 100)
    idx.search_plain(qd, q.q_offsets, 100, 100, out=out)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    idx.search_plain(qd, q.q_offsets, 100, 100, out=out)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sample = _spread(0, nq, n_check)
    rows = [t.cpu().numpy()[sample] for t in out]
    res = dict(qps=nq / el, ms_per_query=el / nq * 1e3, n_docs=c.n_docs, nnz=idx.nnz, queries=nq)
    idx.free()
    return res, dict(queries=[q.query(i).copy() for i in sample], rows=rows, k=100)


def tokenize_leg(n_docs: int, n_check: int, n_queries: int = 4096) -> tuple:
    """Tokenization in front of the path (Section 2, "Tokenization"): a seeded multi-script UTF-8
    corpus split on the GPU into words of two or more word characters, lowercased, with a device
    dictionary giving first-occurrence ids (timed after one untimed run); then query texts mapped
    through the dictionary. Keeps the GPU's words of sampled documents, to be checked against the
    oracle's split (the words behind the ids, which do not depend on the order ids are given)."""
    import torch
    from paper_2407_03618_amd import Vocab
    from workloads.text import make_text_corpus, make_text_queries
    lexicon = 200_000
    c = make_text_corpus(n_docs, seed=11, lexicon=lexicon)
    q = make_text_queries(n_queries, seed=12, lexicon=lexicon, corpus_seed=11)
    dev = torch.device("cuda:0")
    text, off = torch.from_numpy(c.data).to(dev), torch.from_numpy(c.offsets).to(dev)
    qt, qo = torch.from_numpy(q.data).to(dev), torch.from_numpy(q.offsets).to(dev)
    Vocab(text, off, lowercase=True).free()  # first run: grows the caching allocator
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    v = Vocab(text, off, lowercase=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    v.map(qt, qo)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    qids, _ = v.map(qt, qo)
    torch.cuda.synchronize()
    mel = time.perf_counter() - t0
    ids, doff = v.corpus()
    ids, doff = ids.cpu().numpy(), doff.cpu().numpy()
    words = v.words()
    sample = _spread(0, n_docs, n_check)
    rows = [(c.doc(d), [words[i] for i in ids[doff[d]:doff[d + 1]]]) for d in sample]
    res = dict(docs=n_docs, bytes=int(c.data.size), tokens=v.n_tokens, vocab=v.vocab_size,
               ms=el * 1e3, GB_per_s=c.data.size / el / 1e9, tokens_per_s=v.n_tokens / el,
               map_queries=n_queries, map_ids=int(qids.numel()), map_ms=mel * 1e3,
               map_queries_per_s=n_queries / mel, lowercase=True)
    v.free()
    return res, dict(rows=rows)


def long_docs_leg(n_check: int, n_batches: int = 4, batch: int = 512) -> tuple:
    """The shifted-variant workload at full size: 5M long documents (mean 300 ids, V = 3M,
    Zipf 1.0), BM25+ (delta = 1) and BM25L (delta = 0.5), k1 = 1.2, b = 0.75, bf16 scores,
    30-200-id queries, top-1000, batched form. Keeps sampled rows of each for the parity check."""
    import torch
    from paper_2407_03618_amd import Index
    from workloads import CONFIGS, make_corpus, make_queries
    cfg = CONFIGS[3]
    c = make_corpus(3)
    q = make_queries(3, n_queries=batch * (n_batches + 1), vocab=c.vocab)
    dev = torch.device("cuda:0")
    tok = torch.from_numpy(c.tokens).to(dev)
    off = torch.from_numpy(c.doc_offsets).to(dev)
    qd = torch.from_numpy(q.q_ids).to(dev)
    k = int(cfg["k"])
    sample = _spread(0, batch, n_check)
    legs, checks = {}, {}
    for variant, delta in (("bm25plus", 1.0), ("bm25l", 0.5)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        idx = Index(tok, off, c.vocab, cfg["k1"], cfg["b"], delta, variant, "bf16")
        torch.cuda.synchronize()
        build_ms = (time.perf_counter() - t0) * 1e3
        out = idx._outputs(batch, k)
        idx.search_batch(qd, q.q_offsets[:batch + 1], k, k, out=out)  # warm-up, parity rows
        torch.cuda.synchronize()
        rows = [t.cpu().numpy()[sample] for t in out]
        t0 = time.perf_counter()
        for b in range(1, n_batches + 1):
            o = q.q_offsets[b * batch:(b + 1) * batch + 1]
            base = int(o[0])
            idx.search_batch(qd[base:], o - base, k, k, out=out)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        legs[variant] = dict(qps=n_batches * batch / el, ms_per_batch=el / n_batches * 1e3,
                             batch=batch, k=k, n_docs=c.n_docs, nnz=idx.nnz, build_ms=build_ms,
                             build_nnz_per_s=idx.nnz / (build_ms / 1e3), delta=delta,
                             dtype="bf16", range=idx.range_stats())
        checks[variant] = dict(rows=rows, k=k, delta=delta)
        log(f"[long docs {variant}]", legs[variant])
        idx.free()
        del out
        torch.cuda.empty_cache()
    return legs, checks, [q.query(i).copy() for i in sample]


def graph_leg(idx, q_dev, queries, k, first, full_batch, reps=40, small=64) -> dict:
    """Eager launches against one HIP graph launch per batch (graph mode), on 64-query
    micro-batches (where launch gaps weigh most) and on full batches."""
    import torch
    res = {}
    for name, n, r in (("micro_batch_64", small, reps), ("batch_full", full_batch, 4)):
        out = idx._outputs(n, k)

        def run(i):
            lo = first + i * n
            off = queries.q_offsets[lo:lo + n + 1]
            base = int(off[0])
            idx.search_batch(q_dev[base:], off - base, k, k, out=out)

        row = {}
        for mode in (False, True):
            idx.set_graphs(mode)
            run(0)
            run(1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(r):
                run(i % 2)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / r
            row["graph" if mode else "eager"] = dict(ms_per_batch=dt * 1e3, qps=n / dt)
        idx.set_graphs(False)
        res[name] = row
    res["graph_stats"] = idx.graph_stats()
    return res


def serving_leg(idx, corpus, rates, seconds, warmup_s, budget, n_check):
    """Open-loop Poisson arrivals at fixed rates over the resident index. Each rate runs
    warmup_s + seconds of arrivals; statistics cover the requests that arrive after warmup_s.
    A separate short window at the lowest rate keeps its result rows for the parity check."""
    from paper_2407_03618_amd import Server
    from workloads import make_queries
    from workloads.synth import poisson_arrivals
    out = []
    srv = Server(idx, hbm_budget_bytes=budget, max_slots=1 << 20, max_batch=4096, max_k=1000,
                 n_streams=4)
    for rate in rates:
        n = int(rate * (seconds + warmup_s))
        q = make_queries(4, n_queries=n, vocab=corpus.vocab)
        arr = poisson_arrivals(rate, n, 4004 + int(rate)) * 1e6
        st0 = srv.stats()
        t0 = time.perf_counter()
        lat, queue, _, _, cnt = srv.replay(q.q_ids, q.q_offsets, q.k, arr, 1000,
                                           keep_results=False)
        wall = time.perf_counter() - t0
        st = srv.stats()
        w = arr >= warmup_s * 1e6
        ok = np.isfinite(lat) & w
        svc = lat - queue
        # requests of the measured window completed per second of that window's span
        span = (np.nanmax(arr[ok] + lat[ok]) - arr[w].min()) / 1e6 if ok.any() else float("nan")
        rec = dict(offered_qps=rate, n=n, window_s=seconds, warmup_s=warmup_s,
                   achieved_qps=float(ok.sum() / span),
                   p50_ms=float(np.percentile(lat[ok], 50) / 1e3),
                   p99_ms=float(np.percentile(lat[ok], 99) / 1e3),
                   queue_p50_ms=float(np.percentile(queue[ok], 50) / 1e3),
                   queue_p99_ms=float(np.percentile(queue[ok], 99) / 1e3),
                   service_p50_ms=float(np.percentile(svc[ok], 50) / 1e3),
                   service_p99_ms=float(np.percentile(svc[ok], 99) / 1e3),
                   errors=int(np.sum(cnt < 0)),
                   batches=st["batches"] - st0["batches"],
                   mean_batch=(st["completed"] - st0["completed"]) /
                   max(1, st["batches"] - st0["batches"]),
                   rejected_busy=st["rejected_busy"] - st0["rejected_busy"],
                   rejected_nomem=st["rejected_nomem"] - st0["rejected_nomem"],
                   mean_lanes_busy=(st["lane_busy_s"] - st0["lane_busy_s"]) / wall,
                   max_lanes_busy=st["max_lanes_busy"], wall_s=wall)
        out.append(rec)
        log("[serve]", rec)
    # parity window: 2000 requests at the lowest rate, result rows kept
    n = 2000
    q = make_queries(4, n_queries=n, vocab=corpus.vocab)
    arr = poisson_arrivals(rates[0], n, 4104) * 1e6
    lat, queue, ids, sc, cnt = srv.replay(q.q_ids, q.q_offsets, q.k, arr, 1000)
    srv.close()
    sample = _spread(0, n, n_check)
    check = dict(queries=[q.query(i).copy() for i in sample], k=q.k[sample].copy(),
                 rows=[ids[sample], sc[sample], cnt[sample]])
    return out, check


# ------------------------------------------------------------------------------------------
# CPU baseline leg: the FP64 oracle (test infrastructure) timed on the host and used to check
# sampled GPU rows of every timed configuration.

def _cpu_long_docs_oracle(variant: str, delta: float, queries: list, out_dir: str) -> dict:
    """Runs in a child process: the FP64 oracle rows of the sampled queries' tokens over the 5M
    long-document corpus, and per query B and sum |S| for every document, saved as .npy."""
    sys.path.insert(0, ROOT)
    from oracle import eager
    from tests.helpers import oracle_scores
    from workloads import CONFIGS, make_corpus
    cfg = CONFIGS[3]
    c = make_corpus(3)
    toks = np.unique(np.concatenate(queries))
    t0 = time.time()
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab, cfg["k1"], cfg["b"], delta,
                            variant, token_subset=toks)
    build_s = time.time() - t0
    del c
    files = []
    for j, q in enumerate(queries):
        b, a = oracle_scores(ref, q)
        fb = os.path.join(out_dir, f"{variant}_{j}_b.npy")
        fa = os.path.join(out_dir, f"{variant}_{j}_abs.npy")
        np.save(fb, b)
        np.save(fa, a)
        files.append((fb, fa))
    return dict(build_s=build_s, tokens=int(toks.size), files=files)


def cpu_background_start(long_queries: list):
    """Starts the 5M-document oracle jobs (one child process per variant) so that they run while
    the GPU legs do."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    tmp = tempfile.mkdtemp(prefix="bm25_oracle_")
    # at the lowest scheduling priority: the timed legs' host thread keeps its core
    ex = ProcessPoolExecutor(max_workers=2, mp_context=mp.get_context("spawn"),
                             initializer=os.nice, initargs=(19,))
    futs = {v: ex.submit(_cpu_long_docs_oracle, v, d, long_queries, tmp)
            for v, d in (("bm25plus", 1.0), ("bm25l", 0.5))}
    return ex, futs, tmp


def _parity_stats(errs: list, n_q: int, rtol: float, failures: list) -> dict:
    e = np.concatenate(errs) if errs else np.zeros(0)
    return dict(queries_checked=n_q, results_checked=int(e.size),
                max_rel_err=float(e.max(initial=0.0)),
                p99_rel_err=float(np.percentile(e, 99)) if e.size else 0.0, rtol=rtol,
                ok=not failures, failures=failures[:3])


def _check_rows(ref, queries, rows, ks, rtol, name, threads):
    """Checks sampled GPU rows against the oracle index `ref` in a thread pool."""
    from concurrent.futures import ThreadPoolExecutor

    from tests.helpers import check_query, oracle_scores
    ids, sc, cnt = rows
    ks = np.broadcast_to(np.asarray(ks), (len(queries),))

    def one(j):
        b, a = oracle_scores(ref, queries[j])
        try:
            return check_query(ids[j], sc[j], cnt[j], b, a, int(ks[j]), rtol, f"{name} {j}",
                               all_errors=True), None
        except AssertionError as e:
            return None, str(e)

    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(one, range(len(queries))))
    errs = [r for r, f in res if r is not None]
    fails = [f for _, f in res if f is not None]
    return _parity_stats(errs, len(queries), rtol, fails)


def cpu_baseline_leg(corpus, queries, time_idx, single_idx, checks, bg, threads) -> tuple:
    """The oracle (the paper's method in FP64) on the host cores: index rows of the sampled
    queries' tokens, then per query slice-and-sum plus the paper's partition-then-sort top-k,
    timed on a thread pool and on one thread; the oracle's own index build rate on a prefix of
    the corpus; and the parity of every sampled GPU row set in `checks`."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import eager
    from tests.helpers import RTOL, check_query
    from workloads import CONFIGS, make_corpus
    cfg = CONFIGS[2]
    k = int(cfg["k"])
    parity = {}
    # wait for the background oracle jobs first: the timing below needs idle host cores
    long_res = {}
    if bg is not None:
        ex, futs, tmp = bg
        for v, f in futs.items():
            try:
                long_res[v] = f.result()
            except Exception as e:  # reported, not fatal
                long_res[v] = dict(error=repr(e))
        ex.shutdown()
    # 8.8M-document rows for the timing sample and every 8.8M-document parity sample
    qs_time = [queries.query(i) for i in time_idx]
    all_q = list(qs_time)
    for name in ("cfg2_f16", "cfg4_serving"):
        if name in checks:
            all_q += list(checks[name]["queries"])
    subset = np.unique(np.concatenate(all_q))
    t0 = time.time()
    ref = eager.build_index(corpus.tokens, corpus.doc_offsets, corpus.vocab, cfg["k1"], cfg["b"],
                            cfg["delta"], cfg["variant"], token_subset=subset)
    log(f"[cpu] oracle rows for {subset.size} tokens over {corpus.n_docs} documents in "
        f"{time.time() - t0:.1f}s")

    def one(q):
        return eager.search_partitioned(ref, q, k)

    t0 = time.perf_counter()
    for i in single_idx:
        one(queries.query(i))
    single = len(single_idx) / (time.perf_counter() - t0)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(one, qs_time))
    multi = len(qs_time) / (time.perf_counter() - t0)
    # the oracle's index build on a prefix of the same corpus
    nb = min(corpus.n_docs, 1_000_000)
    te = int(corpus.doc_offsets[nb])
    t0 = time.perf_counter()
    bref = eager.build_index(corpus.tokens[:te], corpus.doc_offsets[:nb + 1], corpus.vocab,
                             cfg["k1"], cfg["b"], cfg["delta"], cfg["variant"])
    bt = time.perf_counter() - t0
    build = dict(nnz_per_s=bref.nnz / bt, docs=nb, tokens=te, nnz=bref.nnz, seconds=bt,
                 threads=1)
    del bref
    best = dict(value=multi, cores=threads) if multi > single else dict(value=single, cores=1)
    cpu = dict(value=best["value"], unit="queries/s", cores=best["cores"], kind="oracle",
               sample=(f"{len(qs_time)} queries of the benchmark stream over the full "
                       f"{corpus.n_docs}-document index, FP64 slice-and-sum of the query rows "
                       f"and the paper's partition-then-sort top-{k} ({threads}-thread pool: "
                       f"{multi:.2f} q/s); {len(single_idx)} of them on one thread: "
                       f"{single:.3f} q/s"),
               single_thread_qps=single, pool_qps=multi, pool_threads=threads,
               build=build, cpu_model=_cpu_model(), host_cpus=os.cpu_count(),
               affinity=len(os.sched_getaffinity(0)))
    log("[cpu]", cpu)

    # parity of the 8.8M-document configurations
    for name, rtol in (("cfg2_f16", RTOL["f16"]), ("cfg2_f32", RTOL["f32"]),
                       ("cfg4_serving", RTOL["f16"])):
        c = checks.get(name)
        if c is None:
            continue
        parity[name] = _check_rows(ref, c["queries"], c["rows"], c["k"], rtol, name, threads)
        log(f"[parity {name}]", parity[name])
    del ref
    # 1M documents, per-query form
    c = checks.get("cfg1_plain")
    if c is not None:
        cfg1 = CONFIGS[1]
        c1 = make_corpus(1)
        r1 = eager.build_index(c1.tokens, c1.doc_offsets, c1.vocab, cfg1["k1"], cfg1["b"],
                               cfg1["delta"], cfg1["variant"],
                               token_subset=np.unique(np.concatenate(c["queries"])))
        parity["cfg1_plain"] = _check_rows(r1, c["queries"], c["rows"], c["k"], RTOL["f32"],
                                           "cfg1_plain", threads)
        log("[parity cfg1_plain]", parity["cfg1_plain"])
        del r1, c1
    # 5M long documents (oracle computed in the background)
    for v in ("bm25plus", "bm25l"):
        c = checks.get(f"cfg3_{v}")
        if c is None:
            continue
        res = long_res.get(v, {})
        if "files" not in res:
            parity[f"cfg3_{v}"] = dict(ok=False, failures=[res.get("error", "not run")])
            continue
        errs, fails = [], []
        ids, sc, cnt = c["rows"]
        for j, (fb, fa) in enumerate(res["files"]):
            b = np.load(fb)
            a = np.load(fa)
            try:
                errs.append(check_query(ids[j], sc[j], cnt[j], b, a, c["k"], RTOL["bf16"],
                                        f"cfg3 {v} {j}", all_errors=True))
            except AssertionError as e:
                fails.append(str(e))
        parity[f"cfg3_{v}"] = _parity_stats(errs, len(res["files"]), RTOL["bf16"], fails)
        parity[f"cfg3_{v}"]["oracle_build_s"] = res["build_s"]
        log(f"[parity cfg3_{v}]", parity[f"cfg3_{v}"])
    # tokenization: the GPU's words of sampled documents against the oracle's split
    c = checks.get("tokenize")
    if c is not None:
        from oracle import tokenize as T
        fails, n_tok = [], 0
        for j, (doc, got) in enumerate(c["rows"]):
            want = T.split(doc, lowercase=True)
            n_tok += len(want)
            if got != want:
                fails.append(f"document sample {j}: {len(got)} words, oracle {len(want)}")
        parity["tokenize"] = dict(docs_checked=len(c["rows"]), tokens_checked=n_tok,
                                  ok=not fails, failures=fails[:3])
        log("[parity tokenize]", parity["tokenize"])
    if bg is not None:
        import shutil
        shutil.rmtree(bg[2], ignore_errors=True)
    return cpu, parity


# ------------------------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--n-docs", type=int, default=None, help="override corpus size (testing)")
    ap.add_argument("--cpu-sample", type=int, default=256)
    ap.add_argument("--cpu-single", type=int, default=32)
    ap.add_argument("--check", type=int, default=64, help="queries checked per configuration")
    ap.add_argument("--check-long", type=int, default=6, help="queries checked per 5M variant")
    ap.add_argument("--plain-queries", type=int, default=256)
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-warmup", type=float, default=1.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-tokenize", action="store_true")
    ap.add_argument("--tokenize-docs", type=int, default=500_000,
                    help="documents of the seeded text corpus the tokenization leg splits")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-long", action="store_true", help="skip the 5M long-document leg")
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP graph leg")
    ap.add_argument("--fixed-plan", action="store_true",
                    help="use the automatic launch shape instead of the autotuned one")
    ap.add_argument("--plan", default=None,
                    help="fixed launch shape q_tile,waves,doc_tile,doc_groups for the headline "
                         "batches (profiling: no autotuning pass)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the index would shard by document range)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2407_03618_amd import Index
    from workloads import CONFIGS, make_corpus, make_queries

    cfg = dict(CONFIGS[2])
    B = args.batch
    k = int(cfg["k"])
    t0 = time.time()
    corpus = make_corpus(2, n_docs=args.n_docs)
    n_queries = max(B * (args.steps + args.warmup), B)
    queries = make_queries(2, n_queries=min(n_queries, cfg["n_queries"]) if args.n_docs is None
                           else n_queries, vocab=corpus.vocab)
    log(f"[gen] {corpus.n_docs} docs, {corpus.n_tokens} tokens, {queries.n} queries "
        f"in {time.time() - t0:.1f}s")
    checks = {}
    bg = None
    long_queries = None
    dev = torch.device("cuda:0")
    tok_d = torch.from_numpy(corpus.tokens).to(dev)
    off_d = torch.from_numpy(corpus.doc_offsets).to(dev)
    torch.cuda.synchronize()

    # index build (untimed for the query metric; reported with its own roofline). The first
    # build also grows PyTorch's caching allocator, which the index's memory comes from; it is
    # reported as the cold build, and the builds after it reuse the cached memory.
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cold = Index(tok_d, off_d, corpus.vocab, cfg["k1"], cfg["b"], cfg["delta"], cfg["variant"],
                 "f16")
    torch.cuda.synchronize()
    cold_ms = (time.perf_counter() - t0) * 1e3
    cold.free()
    log(f"[build] cold f16 in {cold_ms:.1f} ms")
    builds = {}
    for dtype in ("f16", "f32"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        idx = Index(tok_d, off_d, corpus.vocab, cfg["k1"], cfg["b"], cfg["delta"], cfg["variant"],
                    dtype)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        builds[dtype] = (idx, ms)
        log(f"[build] {dtype}: nnz {idx.nnz} in {ms:.1f} ms ({idx.nnz / ms / 1e6:.2f} G nnz/s)")
    idx, build_ms = builds["f16"]
    idx32 = builds["f32"][0]
    del tok_d, off_d
    torch.cuda.empty_cache()
    df = idx.export()["df"].cpu().numpy()
    build_info = {dt: dict(build_roofline(corpus.n_tokens, corpus.n_docs, ix.nnz, corpus.vocab,
                                          2 if dt == "f16" else 4, ms), range=ix.range_stats())
                  for dt, (ix, ms) in builds.items()}
    build_info["f16_cold_ms"] = cold_ms
    # serving before the long-document oracle starts on the host: the scheduler thread and the
    # per-batch host steps are on every request's latency path
    serving = None
    if not args.no_serve:
        serving, checks["cfg4_serving"] = serving_leg(
            idx, corpus, CONFIGS[4]["rates"], args.serve_seconds, args.serve_warmup,
            budget=8 << 30, n_check=args.check)
        torch.cuda.empty_cache()
    if not args.no_long and not args.no_cpu:
        # the long-document oracle runs on the host while the GPU legs below run (after the
        # build timings, which include host steps)
        qs3 = make_queries(3, n_queries=512, vocab=CONFIGS[3]["vocab"])
        long_queries = [qs3.query(i).copy() for i in _spread(0, 512, args.check_long)]
        bg = cpu_background_start(long_queries)

    # one plain device copy of 1 GiB (1 GiB read, 1 GiB written): hardware byte counters taken
    # on this same command are scaled by what they read for it
    from paper_2407_03618_amd import bm25 as _bm25
    cal_src = torch.zeros(1 << 28, dtype=torch.int32, device=dev)
    cal_dst = torch.empty_like(cal_src)
    _bm25.copy_bytes(cal_dst, cal_src, 1 << 30)
    torch.cuda.synchronize()
    del cal_src, cal_dst

    q_dev = torch.from_numpy(queries.q_ids).to(dev)
    n_batches = queries.n // B
    out = idx._outputs(B, k)

    def batch(i):
        lo = (i % n_batches) * B
        off = queries.q_offsets[lo:lo + B + 1]
        base = int(off[0])
        return lo, q_dev[base:], off - base

    tuned = None
    if args.plan:
        qt, w, dt, g = (int(x) for x in args.plan.split(","))
        idx.set_plan(dict(q_tile=qt, waves=w, doc_tile=dt, doc_groups=g))
    elif not args.fixed_plan:
        # one autotuning pass for this shape class (batch size, longest query, list size) on the
        # first warm-up batch; later batches of the class run the tuned shape
        _, qd, off = batch(0)
        t0 = time.perf_counter()
        tuned = idx.autotune(qd, off, k, k)
        log(f"[tune] {tuned} in {time.perf_counter() - t0:.1f}s")
    max_qlen = int(np.diff(queries.q_offsets).max())
    plan = idx.get_plan(B, max_qlen, k)
    log("[plan]", plan)

    for i in range(args.warmup):
        _, qd, off = batch(i)
        idx.search_batch(qd, off, k, k, out=out)
    torch.cuda.synchronize()
    idx.kernel_time_read()
    idx.kernel_timing(True)
    t0 = time.perf_counter()
    for s in range(args.steps):
        lo, qd, off = batch(args.warmup + s)
        idx.search_batch(qd, off, k, k, out=out)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern_ms, launches = idx.kernel_time_read()
    idx.kernel_timing(False)
    qps = args.steps * B / elapsed
    ms_step = elapsed / args.steps * 1e3
    gather_ms = kern_ms / max(launches, 1)
    # work of the timed launches (averaged over them)
    alg, works = 0, []
    for s in range(args.steps):
        lo = ((args.warmup + s) % n_batches) * B
        q_off = queries.q_offsets[lo:lo + B + 1]
        alg += int(algorithmic_bytes(df, queries.q_ids, q_off, np.full(B, k), 2).sum())
        if s < 4:
            ids_b = queries.q_ids[q_off[0]:q_off[-1]]
            works.append(launch_work(df, ids_b, q_off - q_off[0], k, corpus.n_docs, 2))
    work = {key: float(np.mean([w[key] for w in works])) for key in works[0]}
    traffic = measured_traffic("batched_f16_top100", plan)
    roof = roofline(work, gather_ms, traffic, alg / args.steps)
    log(f"[batched f16] {qps:.0f} q/s, {ms_step:.2f} ms/step, gather kernel {gather_ms:.2f} ms, "
        f"bound {roof['binding']} frac {roof['frac']:.3f}")

    # rows of the last timed batch for the parity sample
    last_lo = ((args.warmup + args.steps - 1) % n_batches) * B
    sample = _spread(0, B, args.check)
    ids_h, sc_h, cnt_h = (t.cpu().numpy() for t in out)
    checks["cfg2_f16"] = dict(queries=[queries.query(last_lo + i).copy() for i in sample],
                              rows=[ids_h[sample], sc_h[sample], cnt_h[sample]], k=k)

    extra = {}
    if serving is not None:
        extra["serving"] = serving
    if not args.no_graph:
        extra["graph_mode"] = graph_leg(idx, q_dev, queries, k, 0, B)
        log("[graph]", extra["graph_mode"])
    # batched FP32 on the same batches: precision comparison and its own parity sample
    if args.plan:
        idx32.set_plan(idx.get_plan(B, max_qlen, k))
    elif tuned is not None:
        _, qd2, off2 = batch(0)
        idx32.autotune(qd2, off2, k, k)
    o32 = idx32._outputs(B, k)
    _, qd2, off2 = batch(args.warmup)
    idx32.search_batch(qd2, off2, k, k, out=o32)  # warm-up
    torch.cuda.synchronize()
    reps = max(2, args.steps // 4)
    t0 = time.perf_counter()
    for s in range(reps):
        _, qd2, off2 = batch(args.warmup + s)
        idx32.search_batch(qd2, off2, k, k, out=o32)
    torch.cuda.synchronize()
    extra["batched_fp32"] = dict(qps=reps * B / (time.perf_counter() - t0),
                                 plan=idx32.get_plan(B, max_qlen, k))
    log("[batched f32]", extra["batched_fp32"])
    _, qd2, off2 = batch(args.warmup + args.steps - 1)
    idx32.search_batch(qd2, off2, k, k, out=o32)
    torch.cuda.synchronize()
    i32, s32, c32 = (t.cpu().numpy() for t in o32)
    checks["cfg2_f32"] = dict(queries=checks["cfg2_f16"]["queries"],
                              rows=[i32[sample], s32[sample], c32[sample]], k=k)
    del o32
    # plain per-query FP32 form on the same index recipe
    if not args.no_plain:
        nq = args.plain_queries
        lo = last_lo
        off = queries.q_offsets[lo:lo + nq + 1]
        base = int(off[0])
        qd = q_dev[base:]
        o2 = idx32._outputs(nq, k)
        idx32.search_plain(qd, off - base, k, k, out=o2)  # warm-up
        torch.cuda.synchronize()
        # throughput without per-launch timing events, then a second run for the kernel time
        t0 = time.perf_counter()
        idx32.search_plain(qd, off - base, k, k, out=o2)
        torch.cuda.synchronize()
        pt = time.perf_counter() - t0
        idx32.kernel_time_read()
        idx32.kernel_timing(True)
        idx32.search_plain(qd, off - base, k, k, out=o2)
        torch.cuda.synchronize()
        pk_ms, pl = idx32.kernel_time_read()
        idx32.kernel_timing(False)
        palg = int(algorithmic_bytes(df, queries.q_ids, off, np.full(nq, k), 4).sum())
        extra["plain_fp32"] = dict(
            qps=nq / pt, ms_per_query=pt / nq * 1e3, sweep_kernel_ms=pk_ms / max(pl, 1),
            no_reuse_GBs=palg / (pk_ms / 1e3) / 1e9 if pk_ms > 0 else None,
            no_reuse_frac=palg / (pk_ms / 1e3) / 1e9 / HBM_PEAK_GBS if pk_ms > 0 else None,
            queries=nq)
        log("[plain f32]", extra["plain_fp32"])
        extra["plain_1M_fp32"], checks["cfg1_plain"] = plain_1m_leg(nq, args.check)
        log("[plain 1M f32]", extra["plain_1M_fp32"])
    idx32.free()  # make room for the 5M-document indexes
    torch.cuda.empty_cache()

    if not args.no_tokenize:
        extra["tokenize"], checks["tokenize"] = tokenize_leg(args.tokenize_docs, args.check)
        log("[tokenize]", extra["tokenize"])
        torch.cuda.empty_cache()

    if not args.no_long:
        legs, lchecks, lq = long_docs_leg(args.check_long)
        extra["long_docs_top1000_bf16"] = legs
        for v, c in lchecks.items():
            c["queries"] = lq
            checks[f"cfg3_{v}"] = c

    cpu, parity = None, None
    if not args.no_cpu:
        threads = min(16, len(os.sched_getaffinity(0)))
        time_idx = list(range(last_lo, last_lo + min(args.cpu_sample, B)))
        cpu, parity = cpu_baseline_leg(corpus, queries, time_idx, time_idx[:args.cpu_single],
                                       checks, bg, threads)
    res = {
        "metric": METRIC,
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16",
        "data": "synthetic",
        "config": {
            "workload": (f"{corpus.n_docs}-doc Zipf(1.05) corpus, V={corpus.vocab}, "
                         f"{B}-query batches, top-{k}, FP16 stored scores, FP32 accumulation, "
                         "batched form"),
            "n_docs": corpus.n_docs, "vocab": corpus.vocab, "n_tokens": corpus.n_tokens,
            "nnz": idx.nnz, "batch": B, "k": k, "plan": plan,
            "plan_source": ("fixed" if args.plan else
                            "autotuned" if tuned is not None else "automatic"),
        },
        "roofline": roof,
        "launch_work": work,
        "cpu_baseline": cpu,
        "parity": parity,
        "build": build_info,
        **extra,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
