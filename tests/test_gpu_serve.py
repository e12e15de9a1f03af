"""Continuous-batching server: results alone and in a mix agree (within the FP16 tolerance) and
match the oracle; admission errors; open-loop replay."""
import numpy as np
import pytest

from oracle import eager
from tests.helpers import RTOL, check_query, oracle_scores
from workloads import make_corpus, make_queries

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def setup():
    from paper_2407_03618_amd import Index
    c = make_corpus(4, n_docs=50_000)
    q = make_queries(4, n_queries=48, vocab=c.vocab)
    idx = Index(_dev(c.tokens), _dev(c.doc_offsets), c.vocab, 1.5, 0.75, 0.0, "lucene", "f16")
    ref = eager.build_index(c.tokens, c.doc_offsets, c.vocab, token_subset=np.unique(q.q_ids))
    return c, q, idx, ref


def _collect(server, n, k_stride):
    out = {}
    while len(out) < n:
        for t, cnt, ids, sc in server.poll(64, 2_000_000, k_stride):
            out[t] = (cnt, ids.copy(), sc.copy())
    return out


@pytest.mark.parametrize("graphs", [False, True])
def test_alone_and_in_mix_agree(setup, graphs):
    """Each request alone and in a mix of micro-batches; with graphs, every micro-batch is one
    HIP graph launch on its lane's stream."""
    c, q, idx, ref = setup
    idx.set_graphs(graphs)
    try:
        _alone_and_in_mix(c, q, idx, ref)
    finally:
        idx.set_graphs(False)


def _alone_and_in_mix(c, q, idx, ref):
    from paper_2407_03618_amd import Server
    srv = Server(idx, hbm_budget_bytes=1 << 30, max_slots=4096, max_batch=16, max_k=1000,
                 n_streams=2)
    alone = []
    for i in range(q.n):
        t = srv.submit(q.query(i), int(q.k[i]))
        r = _collect(srv, 1, 1000)
        alone.append(r[t])
    tickets = [srv.submit(q.query(i), int(q.k[i])) for i in range(q.n)]
    mix = _collect(srv, q.n, 1000)
    st = srv.stats()
    assert st["batches"] >= q.n + 2, st  # the mix ran as several micro-batches
    assert st["max_batch_seen"] > 1, st
    assert st["completed"] == 2 * q.n and st["rejected_busy"] == 0, st
    for i, t in enumerate(tickets):
        k = int(q.k[i])
        cnt_a, ids_a, sc_a = alone[i]
        cnt_m, ids_m, sc_m = mix[t]
        assert cnt_a == cnt_m
        b, absS = oracle_scores(ref, q.query(i))
        for cnt, ids, sc in ((cnt_a, ids_a, sc_a), (cnt_m, ids_m, sc_m)):
            check_query(ids, sc, cnt, b, absS, k, RTOL["f16"], f"serve query {i}")
        # same documents scored the same, within the storage tolerance
        common = np.intersect1d(ids_a[:cnt_a], ids_m[:cnt_m])
        pa = {d: s for d, s in zip(ids_a[:cnt_a], sc_a[:cnt_a])}
        pm = {d: s for d, s in zip(ids_m[:cnt_m], sc_m[:cnt_m])}
        for d in common:
            assert abs(pa[d] - pm[d]) <= RTOL["f16"] * absS[d] + 1e-30
    srv.close()


def test_admission_errors(setup):
    from paper_2407_03618_amd import BM25Error, Server
    c, q, idx, ref = setup
    srv = Server(idx, hbm_budget_bytes=1 << 28, max_slots=2, max_batch=4, max_k=100, n_streams=1)
    with pytest.raises(BM25Error) as e:
        srv.submit([1, c.vocab], 10)
    assert e.value.code == -2
    with pytest.raises(BM25Error) as e:
        srv.submit([1, 2], 101)
    assert e.value.code == -1
    srv.close()
    # a budget that cannot hold one request of the longest query is refused at create
    with pytest.raises(BM25Error) as e:
        Server(idx, hbm_budget_bytes=1000, max_slots=8, max_batch=4, max_k=100, n_streams=1)
    assert e.value.code == -3


def test_replay_open_loop(setup):
    from paper_2407_03618_amd import Server
    c, q, idx, ref = setup
    srv = Server(idx, hbm_budget_bytes=1 << 30, max_slots=4096, max_batch=32, max_k=1000,
                 n_streams=2)
    arrivals = np.cumsum(np.full(q.n, 200.0))  # 5k requests/s
    lat, queue, ids, sc, cnt = srv.replay(q.q_ids, q.q_offsets, q.k, arrivals, 1000)
    assert np.all(np.isfinite(lat)) and np.all(lat > 0)
    assert np.all(np.isfinite(queue)) and np.all(queue >= 0) and np.all(queue <= lat)
    for i in range(q.n):
        b, absS = oracle_scores(ref, q.query(i))
        check_query(ids[i], sc[i], cnt[i], b, absS, int(q.k[i]), RTOL["f16"], f"replay {i}")
    srv.close()


def test_budget_reserved_at_create_and_held(setup):
    """The server takes its whole budget from the index's allocator (PyTorch's caching
    allocator) at create; a run of mixed k and lengths allocates nothing more, and close returns
    it."""
    import torch
    from paper_2407_03618_amd import Server
    c, q, idx, ref = setup
    import gc
    gc.collect()  # earlier tests' cyclic garbage must not be freed inside the measured span
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    idx_before = idx.device_bytes()
    budget = 256 << 20
    srv = Server(idx, hbm_budget_bytes=budget, max_slots=4096, max_batch=64, max_k=1000,
                 n_streams=2)
    held = torch.cuda.memory_allocated() - before
    assert budget - 1024 <= held <= budget + 4096, held
    arrivals = np.cumsum(np.full(q.n, 50.0))
    lat, queue, _, _, cnt = srv.replay(q.q_ids, q.q_offsets, q.k, arrivals, 1000,
                                       keep_results=False)
    assert np.all(cnt == np.minimum(q.k, c.n_docs))
    assert torch.cuda.memory_allocated() - before == held
    assert idx.device_bytes() == idx_before  # lanes do not grow the index's scratch
    st = srv.stats()
    assert st["completed"] == q.n and st["max_lanes_busy"] >= 1 and st["lane_busy_s"] > 0, st
    srv.close()
    assert torch.cuda.memory_allocated() == before
