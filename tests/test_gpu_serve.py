"""GPU: concurrent query contexts and the continuous-batching serving loop.

Each request's result in the mix must equal the same request run alone (tolerance 0) on the
index state defined by its sequence number; the alone replay runs on a second index, and the
labels at the end are compared with the oracle.
"""
import threading

import numpy as np
import pytest
import torch

import dblgen
import oracle

pytestmark = pytest.mark.gpu

dbl = pytest.importorskip("paper_2101_09441_amd")
from paper_2101_09441_amd.serve import Request, serve  # noqa: E402


def dev(a):
    return dbl.to_device_ids(a)


@pytest.fixture(scope="module")
def tiny():
    return dblgen.tiny_workload(1)


def test_query_contexts_run_concurrently(tiny):
    w = tiny
    g = dbl.Index.build(w.n, dev(w.src), dev(w.dst))
    want = g.query(dev(w.q_u), dev(w.q_v)).cpu().numpy()
    ctxs = [g.query_context(bfs_slots=64) for _ in range(3)]
    results = [None] * 3
    parts = np.array_split(np.arange(len(w.q_u)), 3)

    def run(i):
        s = torch.cuda.Stream()
        u, v = dev(w.q_u[parts[i]]), dev(w.q_v[parts[i]])
        for _ in range(5):
            out = ctxs[i].query(u, v, stream=s)
        s.synchronize()
        results[i] = out.cpu().numpy()

    th = [threading.Thread(target=run, args=(i,)) for i in range(3)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for i in range(3):
        assert np.array_equal(results[i], want[parts[i]])
    st = g.stats()
    assert st["queries"] == len(w.q_u) * 6  # default context once + three contexts five times
    for c in ctxs:
        c.close()
    assert g.stats()["queries"] == len(w.q_u) * 6
    with pytest.raises(dbl.DblError):
        g.query_context(bfs_slots=4).query(dev([0]), dev([w.n]))


def _trace(w, n, rate, seed, q_size=(1, 3000), i_size=(10, 200)):
    spec = dblgen.serving_trace(w.q_u, w.q_v, w.ins_src, w.ins_dst, n, rate, q_size=q_size,
                                i_size=i_size, seed=seed)
    return [Request(s, k, a, b, t) for s, k, a, b, t in spec]


@pytest.mark.parametrize("realtime,rate", [(True, 3000.0), (False, 1.0)])
def test_serving_results_equal_alone(tiny, realtime, rate):
    w = tiny
    trace = _trace(w, 160, rate, seed=11)
    g = dbl.Index.build(w.n, dev(w.src), dev(w.dst))
    summ = serve(g, trace, workers=4, max_batch=4096, bfs_slots=64, realtime=realtime)
    assert summ["query"]["requests"] + summ["insert"]["requests"] == len(trace)
    _check_against_alone_and_oracle(w, g, trace)
    if not realtime:
        assert summ["device_batches"] < len(trace)  # the backlog was coalesced


def _check_against_alone_and_oracle(w, g, trace):
    """Every answer of the mix equals the same request run alone on a fresh index in sequence
    order, and the oracle's Algorithm 2 on the state its sequence number defines; the final
    labels equal both."""
    a = dbl.Index.build(w.n, dev(w.src), dev(w.dst))
    o = oracle.OracleIndex(w.n, w.src, w.dst).build(threads=8)
    for r in sorted(trace, key=lambda r: r.seq):
        if r.kind == "query":
            alone = a.query(dev(r.a), dev(r.b)).cpu().numpy()
            assert np.array_equal(r.answers, alone), f"request {r.seq} vs alone"
            assert np.array_equal(r.answers, o.query_dbl(r.a, r.b, threads=8)), \
                f"request {r.seq} vs oracle"
        else:
            a.insert_edges(dev(r.a), dev(r.b))
            o.insert(r.a, r.b)
    for x, y, z in zip(g.labels_numpy(), a.labels_numpy(), o.labels()):
        assert np.array_equal(x, y) and np.array_equal(x, z)


def test_serving_memory_budget_defers_batches(tiny):
    """A budget with room for the workers' fixed scratch and one full batch in flight: a
    backlog of query batches is admitted one batch at a time (the rest wait), and every answer
    still equals the oracle's on its sequence state."""
    from paper_2101_09441_amd.serve import GpuExecutor
    w = tiny
    trace = _trace(w, 120, 1.0, seed=21, q_size=(500, 3000))
    g = dbl.Index.build(w.n, dev(w.src), dev(w.dst))
    max_batch = 4096
    fixed = g.query_context_bytes(64, 0, max_batch)
    cap = 3 * fixed + GpuExecutor.footprint(max_batch) + GpuExecutor.footprint(max_batch) // 2
    summ = serve(g, trace, workers=4, max_batch=max_batch, bfs_slots=64, realtime=False,
                 memory_cap=cap)
    assert summ["workers"] == 3
    assert summ["admission_waits"] > 0
    assert 0 < summ["peak_inflight_batch_bytes"] <= summ["batch_budget_bytes"]
    _check_against_alone_and_oracle(w, g, trace)


def test_serving_memory_cap_refuses(tiny):
    w = tiny
    g = dbl.Index.build(w.n, dev(w.src), dev(w.dst))
    with pytest.raises(MemoryError):
        serve(g, _trace(w, 5, 100.0, seed=1), memory_cap=1 << 10)
