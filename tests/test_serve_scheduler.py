"""Host logic of the serving loop, on the CPU: sequence order, coalescing, admission.

The executor here is a test double backed by the oracle: it answers query batches after a delay
on a thread of its own and applies insertions, recording when each device batch ran, so the test
can check that no query batch overlaps an insertion and that every answer equals the answer of
the request run alone on the state its sequence number defines.
"""
import threading
import time

import numpy as np

import dblgen
import oracle
from paper_2101_09441_amd.serve import Executor, Request, Scheduler, latency_summary


class OracleExecutor(Executor):
    def __init__(self, o, workers=3, delay=0.002, admit_after=0):
        self.o = o
        self.workers = workers
        self.delay = delay
        self.lock = threading.Lock()
        self.log = []  # (kind, t_start, t_end, seqs)
        self.admit_calls = 0
        self.admit_after = admit_after

    def admit(self, pairs):
        self.admit_calls += 1
        return self.admit_calls > self.admit_after

    def _q(self, w, reqs, on_done):
        t0 = time.perf_counter()
        u = np.concatenate([r.a for r in reqs])
        v = np.concatenate([r.b for r in reqs])
        time.sleep(self.delay)
        with self.lock:  # the oracle is not thread safe
            ans = self.o.query_dbl(u, v)
        off = 0
        for r in reqs:
            r.answers = ans[off:off + r.size]
            off += r.size
        self.log.append(("query", t0, time.perf_counter(), [r.seq for r in reqs]))
        on_done(w, reqs)

    def query_async(self, worker, reqs, on_done):
        threading.Thread(target=self._q, args=(worker, reqs, on_done), daemon=True).start()

    def insert(self, reqs):
        t0 = time.perf_counter()
        with self.lock:
            for r in reqs:
                self.o.insert(r.a, r.b)
        self.log.append(("insert", t0, time.perf_counter(), [r.seq for r in reqs]))


def _trace(w, n=120, rate=4000.0, seed=3):
    spec = dblgen.serving_trace(w.q_u, w.q_v, w.ins_src, w.ins_dst, n, rate, q_size=(1, 300),
                                i_size=(5, 40), seed=seed)
    return [Request(s, k, a, b, t) for s, k, a, b, t in spec]


def _alone(w, trace):
    o = oracle.OracleIndex(w.n, w.src, w.dst).build()
    out = {}
    for r in sorted(trace, key=lambda r: r.seq):
        if r.kind == "query":
            out[r.seq] = o.query_dbl(r.a, r.b)
        else:
            o.insert(r.a, r.b)
    return out, o.labels()


def _check(w, trace, ex):
    alone, labels = _alone(w, trace)
    for r in trace:
        if r.kind == "query":
            assert np.array_equal(r.answers, alone[r.seq]), r.seq
        assert r.done is not None and r.done >= r.start
    for a, b in zip(ex.o.labels(), labels):
        assert np.array_equal(a, b)
    # no query batch overlaps an insertion
    ins = [(a, b) for k, a, b, _ in ex.log if k == "insert"]
    for k, a, b, _ in ex.log:
        if k == "query":
            for c, d in ins:
                assert b <= c or a >= d


def test_realtime_trace_matches_requests_run_alone():
    w = dblgen.tiny_workload(1)
    trace = _trace(w)
    ex = OracleExecutor(oracle.OracleIndex(w.n, w.src, w.dst).build())
    span = Scheduler(ex, max_batch=1000).run(trace, realtime=True)
    _check(w, trace, ex)
    s = latency_summary(trace, span)
    assert s["query"]["requests"] + s["insert"]["requests"] == len(trace)
    # times are relative to the start of the trace: nothing finishes before it arrives or
    # after the makespan
    for r in trace:
        assert r.arrival <= r.start + 1e-9 and r.start <= r.done <= span + 1e-6


def test_backlog_is_coalesced_and_overlaps():
    """Everything arrives at once: queries between insertions merge into few device batches and
    several batches are in flight together."""
    w = dblgen.tiny_workload(1)
    trace = _trace(w, n=200, seed=5)
    ex = OracleExecutor(oracle.OracleIndex(w.n, w.src, w.dst).build(), workers=4, delay=0.01)
    sch = Scheduler(ex, max_batch=400)
    sch.run(trace, realtime=False)
    _check(w, trace, ex)
    nq = sum(r.kind == "query" for r in trace)
    qbatches = {r.batch_id for r in trace if r.kind == "query"}
    assert len(qbatches) < nq  # coalesced
    qs = sorted((a, b) for k, a, b, _ in ex.log if k == "query")
    assert any(qs[i + 1][0] < qs[i][1] for i in range(len(qs) - 1))  # overlapping batches


def test_admission_refusals_delay_but_do_not_reorder():
    w = dblgen.tiny_workload(1)
    trace = _trace(w, n=60, seed=9)
    ex = OracleExecutor(oracle.OracleIndex(w.n, w.src, w.dst).build(), admit_after=25)
    sch = Scheduler(ex, max_batch=500)
    sch.run(trace, realtime=False)
    assert sch.refusals >= 25
    _check(w, trace, ex)


class BudgetExecutor(OracleExecutor):
    """Admits a batch while the pairs in flight, the new batch's included, fit a budget."""

    def __init__(self, o, budget, **kw):
        super().__init__(o, **kw)
        self.budget = budget
        self.inflight = 0
        self.peak = 0

    def admit(self, pairs):
        if pairs > self.budget:
            raise MemoryError("batch larger than the budget")
        with self.lock:
            return self.inflight + pairs <= self.budget

    def query_async(self, worker, reqs, on_done):
        k = sum(r.size for r in reqs)
        with self.lock:
            self.inflight += k
            self.peak = max(self.peak, self.inflight)

        def done(w, rs, err=None):
            with self.lock:
                self.inflight -= k
            on_done(w, rs, err) if err else on_done(w, rs)

        super().query_async(worker, reqs, done)


def test_memory_budget_limits_batches_in_flight():
    """Batches are cut and deferred so that the pairs in flight never exceed the budget; the
    answers still equal the requests run alone."""
    w = dblgen.tiny_workload(1)
    trace = _trace(w, n=120, seed=13)
    budget = 450
    ex = BudgetExecutor(oracle.OracleIndex(w.n, w.src, w.dst).build(), budget, workers=4,
                        delay=0.005)
    sch = Scheduler(ex, max_batch=400)
    sch.run(trace, realtime=False)
    _check(w, trace, ex)
    assert 0 < ex.peak <= budget
    assert sch.refusals > 0
