"""Serving form: a request loop with continuous batching over one resident index.

Requests (query batches and insertion batches) arrive over time, each with a sequence number.
The scheduler keeps the result of every request equal to running it alone on the index state
defined by its sequence number:

* a query request observes exactly the insertions that precede it, so queries are never in
  flight while an insertion runs, and an insertion waits until every earlier query finished;
* query requests between two insertions are read-only and run concurrently: whenever a worker
  (a query context with its own stream) is free, the queued query requests at the head of the
  line are coalesced into one device batch, as large as the memory budget admits next to the
  batches already in flight, and handed to it;
* consecutive insertion requests are coalesced into one insertion batch (a batch is a set, so
  this equals applying them one after another).

Latency is measured from a request's arrival to its result being on the host.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np


@dataclass
class Request:
    seq: int
    kind: str                 # "query" or "insert"
    a: np.ndarray             # query sources / edge tails (uint32)
    b: np.ndarray             # query targets / edge heads (uint32)
    arrival: float = 0.0      # seconds after the start of the trace
    start: Optional[float] = None
    done: Optional[float] = None
    answers: Optional[np.ndarray] = None
    batch_id: int = -1

    @property
    def size(self) -> int:
        return len(self.a)


class Executor:
    """What the scheduler needs from the device side (the GPU executor below, or a test fake)."""

    workers: int

    def query_async(self, worker: int, reqs: List[Request], on_done: Callable) -> None:
        raise NotImplementedError

    def insert(self, reqs: List[Request]) -> None:
        raise NotImplementedError

    def admit(self, pairs: int) -> bool:
        """Whether a device batch of `pairs` pairs may start now, next to the batches in
        flight. Raises MemoryError if it could not start even with nothing else in flight."""
        return True

    def close(self) -> None:
        pass


class Scheduler:
    """Sequence-ordered dispatch with query coalescing and concurrent query workers."""

    def __init__(self, executor: Executor, max_batch: int = 1 << 17,
                 clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.max_batch = max_batch
        self.clock = clock
        self.cv = threading.Condition()
        self.free = list(range(executor.workers))
        self.inflight = 0
        self.batches = 0
        self.errors: List[BaseException] = []
        self.refusals = 0
        self.t0 = 0.0

    def _finished(self, worker: int, reqs: List[Request], err: Optional[BaseException] = None):
        t = self.clock() - self.t0
        with self.cv:
            for r in reqs:
                r.done = t
            if err is not None:
                self.errors.append(err)
            self.free.append(worker)
            self.inflight -= 1
            self.cv.notify_all()

    def run(self, trace: List[Request], realtime: bool = True) -> float:
        """Serve every request of `trace` (ordered by seq); returns the makespan in seconds."""
        pending = deque(sorted(trace, key=lambda r: r.seq))
        t0 = self.t0 = self.clock()
        offset = (lambda r: r.arrival) if realtime else (lambda r: 0.0)
        while True:
            with self.cv:
                if self.errors:
                    raise self.errors[0]
                if not pending and self.inflight == 0:
                    break
                now = self.clock() - t0
                head = pending[0] if pending else None
                wait_for = None
                if head is None:
                    self.cv.wait()
                    continue
                if offset(head) > now:
                    wait_for = offset(head) - now
                elif head.kind == "query":
                    if not self.free:
                        self.cv.wait()
                        continue
                    # coalesce the ready queries at the head of the line, up to max_batch pairs
                    # and as far as memory admits the batch next to those in flight
                    take, total = 0, 0
                    for r in pending:
                        if r.kind != "query" or offset(r) > now:
                            break
                        if take and total + r.size > self.max_batch:
                            break
                        if not self.ex.admit(total + r.size):
                            break
                        take += 1
                        total += r.size
                    if take == 0:
                        self.refusals += 1
                        if self.inflight:
                            self.cv.wait()
                        else:
                            self.cv.wait(0.001)
                        continue
                    batch = [pending.popleft() for _ in range(take)]
                    worker = self.free.pop()
                    self.inflight += 1
                    tb = self.clock() - t0
                    for r in batch:
                        r.start = tb
                        r.batch_id = self.batches
                    self.batches += 1
                else:
                    if self.inflight:
                        self.cv.wait()  # earlier queries must finish before the index changes
                        continue
                    batch = []
                    while pending and pending[0].kind == "insert" and offset(pending[0]) <= now:
                        batch.append(pending.popleft())
                    worker = None
                    tb = self.clock() - t0
                    for r in batch:
                        r.start = tb
                        r.batch_id = self.batches
                    self.batches += 1
            if wait_for is not None:
                with self.cv:
                    self.cv.wait(min(wait_for, 0.05))
                continue
            if worker is not None:
                self.ex.query_async(worker, batch, self._finished)
            else:
                self.ex.insert(batch)
                t = self.clock() - t0
                for r in batch:
                    r.done = t
        return self.clock() - t0


# Device bytes of one query batch in flight, per pair: the staged pairs (4 + 4 B) and their
# answer bytes (1 B), allocated for the batch and released when it completes.
BATCH_BYTES_PER_PAIR = 9


class GpuExecutor(Executor):
    """Query workers (a query context, a stream, pinned host staging and a host thread each)
    and an insertion path, over one resident index.

    Device memory is budgeted: the budget is `memory_cap` (or the free device memory less
    `reserve`). Each worker's context is a fixed part (visited bitmaps, queues and counters,
    and its undecided-pair list sized for max_batch); each batch in flight adds its staged
    pairs and answers. A batch is admitted only while the fixed parts plus every batch in flight
    plus the new one fit the budget; otherwise it waits for a batch to finish."""

    def __init__(self, index, workers: int = 4, max_batch: int = 1 << 17, bfs_slots: int = 256,
                 memory_cap: Optional[int] = None, reserve: int = 256 << 20):
        import torch

        from .binding import to_device_ids  # noqa: F401  (keeps the binding loaded)

        self.torch = torch
        self.index = index
        self.max_batch = max_batch
        dev = index.device
        fixed = index.query_context_bytes(bfs_slots, 0, max_batch)
        free, _ = torch.cuda.mem_get_info(dev)
        budget = free - reserve if memory_cap is None else min(memory_cap, free - reserve)
        # at least one worker and one batch of max_batch pairs must fit
        fit = max(0, (budget - self.footprint(max_batch)) // fixed) if budget > 0 else 0
        if fit < 1:
            raise MemoryError(f"device memory admits no query worker ({fixed} bytes each plus "
                              f"{self.footprint(max_batch)} for a batch; {budget} available)")
        self.workers = int(min(workers, fit))
        self.memory_cap = memory_cap
        self.reserve = reserve
        self.batch_budget = budget - self.workers * fixed
        self.inflight_bytes = 0
        self.peak_inflight_bytes = 0
        self.mem_lock = threading.Lock()
        self.ctx, self.streams, self.hbuf = [], [], []
        for _ in range(self.workers):
            self.ctx.append(index.query_context(bfs_slots=bfs_slots))
            self.streams.append(torch.cuda.Stream(device=dev))
            self.hbuf.append((torch.empty(max_batch, dtype=torch.int32).pin_memory(),
                              torch.empty(max_batch, dtype=torch.int32).pin_memory(),
                              torch.empty(max_batch, dtype=torch.uint8).pin_memory()))
        self.istream = torch.cuda.Stream(device=dev)
        self.icap = 0
        self.ibuf = None
        self._grow_insert_buffers(1 << 14)
        # the first batch on each worker stream would otherwise wait for the allocator to take
        # device memory from the driver: take one batch's worth per stream now (released to
        # the allocator's cache of that stream, where the batches find it)
        for s in self.streams:
            with torch.cuda.stream(s):
                tmp = [torch.empty(max_batch, dtype=dt, device=dev)
                       for dt in (torch.int32, torch.int32, torch.uint8)]
            s.synchronize()
            del tmp
        # one long-lived host thread per worker, fed through its own job queue
        import queue
        self.jobs = [queue.Queue() for _ in range(self.workers)]
        self.threads = [threading.Thread(target=self._loop, args=(w,), daemon=True)
                        for w in range(self.workers)]
        for t in self.threads:
            t.start()

    def _loop(self, w: int):
        while True:
            job = self.jobs[w].get()
            if job is None:
                return
            self._run_query(w, *job)

    @staticmethod
    def footprint(pairs: int) -> int:
        """Device bytes a batch of `pairs` pairs holds while in flight."""
        return pairs * BATCH_BYTES_PER_PAIR

    def admit(self, pairs: int) -> bool:
        need = self.footprint(pairs)
        if need > self.batch_budget:
            raise MemoryError(f"a query batch of {pairs} pairs needs {need} bytes; the memory "
                              f"budget leaves {self.batch_budget} for batches")
        with self.mem_lock:
            return self.inflight_bytes + need <= self.batch_budget

    def _run_query(self, w: int, reqs: List[Request], on_done):
        torch = self.torch
        total = sum(r.size for r in reqs)
        try:
            hu, hv, ho = self.hbuf[w]
            nu, nv = hu.numpy().view(np.uint32), hv.numpy().view(np.uint32)
            off = 0
            for r in reqs:
                nu[off:off + r.size] = r.a
                nv[off:off + r.size] = r.b
                off += r.size
            s = self.streams[w]
            with torch.cuda.stream(s):
                # the batch's device staging, admitted against the budget by the scheduler
                du = torch.empty(off, dtype=torch.int32, device=self.index.device)
                dv = torch.empty(off, dtype=torch.int32, device=self.index.device)
                do = torch.empty(off, dtype=torch.uint8, device=self.index.device)
                du.copy_(hu[:off], non_blocking=True)
                dv.copy_(hv[:off], non_blocking=True)
                self.ctx[w].query(du, dv, out=do, stream=s)
                ho[:off].copy_(do, non_blocking=True)
            s.synchronize()
            del du, dv, do
            no = ho.numpy()
            off = 0
            for r in reqs:
                r.answers = no[off:off + r.size].copy()
                off += r.size
            self._release(total)
            on_done(w, reqs)
        except BaseException as e:  # reported by the scheduler
            self._release(total)
            on_done(w, reqs, e)

    def _release(self, pairs: int) -> None:
        with self.mem_lock:
            self.inflight_bytes -= self.footprint(pairs)

    def query_async(self, worker: int, reqs: List[Request], on_done) -> None:
        with self.mem_lock:
            self.inflight_bytes += self.footprint(sum(r.size for r in reqs))
            self.peak_inflight_bytes = max(self.peak_inflight_bytes, self.inflight_bytes)
        self.jobs[worker].put((reqs, on_done))

    def insert(self, reqs: List[Request]) -> None:
        torch = self.torch
        total = sum(r.size for r in reqs)
        if total == 0:
            return
        if total > self.icap:
            self._grow_insert_buffers(total)
        ha, hb, da, db = self.ibuf
        na, nb = ha.numpy().view(np.uint32), hb.numpy().view(np.uint32)
        off = 0
        for r in reqs:
            na[off:off + r.size] = r.a
            nb[off:off + r.size] = r.b
            off += r.size
        s = self.istream
        with torch.cuda.stream(s):
            da[:off].copy_(ha[:off], non_blocking=True)
            db[:off].copy_(hb[:off], non_blocking=True)
            self.index.insert_edges(da[:off], db[:off], stream=s)
        s.synchronize()

    def _grow_insert_buffers(self, cap: int) -> None:
        """Pinned host staging and device copies for insertion batches of up to cap edges."""
        torch = self.torch
        self.icap = max(cap, 1 << 14)
        self.ibuf = (torch.empty(self.icap, dtype=torch.int32).pin_memory(),
                     torch.empty(self.icap, dtype=torch.int32).pin_memory(),
                     torch.empty(self.icap, dtype=torch.int32, device=self.index.device),
                     torch.empty(self.icap, dtype=torch.int32, device=self.index.device))

    def close(self) -> None:
        for q in self.jobs:
            q.put(None)
        for t in self.threads:
            t.join()
        for c in self.ctx:
            c.close()
        self.ctx = []


def latency_summary(trace: List[Request], makespan: float) -> dict:
    out = {"makespan_s": makespan, "requests": len(trace)}
    for kind in ("query", "insert"):
        rs = [r for r in trace if r.kind == kind]
        if not rs:
            continue
        lat = np.array([r.done - r.arrival for r in rs]) * 1e3
        units = sum(r.size for r in rs)
        out[kind] = {"requests": len(rs), "units": units,
                     "per_s": units / makespan if makespan > 0 else None,
                     "latency_ms_p50": float(np.percentile(lat, 50)),
                     "latency_ms_p99": float(np.percentile(lat, 99)),
                     "latency_ms_max": float(lat.max())}
    return out


def serve_alone(index, trace: List[Request], realtime: bool = True) -> dict:
    """The same trace without continuous batching: one request at a time in sequence order, each
    started when it has arrived and the one before it is done (so queueing counts in its
    latency), on one stream; returns the summary of `serve`."""
    import torch

    from .binding import to_device_ids

    t0 = time.perf_counter()
    for r in sorted(trace, key=lambda x: x.seq):
        if realtime:
            while time.perf_counter() - t0 < r.arrival:
                pass
        r.start = time.perf_counter() - t0
        a, b = to_device_ids(r.a, index.device), to_device_ids(r.b, index.device)
        if r.kind == "query":
            r.answers = index.query(a, b).cpu().numpy()
        else:
            index.insert_edges(a, b)
            torch.cuda.current_stream(index.device).synchronize()
        r.done = time.perf_counter() - t0
    return latency_summary(trace, time.perf_counter() - t0)


def serve(index, trace: List[Request], workers: int = 4, max_batch: int = 1 << 17,
          bfs_slots: int = 256, realtime: bool = True, memory_cap: Optional[int] = None):
    """Run `trace` through a continuous-batching server over `index`; returns a summary."""
    ex = GpuExecutor(index, workers=workers, max_batch=max_batch, bfs_slots=bfs_slots,
                     memory_cap=memory_cap)
    try:
        sch = Scheduler(ex, max_batch=max_batch)
        span = sch.run(trace, realtime=realtime)
    finally:
        ex.close()
    s = latency_summary(trace, span)
    s.update(workers=ex.workers, device_batches=sch.batches, admission_waits=sch.refusals,
             batch_budget_bytes=int(ex.batch_budget),
             peak_inflight_batch_bytes=int(ex.peak_inflight_bytes))
    return s
