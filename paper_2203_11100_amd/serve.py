"""Continuous-batching search server over one resident database.

Requests (protein queries) arrive over time.  The server keeps a fixed number
of slots, each a search context of the database with its own HIP stream and
buffers; the slot count is what a device-memory budget admits.  Whenever a
slot is free and requests are waiting, the waiting requests (up to
`max_batch`, oldest first) are launched together on that slot - one search,
or one batched search with the queries paired two per register lane - while
earlier launches are still running on other slots, so work from requests that
arrived at different times overlaps on the device.  A request's latency is
its completion time (the GPU timestamp of its launch's last kernel, mapped to
the host clock) minus its arrival time.

All scoring runs in libswdb.so's kernels; this module only schedules.  The
executor and clock are pluggable so the scheduling logic can be tested
without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from . import SW_OPT_GRAPHS


@dataclasses.dataclass
class Request:
    rid: int
    query: np.ndarray
    arrival: float                      # seconds on the server clock
    admitted: Optional[float] = None
    done: Optional[float] = None
    slot: Optional[int] = None
    batch_size: int = 0
    scores: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class RealClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def sleep(self, dt: float):
        if dt > 0:
            time.sleep(dt)


class VirtualClock:
    """A clock that only moves when the scheduler sleeps (for tests)."""

    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def sleep(self, dt: float):
        self.t += max(dt, 0.0)


class GpuExecutor:
    """Runs request batches on search contexts, one HIP stream per slot."""

    def __init__(self, db, matrix, gap_open: int, gap_extend: int, n_slots: int,
                 max_batch: int, max_query_len: int, clock):
        import torch
        self.torch = torch
        self.db, self.matrix, self.go, self.ge = db, matrix, gap_open, gap_extend
        self.n_slots, self.max_batch, self.max_query_len = n_slots, max_batch, max_query_len
        self.clock = clock
        n = db.n_seqs
        self.ctx = [db.context() for _ in range(n_slots)]
        for c in self.ctx:
            c.set_option(SW_OPT_GRAPHS, 0)      # every batch is new: no capture
        self.stream = [torch.cuda.Stream() for _ in range(n_slots)]
        self.d_out = [torch.empty((max_batch, n), dtype=torch.int32, device="cuda")
                      for _ in range(n_slots)]
        self.d_q = [torch.empty(max_batch * max_query_len + 1, dtype=torch.uint8, device="cuda")
                    for _ in range(n_slots)]
        self.h_out = [torch.empty((max_batch, n), dtype=torch.int32).pin_memory()
                      for _ in range(n_slots)]
        self.ev = [torch.cuda.Event(enable_timing=True) for _ in range(n_slots)]
        self.k = [0] * n_slots
        # map GPU event times to the host clock
        torch.cuda.synchronize()
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record()
        self.ref.synchronize()
        self.ref_host = clock.now()

    @staticmethod
    def slot_bytes(db, max_batch: int, max_query_len: int) -> int:
        """Device bytes one slot needs: context scratch, outputs, queries and
        the per-query profiles of a full batch."""
        n = db.n_seqs
        prof = max_batch * (max_query_len + 512) * (26 * 4 + 25)
        return db.context_bytes() + max_batch * n * 4 + max_batch * max_query_len + prof

    def warm(self):
        """Runs a full-size batch on every slot so no buffer grows later."""
        rng = np.random.default_rng(0)
        for s in range(self.n_slots):
            qs = [rng.integers(0, 20, self.max_query_len).astype(np.uint8)
                  for _ in range(self.max_batch)]
            self.launch(s, qs)
        self.torch.cuda.synchronize()

    def launch(self, slot: int, queries: Sequence[np.ndarray]):
        torch = self.torch
        k = len(queries)
        cat = np.concatenate(queries) if k else np.zeros(0, np.uint8)
        st = self.stream[slot]
        with torch.cuda.stream(st):
            dq = self.d_q[slot][:len(cat)]
            if len(cat):
                dq.copy_(torch.from_numpy(cat), non_blocking=False)
            if k == 1:
                self.ctx[slot].search_async(dq, self.matrix, self.go, self.ge,
                                            self.d_out[slot][0], st)
            else:
                qoffs = np.zeros(k + 1, np.int64)
                np.cumsum([len(q) for q in queries], out=qoffs[1:])
                self.ctx[slot].search_batch_async(dq, qoffs, self.matrix, self.go, self.ge,
                                                  self.d_out[slot][:k], st)
            self.h_out[slot][:k].copy_(self.d_out[slot][:k], non_blocking=True)
            self.ev[slot].record(st)
        self.k[slot] = k

    def poll(self, slot: int) -> bool:
        return self.ev[slot].query()

    def finish(self, slot: int):
        self.ev[slot].synchronize()
        t = self.ref_host + self.ref.elapsed_time(self.ev[slot]) / 1e3
        rows = [self.h_out[slot][i].numpy().copy() for i in range(self.k[slot])]
        return rows, t

    def close(self):
        self.torch.cuda.synchronize()
        for c in self.ctx:
            c.close()


class Server:
    """Admission by memory, continuous batching, latency bookkeeping.

    db             : the resident Database
    memory_budget  : device bytes the server may use for slots (None: 4 GiB)
    max_slots      : upper bound on concurrent launches
    max_batch      : requests launched together on one slot
    max_query_len  : longer queries are rejected at submission
    """

    def __init__(self, db, matrix, gap_open: int = 10, gap_extend: int = 2, *,
                 memory_budget: Optional[int] = None, max_slots: int = 8, max_batch: int = 8,
                 max_query_len: int = 5000, clock=None, executor_factory: Callable = None,
                 slot_bytes: Optional[int] = None):
        self.clock = clock or RealClock()
        budget = (4 << 30) if memory_budget is None else int(memory_budget)
        per_slot = slot_bytes if slot_bytes is not None else \
            GpuExecutor.slot_bytes(db, max_batch, max_query_len)
        self.n_slots = int(min(max_slots, budget // max(per_slot, 1)))
        if self.n_slots < 1:
            raise MemoryError("memory budget %d B admits no slot (%d B per slot)"
                              % (budget, per_slot))
        self.max_batch, self.max_query_len = max_batch, max_query_len
        factory = executor_factory or GpuExecutor
        self.ex = factory(db, matrix, gap_open, gap_extend, self.n_slots, max_batch,
                          max_query_len, self.clock)
        self.poll_interval = 2e-4

    def close(self):
        self.ex.close()

    def run(self, queries: Sequence[np.ndarray], arrivals: Sequence[float]) -> List[Request]:
        """Serves a trace: query i arrives `arrivals[i]` seconds after start."""
        order = np.argsort(np.asarray(arrivals, dtype=np.float64), kind="stable")
        reqs = [Request(int(i), np.ascontiguousarray(queries[i], dtype=np.uint8),
                        float(arrivals[i])) for i in order]
        for r in reqs:
            if len(r.query) > self.max_query_len:
                raise ValueError("request %d: query longer than %d" % (r.rid, self.max_query_len))
        start = self.clock.now()
        for r in reqs:
            r.arrival += start
        pending: collections.deque = collections.deque()
        busy: Dict[int, List[Request]] = {}
        free = list(range(self.n_slots))[::-1]
        nxt, done = 0, 0
        while done < len(reqs):
            now = self.clock.now()
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                pending.append(reqs[nxt])
                nxt += 1
            progressed = False
            for slot in list(busy):
                if self.ex.poll(slot):
                    rows, t = self.ex.finish(slot)
                    for r, row in zip(busy.pop(slot), rows):
                        r.scores, r.done = row, max(t, r.admitted)
                        done += 1
                    free.append(slot)
                    progressed = True
            while free and pending:
                slot = free.pop()
                k = min(self.max_batch, len(pending))
                batch = [pending.popleft() for _ in range(k)]
                now = self.clock.now()
                for r in batch:
                    r.admitted, r.slot, r.batch_size = now, slot, k
                self.ex.launch(slot, [r.query for r in batch])
                busy[slot] = batch
                progressed = True
            if not progressed:
                # poll running launches; with a free slot, wake exactly at the
                # next arrival if it comes sooner
                wait = self.poll_interval if busy else math.inf
                if free and nxt < len(reqs):
                    wait = min(wait, max(reqs[nxt].arrival - self.clock.now(), 0.0))
                self.clock.sleep(0.0 if wait == math.inf else wait)
        for r in reqs:
            r.arrival -= start
            r.admitted -= start
            r.done -= start
        return sorted(reqs, key=lambda r: r.rid)


def summarize(reqs: Sequence[Request], n_residues: int) -> dict:
    """p50/p99 latency and throughput (GCUPS over the first arrival to the
    last completion) of a served trace."""
    lat = np.array([r.latency for r in reqs], dtype=np.float64)
    cells = float(sum(len(r.query) for r in reqs)) * n_residues
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    return {"requests": len(reqs), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat.max() * 1e3), "window_s": span, "gcups": cells / span / 1e9,
            "mean_batch": float(np.mean([r.batch_size for r in reqs]))}
