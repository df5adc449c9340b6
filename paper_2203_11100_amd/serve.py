"""Continuous-batching search server over one resident database.

Requests (protein queries) arrive over time.  The server runs a fixed number
of slots, each a search context of the database with its own HIP stream and
scratch, and admits requests by device memory: every request holds the
device bytes its search needs (its score row, its query and its share of the
batch's profiles) from launch until its scores are back on the host, and a
request is launched only while the bytes of all launched requests stay
within the memory left after the slots' fixed scratch.  Whenever a slot is
free and requests are waiting, the waiting requests (oldest first, up to
`max_batch`, as many as the memory admits) are launched together on that
slot - one search, or one batched search with the queries paired two per
register lane - while earlier launches are still running on other slots, so
work from requests that arrived at different times overlaps on the device.

A request still waiting `request_timeout` seconds after its arrival is
dropped ("timeout"); `cancel(rid)` drops a waiting request at once and
discards the scores of a launched one ("cancelled"); a request whose bytes
exceed the request memory on their own is refused at arrival ("rejected").
A served request's latency is its completion time (the GPU timestamp of its
launch's last copy, mapped to the host clock) minus its arrival time.

All scoring runs in libswdb.so's kernels; this module only schedules.  The
executor and clock are pluggable so the scheduling logic can be tested
without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import threading
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

from . import SW_OPT_GRAPHS


@dataclasses.dataclass
class Request:
    rid: int
    query: np.ndarray
    arrival: float                      # seconds on the server clock
    nbytes: int = 0                     # device bytes held while launched
    admitted: Optional[float] = None
    done: Optional[float] = None
    slot: Optional[int] = None
    batch_size: int = 0
    scores: Optional[np.ndarray] = None
    status: str = "pending"             # then "done", "timeout", "cancelled" or "rejected"

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


def request_bytes(n_seqs: int, query_len: int) -> int:
    """Device bytes one request holds while launched: its int32 score row,
    its query codes, and its profiles (the binary16 pair profile, 26 codes x
    4 bytes per row, and the 32-bit kernel's int8 profile, 25 codes per row
    padded to 512 rows)."""
    return 4 * n_seqs + query_len + 104 * (query_len + 32) + 25 * (query_len + 512)


class GpuExecutor:
    """Runs request batches on search contexts, one HIP stream per slot.
    Score rows and query buffers come from PyTorch's caching allocator (one
    allocation per launch, reused once warm); query bytes go up and scores
    come back through pinned host buffers, so a launch never blocks the
    scheduling thread."""

    def __init__(self, db, matrix, gap_open: int, gap_extend: int, n_slots: int,
                 max_batch: int, clock):
        import torch
        self.torch = torch
        self.db, self.matrix, self.go, self.ge = db, matrix, gap_open, gap_extend
        self.n_slots, self.max_batch = n_slots, max_batch
        self.clock = clock
        n = db.n_seqs
        self.ctx = [db.context() for _ in range(n_slots)]
        for c in self.ctx:
            c.set_option(SW_OPT_GRAPHS, 0)      # every batch is new: no capture
        self.stream = [torch.cuda.Stream() for _ in range(n_slots)]
        self.h_out = [torch.empty((max_batch, n), dtype=torch.int32).pin_memory()
                      for _ in range(n_slots)]
        self.h_q = [torch.empty(1, dtype=torch.uint8).pin_memory() for _ in range(n_slots)]
        self.live = [None] * n_slots            # device buffers of the slot's launch
        self.ev = [torch.cuda.Event(enable_timing=True) for _ in range(n_slots)]
        self.k = [0] * n_slots
        # map GPU event times to the host clock
        torch.cuda.synchronize()
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record()
        self.ref.synchronize()
        self.ref_host = clock.now()

    @staticmethod
    def slot_bytes(db, max_batch: int) -> int:
        """Fixed device bytes of one slot: its search context's scratch."""
        return db.context_bytes()

    def warm(self, query_len: int = 5000):
        """Runs a full batch of long queries on every slot, so that no
        context buffer, pinned buffer or allocator block grows later."""
        rng = np.random.default_rng(0)
        for s in range(self.n_slots):
            qs = [rng.integers(0, 20, query_len).astype(np.uint8) for _ in range(self.max_batch)]
            self.launch(s, qs)
        for s in range(self.n_slots):
            self.finish(s)

    def launch(self, slot: int, queries: Sequence[np.ndarray]):
        torch = self.torch
        k = len(queries)
        cat = np.concatenate(queries) if k else np.zeros(0, np.uint8)
        st = self.stream[slot]
        if self.h_q[slot].numel() < len(cat):
            self.h_q[slot] = torch.empty(max(len(cat), 1), dtype=torch.uint8).pin_memory()
        hq = self.h_q[slot][:len(cat)]
        if len(cat):
            hq.numpy()[:] = cat
        with torch.cuda.stream(st):
            dq = torch.empty(max(len(cat), 1), dtype=torch.uint8, device="cuda")[:len(cat)]
            d_out = torch.empty((k, self.db.n_seqs), dtype=torch.int32, device="cuda")
            if len(cat):
                dq.copy_(hq, non_blocking=True)
            if k == 1:
                self.ctx[slot].search_async(dq, self.matrix, self.go, self.ge, d_out[0], st)
            else:
                qoffs = np.zeros(k + 1, np.int64)
                np.cumsum([len(q) for q in queries], out=qoffs[1:])
                self.ctx[slot].search_batch_async(dq, qoffs, self.matrix, self.go, self.ge,
                                                  d_out, st)
            self.h_out[slot][:k].copy_(d_out, non_blocking=True)
            self.ev[slot].record(st)
        self.live[slot] = (dq, d_out)
        self.k[slot] = k

    def poll(self, slot: int) -> bool:
        return self.ev[slot].query()

    def finish(self, slot: int):
        self.ev[slot].synchronize()
        t = self.ref_host + self.ref.elapsed_time(self.ev[slot]) / 1e3
        rows = [self.h_out[slot][i].numpy().copy() for i in range(self.k[slot])]
        self.live[slot] = None
        return rows, t

    def close(self):
        self.torch.cuda.synchronize()
        for c in self.ctx:
            c.close()


class Server:
    """Admission by memory, continuous batching, timeouts, cancellation and
    latency bookkeeping.

    db              : the resident Database
    memory_budget   : device bytes for the slots' scratch and the launched
                      requests together (None: 4 GiB)
    max_slots       : upper bound on concurrent launches
    max_batch       : requests launched together on one slot
    request_timeout : seconds a request may wait for launch (None: no limit)
    min_request_len : the slot count leaves room for one request of this
                      query length beside the slots' scratch
    """

    def __init__(self, db, matrix, gap_open: int = 10, gap_extend: int = 2, *,
                 memory_budget: Optional[int] = None, max_slots: int = 8, max_batch: int = 8,
                 request_timeout: Optional[float] = None, min_request_len: int = 5000,
                 clock=None, executor_factory: Callable = None,
                 slot_bytes: Optional[int] = None,
                 request_bytes_fn: Optional[Callable[[int], int]] = None):
        self.clock = clock or RealClock()
        budget = (4 << 30) if memory_budget is None else int(memory_budget)
        per_slot = slot_bytes if slot_bytes is not None else \
            GpuExecutor.slot_bytes(db, max_batch)
        self.request_bytes = request_bytes_fn or (lambda m: request_bytes(db.n_seqs, m))
        room = self.request_bytes(min_request_len)
        self.n_slots = int(min(max_slots, (budget - room) // max(per_slot, 1)))
        if self.n_slots < 1:
            raise MemoryError("memory budget %d B admits no slot (%d B per slot, %d B for one "
                              "request)" % (budget, per_slot, room))
        self.request_memory = budget - self.n_slots * per_slot
        self.max_batch = max_batch
        self.request_timeout = request_timeout
        factory = executor_factory or GpuExecutor
        self.ex = factory(db, matrix, gap_open, gap_extend, self.n_slots, max_batch, self.clock)
        self.poll_interval = 2e-4
        self.inflight_bytes = 0
        self.peak_bytes = 0
        self._cancel = set()
        self._cancel_lock = threading.Lock()

    def close(self):
        self.ex.close()

    def cancel(self, rid: int):
        """Cancels request `rid` (any thread): dropped if still waiting, its
        scores discarded if already launched."""
        with self._cancel_lock:
            self._cancel.add(int(rid))

    def _cancelled(self, rid: int) -> bool:
        with self._cancel_lock:
            return rid in self._cancel

    def run(self, queries: Sequence[np.ndarray], arrivals: Sequence[float]) -> List[Request]:
        """Serves a trace: query i arrives `arrivals[i]` seconds after start.
        Returns every request (by rid) with its status."""
        order = np.argsort(np.asarray(arrivals, dtype=np.float64), kind="stable")
        reqs = [Request(int(i), np.ascontiguousarray(queries[i], dtype=np.uint8),
                        float(arrivals[i])) for i in order]
        for r in reqs:
            r.nbytes = int(self.request_bytes(len(r.query)))
        start = self.clock.now()
        for r in reqs:
            r.arrival += start
        pending: collections.deque = collections.deque()
        busy: Dict[int, List[Request]] = {}
        free = list(range(self.n_slots))[::-1]
        nxt, closed = 0, 0

        def close_req(r, status, t):
            nonlocal closed
            r.status, r.done = status, t
            closed += 1

        while closed < len(reqs):
            now = self.clock.now()
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                r = reqs[nxt]
                nxt += 1
                if r.nbytes > self.request_memory:
                    close_req(r, "rejected", now)
                else:
                    pending.append(r)
            progressed = False
            for slot in list(busy):
                if self.ex.poll(slot):
                    rows, t = self.ex.finish(slot)
                    for r, row in zip(busy.pop(slot), rows):
                        self.inflight_bytes -= r.nbytes
                        if self._cancelled(r.rid):
                            close_req(r, "cancelled", max(t, r.admitted))
                        else:
                            r.scores = row
                            close_req(r, "done", max(t, r.admitted))
                    free.append(slot)
                    progressed = True
            # waiting requests that were cancelled or waited too long
            if pending:
                now = self.clock.now()
                keep = collections.deque()
                for r in pending:
                    if self._cancelled(r.rid):
                        close_req(r, "cancelled", now)
                    elif self.request_timeout is not None and \
                            now - r.arrival > self.request_timeout:
                        close_req(r, "timeout", now)
                    else:
                        keep.append(r)
                progressed |= len(keep) != len(pending)
                pending = keep
            # launch: oldest first, as many as fit the request memory
            while free and pending and \
                    self.inflight_bytes + pending[0].nbytes <= self.request_memory:
                slot = free.pop()
                batch = []
                while pending and len(batch) < self.max_batch and \
                        self.inflight_bytes + pending[0].nbytes <= self.request_memory:
                    r = pending.popleft()
                    self.inflight_bytes += r.nbytes
                    batch.append(r)
                self.peak_bytes = max(self.peak_bytes, self.inflight_bytes)
                now = self.clock.now()
                for r in batch:
                    r.admitted, r.slot, r.batch_size = now, slot, len(batch)
                self.ex.launch(slot, [r.query for r in batch])
                busy[slot] = batch
                progressed = True
            if not progressed:
                # poll running launches; with a free slot and memory, wake
                # exactly at the next arrival or timeout if it comes sooner
                wait = self.poll_interval if busy else math.inf
                if free and nxt < len(reqs):
                    wait = min(wait, max(reqs[nxt].arrival - self.clock.now(), 0.0))
                if pending and self.request_timeout is not None:
                    due = pending[0].arrival + self.request_timeout - self.clock.now()
                    wait = min(wait, max(due, 0.0) + 1e-9)
                self.clock.sleep(0.0 if wait == math.inf else wait)
        for r in reqs:
            r.arrival -= start
            if r.admitted is not None:
                r.admitted -= start
            r.done -= start
        return sorted(reqs, key=lambda r: r.rid)


def summarize(reqs: Sequence[Request], n_residues: int) -> dict:
    """p50/p99 latency and throughput (GCUPS of the served requests over the
    first arrival to the last completion) of a served trace, with the count
    of each other outcome."""
    served = [r for r in reqs if r.status == "done"]
    counts = collections.Counter(r.status for r in reqs)
    out = {"requests": len(reqs), "served": len(served), "timeout": counts.get("timeout", 0),
           "cancelled": counts.get("cancelled", 0), "rejected": counts.get("rejected", 0)}
    if not served:
        return out
    lat = np.array([r.latency for r in served], dtype=np.float64)
    cells = float(sum(len(r.query) for r in served)) * n_residues
    span = max(r.done for r in served) - min(r.arrival for r in reqs)
    out.update({"p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
                "max_ms": float(lat.max() * 1e3), "window_s": span, "gcups": cells / span / 1e9,
                "mean_batch": float(np.mean([r.batch_size for r in served]))})
    return out
