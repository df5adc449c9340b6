"""Serving loop: admission by memory, continuous batching, timeouts,
cancellation, latency bookkeeping (CPU, virtual clock, executor that scores
with the oracle), and on the GPU, identical results for a request alone and
in a served mix."""
import numpy as np
import pytest

import oracle.cpu as ocpu
import swinputs
from paper_2203_11100_amd import serve

B62 = swinputs.blosum62()


class FakeExecutor:
    """Scores with the CPU oracle; a launch 'runs' for cells / rate seconds
    of virtual time.  Records every launch for the checks."""

    rate = 2e9          # cells per second of virtual time
    overhead = 1e-3

    def __init__(self, db, matrix, go, ge, n_slots, max_batch, clock):
        self.db, self.matrix, self.go, self.ge = db, matrix, go, ge
        self.clock = clock
        self.end = {}
        self.rows = {}
        self.launches = []        # (time, slot, k)
        self.max_inflight = 0

    def launch(self, slot, queries):
        now = self.clock.now()
        assert slot not in self.end or self.end[slot] is None
        cells = sum(len(q) for q in queries) * self.db.n_residues
        self.end[slot] = now + self.overhead + cells / self.rate
        self.rows[slot] = [ocpu.search(q, self.db.residues, self.db.offsets, self.matrix,
                                       self.go, self.ge) for q in queries]
        self.launches.append((now, slot, len(queries)))
        self.max_inflight = max(self.max_inflight, sum(1 for v in self.end.values() if v is not None))

    def poll(self, slot):
        return self.clock.now() >= self.end[slot]

    def finish(self, slot):
        t = self.end[slot]
        self.end[slot] = None
        return self.rows.pop(slot), t

    def close(self):
        pass


def _db():
    rng = np.random.default_rng(1)
    lengths = rng.integers(20, 300, 150)
    res, offs = swinputs.make_database(lengths, rng)
    w = swinputs.workloads.Workload("t", res, offs, [], B62, 10, 2)
    return w


def _trace(n, qps, seed=2, lo=30, hi=200):
    rng = np.random.default_rng(seed)
    qs = [swinputs.random_residues(int(m), rng) for m in rng.integers(lo, hi, n)]
    arr = np.cumsum(rng.exponential(1.0 / qps, n))
    return qs, arr


def _server(db, **kw):
    ex = {}

    def factory(*a):
        ex["x"] = FakeExecutor(*a)
        return ex["x"]
    kw.setdefault("slot_bytes", 100)
    kw.setdefault("memory_budget", 300)
    kw.setdefault("request_bytes_fn", lambda m: 0)
    srv = serve.Server(db, B62, 10, 2, clock=serve.VirtualClock(), executor_factory=factory, **kw)
    return srv, ex["x"]


def test_every_request_served_with_exact_scores():
    db = _db()
    qs, arr = _trace(40, qps=200)
    srv, ex = _server(db, max_batch=4)
    reqs = srv.run(qs, arr)
    assert [r.rid for r in reqs] == list(range(40))
    for r, q in zip(reqs, qs):
        assert (r.scores == ocpu.search(q, db.residues, db.offsets, B62, 10, 2)).all()
        assert r.done >= r.admitted >= r.arrival - 1e-12


def test_memory_budget_sets_slots():
    db = _db()
    srv, ex = _server(db, slot_bytes=100, memory_budget=350, max_slots=8)
    assert srv.n_slots == 3 and srv.request_memory == 50
    srv, ex = _server(db, slot_bytes=100, memory_budget=10**6, max_slots=5)
    assert srv.n_slots == 5
    with pytest.raises(MemoryError):
        _server(db, slot_bytes=100, memory_budget=99)


def test_continuous_batching_admits_as_slots_free():
    db = _db()
    qs, arr = _trace(60, qps=2000, seed=3)          # arrivals far faster than service
    srv, ex = _server(db, max_batch=3, slot_bytes=100, memory_budget=200)   # 2 slots
    reqs = srv.run(qs, arr)
    assert ex.max_inflight <= 2
    assert all(k <= 3 for _, _, k in ex.launches)
    assert any(k > 1 for _, _, k in ex.launches)               # waiting requests batch up
    # FIFO: admission order follows arrival order
    adm = sorted(reqs, key=lambda r: (r.admitted, r.arrival))
    assert [r.rid for r in adm] == sorted(r.rid for r in reqs)
    # a request that arrived while both slots were busy starts at the first
    # poll after a slot frees; with a slot free it starts at its arrival
    done_times = sorted(r.done for r in reqs)
    for r in reqs:
        if r.admitted > r.arrival + 1e-9:
            gap = min(r.admitted - t for t in done_times if t <= r.admitted + 1e-12)
            assert 0 <= gap <= srv.poll_interval + 1e-9
    # launches overlap in time: work from requests of different arrival times
    # is in flight together
    spans = sorted((min(r.admitted for r in reqs if r.slot == s and r.admitted == t0),
                    max(r.done for r in reqs if r.slot == s and r.admitted == t0))
                   for t0, s, _ in ex.launches)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))


def test_idle_server_launches_at_arrival():
    db = _db()
    qs, arr = _trace(10, qps=2, seed=4)            # sparse arrivals
    srv, ex = _server(db, max_batch=4)
    reqs = srv.run(qs, arr)
    for r in reqs:
        assert abs(r.admitted - r.arrival) < 1e-9
        assert r.batch_size == 1
        assert r.latency == pytest.approx(FakeExecutor.overhead + len(r.query) * db.n_residues
                                          / FakeExecutor.rate)


def test_summary_percentiles():
    db = _db()
    qs, arr = _trace(50, qps=500, seed=5)
    srv, ex = _server(db, max_batch=2)
    reqs = srv.run(qs, arr)
    s = serve.summarize(reqs, db.n_residues)
    lat = np.array([r.latency for r in reqs]) * 1e3
    assert s["p50_ms"] == pytest.approx(np.percentile(lat, 50))
    assert s["p99_ms"] == pytest.approx(np.percentile(lat, 99))
    assert s["p99_ms"] >= s["p50_ms"] > 0
    assert s["requests"] == 50 and s["gcups"] > 0


def test_memory_admits_requests_by_their_bytes():
    """With request bytes = query length and 400 bytes of request memory, the
    launched requests never hold more than 400 bytes at once, a batch stops
    at the first request that does not fit (FIFO), and every request is
    still served exactly."""
    db = _db()
    qs, arr = _trace(40, qps=5000, seed=8, lo=60, hi=200)    # a burst
    srv, ex = _server(db, max_batch=8, slot_bytes=100, memory_budget=100 * 4 + 400,
                      max_slots=4, min_request_len=0, request_bytes_fn=lambda m: m)
    assert srv.n_slots == 4 and srv.request_memory == 400
    reqs = srv.run(qs, arr)
    assert srv.peak_bytes <= 400
    assert all(r.status == "done" for r in reqs)
    # the bytes launched together never exceed the request memory
    for t0, slot, k in ex.launches:
        live = [r for r in reqs if r.admitted <= t0 + 1e-12 < r.done]
        assert sum(len(r.query) for r in live) <= 400
    adm = sorted(reqs, key=lambda r: (r.admitted, r.arrival))
    assert [r.rid for r in adm] == sorted(r.rid for r in reqs)
    for r, q in zip(reqs, qs):
        assert (r.scores == ocpu.search(q, db.residues, db.offsets, B62, 10, 2)).all()


def test_request_larger_than_memory_is_rejected():
    db = _db()
    qs = [np.zeros(50, np.uint8), np.zeros(500, np.uint8), np.zeros(60, np.uint8)]
    srv, ex = _server(db, slot_bytes=100, memory_budget=100 + 300, max_slots=1,
                      min_request_len=0, request_bytes_fn=lambda m: m)
    reqs = srv.run(qs, [0.0, 0.001, 0.002])
    assert [r.status for r in reqs] == ["done", "rejected", "done"]
    assert reqs[1].scores is None
    assert serve.summarize(reqs, db.n_residues)["rejected"] == 1


def test_waiting_requests_time_out():
    """One slot, a burst: requests still waiting after the timeout are
    dropped when it passes; the launched ones complete."""
    db = _db()
    qs, arr = _trace(30, qps=10000, seed=9, lo=150, hi=200)
    srv, ex = _server(db, max_batch=2, slot_bytes=100, memory_budget=100, max_slots=1,
                      min_request_len=0, request_timeout=0.05)
    reqs = srv.run(qs, arr)
    st = [r.status for r in reqs]
    assert "timeout" in st and "done" in st
    for r in reqs:
        if r.status == "timeout":
            assert r.admitted is None and r.scores is None
            assert r.done - r.arrival == pytest.approx(0.05, abs=srv.poll_interval + 1e-6)
        else:
            assert r.admitted - r.arrival <= 0.05 + 1e-9
            assert (r.scores == ocpu.search(r.query, db.residues, db.offsets, B62, 10, 2)).all()
    s = serve.summarize(reqs, db.n_residues)
    assert s["timeout"] == st.count("timeout") and s["served"] == st.count("done")


def test_cancel_waiting_and_launched_requests():
    """A request cancelled after its launch completes on the device but its
    scores are discarded; one cancelled while waiting is never launched."""
    db = _db()
    qs, arr = _trace(12, qps=10000, seed=10, lo=150, hi=200)
    srv, ex = _server(db, max_batch=1, slot_bytes=100, memory_budget=100, max_slots=1,
                      min_request_len=0)
    launch = ex.launch

    def launch_then_cancel(slot, queries):       # another thread cancels 0 and 7
        launch(slot, queries)
        if len(ex.launches) == 1:
            srv.cancel(0)
            srv.cancel(7)
    ex.launch = launch_then_cancel
    reqs = srv.run(qs, arr)
    assert reqs[0].status == "cancelled" and reqs[0].admitted is not None
    assert reqs[7].status == "cancelled" and reqs[7].admitted is None
    assert len(ex.launches) == 11
    assert all(r.status == "done" for r in reqs if r.rid not in (0, 7))
    assert reqs[0].scores is None and reqs[7].scores is None


@pytest.mark.gpu
def test_served_results_same_alone_and_in_mix():
    import torch
    import paper_2203_11100_amd as sw
    assert torch.cuda.is_available()
    w = swinputs.config("plain", scale=0.02)
    qs, arr = _trace(36, qps=400, seed=6, lo=30, hi=900)
    with sw.Database(w.residues, w.offsets) as db:
        srv = serve.Server(db, w.matrix, 10, 2, max_slots=3, max_batch=4)
        srv.ex.warm(1024)
        reqs = srv.run(qs, arr)
        srv.close()
        alone = [db.search(q, w.matrix, 10, 2) for q in qs]
    assert any(r.batch_size > 1 for r in reqs)
    assert all(r.status == "done" for r in reqs)
    for r, a in zip(reqs, alone):
        assert (r.scores == a).all(), r.rid
    rng = np.random.default_rng(7)
    ids = rng.choice(w.n_seqs, 30, replace=False)
    for r in reqs[::6]:
        want = ocpu.search(r.query, w.residues, w.offsets, w.matrix, 10, 2, ids=ids)
        assert (r.scores[ids] == want).all()
    s = serve.summarize(reqs, w.n_residues)
    assert np.isfinite(s["p99_ms"]) and s["p99_ms"] >= s["p50_ms"] > 0
