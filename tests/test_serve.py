"""Serving loop: admission by memory, continuous batching, latency
bookkeeping (CPU, virtual clock, executor that scores with the oracle), and
on the GPU, identical results for a request alone and in a served mix."""
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

    def __init__(self, db, matrix, go, ge, n_slots, max_batch, max_query_len, clock):
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
    assert srv.n_slots == 3
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


def test_rejects_over_long_query():
    db = _db()
    srv, ex = _server(db, max_query_len=100)
    with pytest.raises(ValueError):
        srv.run([np.zeros(101, np.uint8)], [0.0])


@pytest.mark.gpu
def test_served_results_same_alone_and_in_mix():
    import torch
    import paper_2203_11100_amd as sw
    assert torch.cuda.is_available()
    w = swinputs.config("plain", scale=0.02)
    qs, arr = _trace(36, qps=400, seed=6, lo=30, hi=900)
    with sw.Database(w.residues, w.offsets) as db:
        srv = serve.Server(db, w.matrix, 10, 2, max_slots=3, max_batch=4, max_query_len=1024)
        srv.ex.warm()
        reqs = srv.run(qs, arr)
        srv.close()
        alone = [db.search(q, w.matrix, 10, 2) for q in qs]
    assert any(r.batch_size > 1 for r in reqs)
    for r, a in zip(reqs, alone):
        assert (r.scores == a).all(), r.rid
    rng = np.random.default_rng(7)
    ids = rng.choice(w.n_seqs, 30, replace=False)
    for r in reqs[::6]:
        want = ocpu.search(r.query, w.residues, w.offsets, w.matrix, 10, 2, ids=ids)
        assert (r.scores[ids] == want).all()
    s = serve.summarize(reqs, w.n_residues)
    assert np.isfinite(s["p99_ms"]) and s["p99_ms"] >= s["p50_ms"] > 0
