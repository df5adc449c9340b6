"""GPU parity of the hybrid CPU + GPU search (sw_search_hybrid): every score
compared with the oracle, whichever side computed it."""
import sys

import numpy as np
import pytest

import oracle.cpu as ocpu
import swinputs

pytestmark = pytest.mark.gpu

B62 = swinputs.blosum62()


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def sw():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2203_11100_amd as lib
    return lib


def _covered(st, offs, lengths_of_short):
    """Every short sequence is scored by one side at least: the GPU's bins
    hold 128 slots each, the host's count is of sequences."""
    return st["gpu_bins"] * 128 + st["cpu_seqs"] >= lengths_of_short


@pytest.mark.parametrize("threads,share", [(1, 300), (4, 300), (0, 300), (4, 0), (8, 1000)])
def test_hybrid_matches_oracle(sw, threads, share):
    """Fixed host shares (the host certainly scores some sequences, up to
    all it can reach) and the planned split; every score exact."""
    rng = np.random.default_rng(40 + threads)
    lengths = np.concatenate([[0, 0, 1, 5, 64, 129], rng.integers(20, 700, 6000),
                              [2100, 3000, 9000]]).astype(np.int64)
    res, offs = swinputs.make_database(lengths, rng)
    n_short = int((lengths < sw.SW_DEFAULT_LONG_THRESHOLD).sum())
    with sw.Database(res, offs) as db:
        db.set_option(sw.SW_OPT_HYBRID_SHARE, share)
        for m in (1, 144, 600):
            q = swinputs.random_residues(m, rng)
            say("hybrid threads=%d share=%d m=%d" % (threads, share, m))
            got, st = db.search_hybrid(q, B62, 10, 2, cpu_threads=threads)
            want = ocpu.search(q, res, offs, B62, 10, 2)
            assert (got == want).all(), np.nonzero(got != want)[0][:5]
            assert st["gpu_bins"] <= sw.plan(offs)["n_bins"]
            assert _covered(st, offs, n_short)
            assert st["gpu_cells"] + st["cpu_cells"] == m * int(offs[-1])
            if share:
                assert st["cpu_seqs"] > 0


def test_hybrid_planted_scores_beyond_half_precision_on_both_sides(sw):
    """Scores beyond the half-precision range in short bins of every length:
    exact whether the GPU (rescoring list) or the host (16-bit, 32-bit
    rescoring) scores them; the host is planned half of the cells and keeps
    every sequence it reaches before the GPU does."""
    rng = np.random.default_rng(50)
    W = 17
    q = np.full(1500, W, np.uint8)
    lengths = rng.integers(20, 1600, 6000).astype(np.int64)
    res, offs = swinputs.make_database(lengths, rng)
    res = res.copy()
    planted = rng.choice(np.nonzero(lengths >= 200)[0], 300, replace=False)
    for sid in planted:
        k = int(min(lengths[sid], 1500))
        res[offs[sid]:offs[sid] + k] = W
    with sw.Database(res, offs) as db:
        db.set_option(sw.SW_OPT_HYBRID_SHARE, 500)
        got, st = db.search_hybrid(q, B62, 10, 2, cpu_threads=8)
    say("planted hybrid: %s" % st)
    want = ocpu.search(q, res, offs, B62, 10, 2)
    assert (got == want).all()
    assert (want[planted] > 2048).all() and st["cpu_seqs"] > 0 and st["gpu_bins"] > 0


def test_hybrid_planned_split_does_not_slow_the_search(sw):
    """With the split planned from measured rates, repeated hybrid searches
    of a query take about as long as the GPU-only search of it (the host
    never holds the GPU back for long), with identical scores."""
    import time
    rng = np.random.default_rng(60)
    lengths = swinputs.lognormal_lengths(60_000, 355.0, 0.75, 20, 5000, rng)
    res, offs = swinputs.make_database(lengths, rng)
    q = swinputs.random_residues(400, rng)
    with sw.Database(res, offs) as db:
        # the GPU-only search on the same kernels (the hybrid search hands no
        # bins to the long-pair kernel)
        db.set_option(sw.SW_OPT_OFFLOAD_BINS, 0)
        base = db.search(q, B62, 10, 2)
        t0 = time.perf_counter()
        for _ in range(5):
            db.search(q, B62, 10, 2)
        gpu_s = (time.perf_counter() - t0) / 5
        for _ in range(3):                 # the rates settle
            got, st = db.search_hybrid(q, B62, 10, 2)
        t0 = time.perf_counter()
        for _ in range(5):
            got, st = db.search_hybrid(q, B62, 10, 2)
        hyb_s = (time.perf_counter() - t0) / 5
    say("gpu-only %.2f ms, hybrid %.2f ms, %s" % (gpu_s * 1e3, hyb_s * 1e3, st))
    assert (got == base).all()
    assert hyb_s < 1.5 * gpu_s + 2e-3


def test_hybrid_full_size_plain_shortest_query(sw):
    from conftest import workload, oracle_row
    w = workload("plain")
    q = w.queries[0]
    with sw.Database(w.residues, w.offsets) as db:
        say("hybrid, full plain database, m=%d" % len(q))
        got, st = db.search_hybrid(q, w.matrix, 10, 2)
        say("hybrid stats: %s" % st)
    want = oracle_row(w, q)
    assert (got == want).all(), np.nonzero(got != want)[0][:5]
