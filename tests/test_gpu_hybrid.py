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


@pytest.mark.parametrize("threads", [1, 4, 0])
def test_hybrid_matches_oracle(sw, threads):
    rng = np.random.default_rng(40 + threads)
    lengths = np.concatenate([[0, 0, 1, 5, 64, 129], rng.integers(20, 700, 6000),
                              [2100, 3000, 9000]]).astype(np.int64)
    res, offs = swinputs.make_database(lengths, rng)
    with sw.Database(res, offs) as db:
        for m in (1, 144, 600):
            q = swinputs.random_residues(m, rng)
            say("hybrid threads=%d m=%d" % (threads, m))
            got, st = db.search_hybrid(q, B62, 10, 2, cpu_threads=threads)
            want = ocpu.search(q, res, offs, B62, 10, 2)
            assert (got == want).all(), np.nonzero(got != want)[0][:5]
            assert st["gpu_bins"] + st["cpu_bins"] == sw.plan(offs)["n_bins"]
            assert st["gpu_cells"] + st["cpu_cells"] == m * int(offs[-1])


def test_hybrid_planted_overflow_on_both_sides(sw):
    """Scores beyond 16 bits in short bins: exact whether the GPU (rescoring
    list) or the host (32-bit rescoring) scores them."""
    rng = np.random.default_rng(50)
    W = 17
    q = np.full(1500, W, np.uint8)
    lengths = rng.integers(20, 1600, 3000).astype(np.int64)
    res, offs = swinputs.make_database(lengths, rng)
    res = res.copy()
    big = np.nonzero(lengths >= 1500)[0]
    for sid in big[:40]:
        res[offs[sid]:offs[sid] + 1500] = W
    with sw.Database(res, offs) as db:
        got, st = db.search_hybrid(q, B62, 10, 2, cpu_threads=8)
    want = ocpu.search(q, res, offs, B62, 10, 2)
    assert (got == want).all()
    assert (got[big[:40]] == 11 * 1500).all()


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
