"""Failure paths on the GPU, forced from the host: a concurrent call on a
busy handle returns SW_EBUSY, and a database load that cannot get device
memory returns SW_ENOMEM and leaves the library usable.  No kernel is made
to fault; every launch completes normally."""
import sys
import threading
import time

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


def test_concurrent_call_on_busy_handle_is_ebusy(sw):
    """While one thread's batched search (about a second of work) holds the
    handle, a second thread's search on it returns SW_EBUSY at once; the
    first search's scores stay exact and the handle works afterwards."""
    rng = np.random.default_rng(1)
    res, offs = swinputs.make_database(rng.integers(200, 500, 100_000).astype(np.int64), rng)
    qs = [swinputs.random_residues(5000, rng) for _ in range(30)]
    small = swinputs.random_residues(100, rng)
    with sw.Database(res, offs) as db:
        started = threading.Event()
        result = {}

        def long_call():
            started.set()
            result["rows"] = db.search_batch(qs, B62, 10, 2)

        t = threading.Thread(target=long_call)
        t.start()
        started.wait()
        time.sleep(0.1)
        say("second call while the batch runs")
        with pytest.raises(sw.SwError) as ei:
            db.search(small, B62, 10, 2)
        busy_during = t.is_alive()
        t.join()
        assert ei.value.code == sw._native.SW_EBUSY and busy_during
        ids = rng.choice(db.n_seqs, 20, replace=False)
        assert (result["rows"][0][ids] == ocpu.search(qs[0], res, offs, B62, 10, 2, ids=ids)).all()
        assert (db.search(small, B62, 10, 2) == ocpu.search(small, res, offs, B62, 10, 2)).all()


def test_device_memory_exhausted_is_enomem(sw):
    """With nearly all device memory taken by another allocation, loading a
    database returns SW_ENOMEM (no handle, no crash); once the memory is
    free again the same load and a search succeed."""
    import torch
    rng = np.random.default_rng(2)
    res, offs = swinputs.make_database(rng.integers(300, 500, 300_000).astype(np.int64), rng)
    free, _ = torch.cuda.mem_get_info()
    hog = torch.empty(max(free - (64 << 20), 1), dtype=torch.uint8, device="cuda")
    say("holding %.1f GB of device memory" % (hog.numel() / 1e9))
    try:
        with pytest.raises(sw.SwError) as ei:
            sw.Database(res, offs)
        assert ei.value.code == sw._native.SW_ENOMEM
    finally:
        del hog
        torch.cuda.empty_cache()
    q = swinputs.random_residues(120, rng)
    with sw.Database(res, offs) as db:
        ids = rng.choice(db.n_seqs, 50, replace=False)
        got = db.search(q, B62, 10, 2)
        assert (got[ids] == ocpu.search(q, res, offs, B62, 10, 2, ids=ids)).all()


def test_library_first_then_torch_in_a_fresh_process():
    """A process that loads a database before it touches PyTorch's GPU
    functions can still use them: the binding lets PyTorch's HIP runtime
    open the device first."""
    import subprocess
    import os
    code = ("import numpy as np, swinputs, paper_2203_11100_amd as sw\n"
            "rng = np.random.default_rng(0)\n"
            "res, offs = swinputs.make_database(rng.integers(20, 300, 500).astype(np.int64), rng)\n"
            "db = sw.Database(res, offs)\n"
            "got = db.search(swinputs.random_residues(50, rng), swinputs.blosum62(), 10, 2)\n"
            "import torch\n"
            "s = torch.cuda.Stream()\n"
            "x = torch.ones(4, device='cuda') * 2\n"
            "assert float(x.sum()) == 8.0 and got.shape == (500,)\n"
            "db.close()\n"
            "print('ok')\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    say("database first, then torch, in a child process")
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stderr[-2000:]
