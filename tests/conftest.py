import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


# Oracle score rows and workloads shared by the full-size GPU parity tests
# (the plain and batched workloads share their database and 20 queries, so a
# row the oracle computed for one is reused by the other within a session).
_WORKLOADS = {}
_ORACLE_ROWS = {}


def workload(name, **kw):
    import swinputs
    key = (name, tuple(sorted(kw.items())))
    if key not in _WORKLOADS:
        _WORKLOADS[key] = swinputs.config(name, **kw)
    return _WORKLOADS[key]


def oracle_row(w, query, go=10, ge=2):
    """Every score of `query` against the whole database of workload `w`,
    from the CPU oracle, cached by (database, query bytes, gaps)."""
    import hashlib
    import numpy as np
    import oracle.cpu as ocpu
    db_key = getattr(w, "_db_key", None)
    if db_key is None:
        h = hashlib.sha1(np.ascontiguousarray(w.residues))
        h.update(np.ascontiguousarray(w.offsets))
        db_key = w._db_key = h.hexdigest()
    key = (db_key, hashlib.sha1(np.ascontiguousarray(query)).hexdigest(), go, ge)
    if key not in _ORACLE_ROWS:
        _ORACLE_ROWS[key] = ocpu.search(query, w.residues, w.offsets, w.matrix, go, ge)
    return _ORACLE_ROWS[key]
