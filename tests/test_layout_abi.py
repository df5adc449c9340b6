"""Host-side tests of the library (no GPU needed): the database layout that
sw_db_load uploads, argument validation, and the exported C ABI."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2203_11100_amd as sw
from paper_2203_11100_amd import _native
import swinputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _db(lengths, seed=0):
    rng = np.random.default_rng(seed)
    lengths = np.asarray(lengths, dtype=np.int64)
    return swinputs.make_database(lengths, rng)


def _unpack(p, offsets):
    """Rebuilds every short sequence from the interleaved store."""
    packed = p["packed"]
    seqs = {}
    for b, (res_off, rb_off, blen, slot0) in enumerate(p["bins"]):
        assert blen % 4 == 0 and blen >= sw.SW_MIN_BIN_LEN
        for k in range(sw.SW_BIN_SEQS):
            words = packed[res_off + k: res_off + (blen // 4) * sw.SW_BIN_SEQS: sw.SW_BIN_SEQS]
            raw = np.ascontiguousarray(words).view(np.uint8).reshape(-1)  # byte x = position 4q+x
            assert (raw % 8 == 0).all()      # bytes hold 8 x code
            codes = raw // 8
            sid = p["slot_seq"][slot0 + k]
            if sid < 0:
                assert (codes == sw.SW_PAD_CODE).all()
                continue
            n = offsets[sid + 1] - offsets[sid]
            assert (codes[n:] == sw.SW_PAD_CODE).all()
            seqs[int(sid)] = codes[:n].copy()
    return seqs


@pytest.mark.parametrize("t_long", [0, 1, 50, 100, 400, 10**6])
def test_pack_roundtrip(t_long):
    rng = np.random.default_rng(3)
    lengths = np.concatenate([rng.integers(0, 600, 700), [0, 0, 1, 2, 3, 4, 5, 1000, 2500]])
    rng.shuffle(lengths)
    res, offs = _db(lengths)
    p = sw.pack(res, offs, t_long)
    info = p["info"]
    thr = t_long if t_long > 0 else sw.SW_DEFAULT_LONG_THRESHOLD
    assert info["long_threshold"] == thr
    seqs = _unpack(p, offs)
    long_ids = p["long_ids"].tolist()
    vthr = info["very_long_threshold"]
    assert vthr == 4 * thr
    nb = info["n_bins"]
    short_ids = [s for s in p["slot_seq"][:nb * sw.SW_BIN_SEQS].tolist() if s >= 0]
    binned_long = [s for s in p["slot_seq"][nb * sw.SW_BIN_SEQS:].tolist() if s >= 0]
    # every sequence is in exactly one short bin or in the long list
    assert sorted(short_ids + long_ids) == list(range(len(lengths)))
    for sid, codes in seqs.items():
        assert (codes == res[offs[sid]:offs[sid + 1]]).all()
    for sid in short_ids:
        assert lengths[sid] < thr
    for sid in long_ids:
        assert lengths[sid] >= thr
    # the long bins hold exactly the long sequences below the very-long cut
    assert sorted(binned_long) == sorted(s for s in long_ids if lengths[s] < vthr)
    assert info["n_very_long"] == sum(1 for s in long_ids if lengths[s] >= vthr)
    assert long_ids[:info["n_very_long"]] == [s for s in long_ids if lengths[s] >= vthr]
    # long list longest first, ties by index
    ll = [(-lengths[s], s) for s in long_ids]
    assert ll == sorted(ll)
    # bins hold length-sorted slots (stable), bin length = padded first length
    for part in (short_ids, binned_long):
        key = [(-lengths[s], s) for s in part]
        assert key == sorted(key)
    for res_off, rb_off, blen, slot0 in p["bins"]:
        first = p["slot_seq"][slot0]
        assert blen == max(sw.SW_MIN_BIN_LEN, (lengths[first] + 3) // 4 * 4)
    # offsets are cumulative
    bins = p["bins"]
    if len(bins):
        assert bins[0, 0] == 0 and bins[0, 1] == 0
        assert (np.diff(bins[:, 0]) == bins[:-1, 2] // 4 * 128).all()
        assert (np.diff(bins[:, 1]) == bins[:-1, 2] // 4 * 128).all()
        assert info["packed_dwords"] == int((bins[:, 2] // 4 * 128).sum())
        assert info["boundary_bytes"] == int((bins[:, 2] // 4 * 128).sum()) * 16


def test_plan_empty_database():
    info = sw.plan(np.zeros(1, dtype=np.int64))
    assert info["n_bins"] == 0 and info["n_long"] == 0 and info["packed_dwords"] == 0


def test_plan_rejects_bad_input():
    with pytest.raises(sw.SwError) as e:
        sw.plan(np.array([0, 5, 3], dtype=np.int64))
    assert e.value.code == _native.SW_EINVAL
    with pytest.raises(sw.SwError) as e:
        sw.plan(np.array([1, 5], dtype=np.int64))
    assert e.value.code == _native.SW_EINVAL
    with pytest.raises(sw.SwError) as e:
        sw.pack(np.array([0, 24, 1], dtype=np.uint8), np.array([0, 3], dtype=np.int64))
    assert e.value.code == _native.SW_EINVAL
    with pytest.raises(sw.SwError) as e:
        sw.plan(np.array([0, 1 << 24], dtype=np.int64))
    assert e.value.code == _native.SW_ERANGE


def test_workload_layout_padding_is_small():
    w = swinputs.config("plain", scale=0.05)
    info = sw.plan(w.offsets)
    assert info["packed_dwords"] * 4 < 1.05 * w.n_residues + 128 * 32 * info["n_bins"]


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "swdb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w]+\s*\*?\s*(sw_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    syms = _declared_symbols()
    assert len(syms) >= 13, syms
    L = _native.lib()
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(_native.SIGNATURES) == syms


def test_no_device_reports_error_not_crash():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    res, offs = _db([5, 6, 7])
    with pytest.raises(sw.SwError) as e:
        sw.Database(res, offs)
    assert e.value.code == _native.SW_EDEVICE


def test_null_handle_calls_fail_cleanly():
    L = _native.lib()
    m = swinputs.blosum62()
    out = np.zeros(4, dtype=np.int32)
    q = np.zeros(3, dtype=np.uint8)
    assert L.sw_search(None, q.ctypes.data, 3, m.ctypes.data, 10, 2, out.ctypes.data) == _native.SW_EINVAL
    assert L.sw_set_option(None, 1, 1) == _native.SW_EINVAL
    assert L.sw_db_info(None, None, None, None, None) == _native.SW_EINVAL
    L.sw_db_free(None)
    assert b"NULL" in L.sw_last_error()


def test_device_argument_checks_reject_bad_buffers():
    """The binding checks what the C ABI cannot (device buffers' dtype,
    layout, size and location) before any call: every rejection raises
    ValueError (here with host tensors, which fail the last check too)."""
    import torch
    from paper_2203_11100_amd import _check_search_args, _check_batch_args
    q = torch.zeros(10, dtype=torch.uint8)
    out = torch.zeros(100, dtype=torch.int32)
    cases = [
        (lambda: _check_search_args(q.to(torch.int32), out, 100), "torch.uint8"),
        (lambda: _check_search_args(q, out.to(torch.int64), 100), "torch.int32"),
        (lambda: _check_search_args(q, out[:50], 100), "at least 100"),
        (lambda: _check_search_args(q, torch.zeros((100, 2), dtype=torch.int32)[:, 0], 100),
         "contiguous"),
        (lambda: _check_search_args(q, out, 100), "GPU memory"),
        (lambda: _check_batch_args(q, np.array([0, 4, 3]), out, 50), "non-decreasing"),
        (lambda: _check_batch_args(q, np.array([1, 4]), out, 50), "start at 0"),
        (lambda: _check_batch_args(q, np.array([0, 4, 11]), out, 50), "at least 11"),
        (lambda: _check_batch_args(q, np.array([0, 4, 10]), out, 51), "at least 102"),
        (lambda: _check_batch_args(q, np.array([0, 4, 10]), out, 50), "GPU memory"),
        (lambda: _check_search_args(np.zeros(10, np.uint8), out, 100), "torch tensor"),
    ]
    for fn, msg in cases:
        with pytest.raises(ValueError, match=msg):
            fn()
