"""Benchmark: GCUPS of Smith-Waterman database search on one MI355X.

One step = the paper's search protocol on the full synthetic stand-in
workload: 20 queries (lengths 144..5478) each searched against the resident
200,000-sequence database (71M residues), BLOSUM62, gaps 10/2, one search
(profile + inter-task + intra-task + rescoring kernels) per query.  GCUPS =
sum over queries of m * N / time (paper section 4.2).  This plain form is the
headline `value`.

Beside it, on the same resident database:
  batched : the 20 queries + 200 of length U[50, 5000] in one batched search
            (paired-query persistent kernel, replayed from a HIP graph)
  served  : Poisson arrivals (50 QPS, lengths log-normal, median 400) through
            the continuous-batching server; p50/p99 latency and GCUPS, and a
            sweep over 10, 25 and 75 QPS plus a saturation point (capacity)
  per_query, host_roundtrip : GCUPS of each query alone; the step through
            host buffers (query upload and score download included)
  topk, modes : top-k hits with alignment ends; global / semi-global scores
  plain_small, long_mix : the small configuration's latency; the long-sequence
            mix (10 queries of 1,000..10,000 vs 50,000 sequences, 2% long)

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--no-batched] [--no-served] [--requests N] [--qps Q]

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GCUPS on 1 MI355X (plain vs batched/served) + p50/p99 query latency"
# HBM traffic of the inter-task kernel on this workload, from rocprofv3
# --pmc FETCH_SIZE and WRITE_SIZE passes over one step's 20 launches (the
# counter summary in profiles/ gives the commands and per-launch values),
# converted to bytes with the counters' readings for a 1 GiB device copy.
# Valid only for the kernel and schedule-selection code it was taken on: bench
# reports null when the digest of that code (comments removed) differs.
TRAFFIC = {"bytes_per_launch": 2.2661e+10, "fetch_bytes": 57.47e9, "write_bytes": 395.74e9,
           "launches": 20, "sources_sha256": "a249759c32e92080bf266af662cbc83bbeded4f712924ea5003a8c8b2876af53"}
TRAFFIC_SOURCES = ("k_inter.hip", "packed16.h", "internal.h", "runtime.hip")
# of runtime.hip only the schedule selection (the fitted tables and the
# choice of rows and waves per query) shapes the inter-task kernel's traffic
SCHEDULE_SECTION = ("constexpr int kDefaultRows", "enum TimedKind")
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2 halves of a packed 16-bit
# instruction x 2.4 GHz = 78.64 T packed 16-bit lane-ops/s
PEAK_HALF_TOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Algorithmic integer operations per cell of Gotoh's recurrence: 1 add
# (H_diag + S), 3 max (E, F, 0), 1 max (running best), 1 subtract (H - open),
# 2 subtract (E - extend, F - extend), 2 max (new E, new F).  The roofline
# fraction `frac` counts these 10 per cell against the packed 16-bit peak.
OPS_PER_CELL = 10
# Packed binary16 instructions the inter-task kernel issues per cell (half-ops
# per cell): 1 fused multiply-add forming H_diag + S for both halves (the
# profile dwords hold (S, 1) and (1, S)), 3 subtract and 3 three-input max for
# the cell, 1/2 three-input max for the running maximum (two rows per op).  A
# three-input max does two of the 10 algorithmic maxima in one issue slot, so
# 10 ops take 7.5 slots and `frac` can exceed 1; `frac_issue` is the fraction
# of the issue slots the kernel's own instruction count needs.
ISSUE_PER_CELL = 7.5


def code_text(src):
    """C++ source without comments, trailing blanks or blank lines (string
    literals in these sources hold no comment markers)."""
    import re
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(ln.rstrip() for ln in src.splitlines() if ln.strip())


def sources_digest(read=None):
    """sha256 over the code (not the comments) of the inter-task kernel, its
    headers and the schedule selection; `read(name)` returns a source's
    text."""
    import hashlib
    if read is None:
        def read(name):
            with open(os.path.join(ROOT, "paper_2203_11100_amd", "csrc", name)) as f:
                return f.read()
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        text = read(name)
        if name == "runtime.hip":
            a, b = text.find(SCHEDULE_SECTION[0]), text.find(SCHEDULE_SECTION[1])
            text = text[a:b] if 0 <= a < b else text
        h.update(code_text(text).encode())
    return h.hexdigest()


def measured_traffic():
    """Counter-measured bytes per launch, or None when the kernel changed."""
    t = TRAFFIC
    if sources_digest() != t["sources_sha256"]:
        return None
    return t["bytes_per_launch"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, fraction=0.02, seed=0):
    """The CPU oracle on a seeded sample of the same workload: every query
    against a random `fraction` of the database sequences."""
    import numpy as np
    import oracle.cpu as ocpu
    rng = np.random.default_rng(seed)
    ids = np.sort(rng.choice(w.n_seqs, max(1, int(w.n_seqs * fraction)), replace=False))
    lens = np.diff(w.offsets)
    res_sample = int(lens[ids].sum())
    threads = ocpu.default_threads()
    cells = 0
    t0 = time.perf_counter()
    for q in w.queries:
        ocpu.search(q, w.residues, w.offsets, w.matrix, w.gap_open, w.gap_extend, ids=ids,
                    threads=threads)
        cells += len(q) * res_sample
    dt = time.perf_counter() - t0
    return {"value": cells / dt / 1e9, "unit": "GCUPS", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": "all %d queries x %d random sequences (%.1f%% of the database, %d "
                      "residues, seed %d); %.1f s" % (len(w.queries), len(ids), 100 * fraction,
                                                      res_sample, seed, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--requests", type=int, default=1000)
    ap.add_argument("--qps", type=float, default=50.0)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the top-k, modes, small and long-mix legs")
    ap.add_argument("--batch-replays", type=int, default=3)
    ap.add_argument("--sweep-requests", type=int, default=400)
    ap.add_argument("--scale", type=float, default=1.0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the search shards by database bins with no "
              "collective on the hot path, and this build runs and reports the single-GPU "
              "share (--gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2203_11100_amd as sw
    import swinputs

    log("generating workload ...")
    w = swinputs.config("plain", scale=args.scale)
    cells_step = w.cells()
    log("workload: %d queries, %d sequences, %d residues, %.3e cells/step"
        % (len(w.queries), w.n_seqs, w.n_residues, cells_step))
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    db = sw.Database(w.residues, w.offsets)
    log("database loaded in %.2f s: %s" % (time.perf_counter() - t0, db.info()))
    d_queries = [torch.from_numpy(q).cuda() for q in w.queries]
    d_outs = [torch.empty(db.n_seqs, dtype=torch.int32, device="cuda") for _ in w.queries]
    stream = torch.cuda.current_stream()

    def step():
        for dq, do in zip(d_queries, d_outs):
            db.search_async(dq, w.matrix, w.gap_open, w.gap_extend, do, stream)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log("warmup step %d done" % i)
    db.stats()                                   # reset counters
    db.set_option(sw.SW_OPT_TIMING, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = db.stats()
    db.set_option(sw.SW_OPT_TIMING, 0)
    log("timed %d steps in %.3f s; kernel stats %s" % (args.steps, dt, st))

    gcups = cells_step * args.steps / dt / 1e9
    n_launch = max(st["n_inter_launches"], 1)
    inter_s = st["ms_inter"] / 1e3
    achieved = st["inter_cells"] * OPS_PER_CELL / inter_s / 1e12 if inter_s > 0 else None
    issued = st["inter_cells"] * ISSUE_PER_CELL / inter_s / 1e12 if inter_s > 0 else None
    roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_HALF_TOPS, "unit": "Tops/s",
            "frac": (achieved / PEAK_HALF_TOPS) if achieved else None,
            "frac_issue": (issued / PEAK_HALF_TOPS) if issued else None,
            "ops_per_cell": OPS_PER_CELL, "issue_per_cell": ISSUE_PER_CELL,
            "traffic": measured_traffic(),
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, mean over the "
                            "step's 20 launches)",
            "kernel": "k_inter_f16 (rows, waves fitted per query; last query: %d, %d)"
                      % (st["rows"], st["waves"]),
            "avg_launch_ms": st["ms_inter"] / n_launch}
    result = {
        "metric": METRIC, "value": gcups, "unit": "GCUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f16+int32", "data": "synthetic",
        "config": {"workload": "plain: 20 queries (144..5478 residues) vs %d synthetic "
                               "sequences (%d residues), BLOSUM62, gaps 10/2, one search per "
                               "query" % (w.n_seqs, w.n_residues),
                   "n_queries": len(w.queries), "n_seqs": w.n_seqs,
                   "n_residues": w.n_residues, "cells_per_step": cells_step,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "kernel_ms_per_step": {k: st[k] / args.steps for k in
                               ("ms_inter", "ms_intra", "ms_rescore")},
    }
    result["per_query"] = per_query_leg(db, w, d_queries, d_outs)
    result["host_roundtrip"] = host_roundtrip_leg(db, w)
    if not args.no_extra:
        result["hybrid"] = hybrid_leg(db, w, result["host_roundtrip"])
    if not args.no_extra:
        result["topk"] = topk_leg(db, w)
        result["modes"] = modes_leg(db, w)
    if not args.no_batched:
        result["batched"] = batched_leg(db, args.scale, args.batch_replays)
    if not args.no_served:
        result["served"] = served_leg(db, args.scale, args.requests, args.qps)
        if not args.no_sweep:
            result["served_sweep"] = served_sweep(db, args.scale, args.sweep_requests)
    del d_outs
    db.close()
    if not args.no_extra:
        result["plain_small"] = plain_small_leg()
        result["long_mix"] = long_mix_leg(args.scale)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample ...")
        result["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(result), flush=True)


def _event_ms(fn, stream=None):
    """Runs fn() between two HIP events on the current stream; returns ms."""
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b)


def per_query_leg(db, w, d_queries, d_outs):
    """GCUPS of each plain query searched alone (device-resident buffers,
    HIP events on the search's stream): GCUPS against query length."""
    rows = []
    for q, dq, do in zip(w.queries, d_queries, d_outs):
        ms = min(_event_ms(lambda: db.search_async(dq, w.matrix, w.gap_open, w.gap_extend, do))
                 for _ in range(2))
        rows.append({"m": len(q), "ms": ms, "gcups": len(q) * w.n_residues / ms / 1e6})
    log("per query: %s" % ", ".join("%d:%.0f" % (r["m"], r["gcups"]) for r in rows))
    return rows


def host_roundtrip_leg(db, w, steps=2):
    """The plain step through the host-buffer call sw_search: each query is
    uploaded and its 800 KB of scores downloaded inside the timed region."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for q in w.queries:
            db.search(q, w.matrix, w.gap_open, w.gap_extend)
    dt = (time.perf_counter() - t0) / steps
    log("host round trip: %.1f ms per step" % (dt * 1e3))
    return {"value": w.cells() / dt / 1e9, "unit": "GCUPS", "ms_per_step": dt * 1e3,
            "form": "sw_search per query: query H2D, search, scores D2H, synchronous"}


def hybrid_leg(db, w, host_rt, steps=2):
    """The plain step through sw_search_hybrid (host cores take bins from the
    back of the work order while the GPU takes chunks from the front),
    against the same step through the GPU-only host-buffer call."""
    totals = {"gpu_cells": 0, "cpu_cells": 0, "cpu_seqs": 0, "gpu_bins": 0}
    threads = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        for q in w.queries:
            _, st = db.search_hybrid(q, w.matrix, w.gap_open, w.gap_extend)
            for k in totals:
                totals[k] += st[k]
            threads = st["cpu_threads"]
    dt = (time.perf_counter() - t0) / steps
    r = {"value": w.cells() / dt / 1e9, "unit": "GCUPS", "ms_per_step": dt * 1e3,
         "gpu_only_ms_per_step": host_rt["ms_per_step"],
         "step_time_change": dt * 1e3 / host_rt["ms_per_step"] - 1.0,
         "cpu_threads": threads,
         "cpu_cell_share": totals["cpu_cells"] / max(1, totals["cpu_cells"] + totals["gpu_cells"]),
         "cpu_seqs_per_step": totals["cpu_seqs"] / steps,
         "gpu_bins_per_step": totals["gpu_bins"] / steps,
         "form": "sw_search_hybrid per query (host buffers), vs sw_search per query"}
    log("hybrid: %s" % r)
    return r


def topk_leg(db, w, k=1000, queries=(0, 8, 19)):
    """The top-k hits with alignment ends (sw_search_topk_async) against the
    plain search of the same query: the extra time of the selection and the
    exact end-coordinate pass over the k hits; then the alignments of the 10
    best (sw_traceback, host call: codes on the device, walks on the host)."""
    import torch
    out = []
    for qi in queries:
        q = w.queries[qi]
        dq = torch.from_numpy(q).cuda()
        d_out = torch.empty(db.n_seqs, dtype=torch.int32, device="cuda")
        d_hits = torch.empty((k, 4), dtype=torch.int32, device="cuda")
        base = min(_event_ms(lambda: db.search_async(dq, w.matrix, 10, 2, d_out))
                   for _ in range(3))
        with_k = min(_event_ms(lambda: db.search_topk_async(dq, w.matrix, 10, 2, k, d_out,
                                                            d_hits)) for _ in range(3))
        torch.cuda.synchronize()
        best = d_hits[:10, 0].cpu().numpy()
        tb = []
        for _ in range(3):
            t0 = time.perf_counter()
            als = db.traceback(q, w.matrix, 10, 2, best)
            tb.append((time.perf_counter() - t0) * 1e3)
        out.append({"m": len(q), "k": k, "search_ms": base, "topk_ms": with_k,
                    "extra_ms": with_k - base, "traceback_10_ms": min(tb),
                    "traceback_10_cells": int(len(q) * sum(int(w.offsets[s + 1] - w.offsets[s])
                                                         for s in best)),
                    "traceback_10_ops": int(sum(len(a["ops"]) for a in als))})
    log("top-k: %s" % out)
    return out


# int32 operations per cell of the global / semi-global recurrence (no floor,
# no running maximum): 1 add, 2 max for H, 1 subtract for the open, 2
# subtract for the extends, 2 max for E and F
MODE_OPS_PER_CELL = 8
# MI355X unpacked 32-bit VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
PEAK_I32_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


def modes_leg(db, w, queries=(0, 8, 14)):
    """Global and semi-global searches (int32 kernels) of three plain queries."""
    import torch
    import paper_2203_11100_amd as sw
    out = {}
    for mode in ("global", "semiglobal"):
        cells, ms_tot, inter_ms, inter_cells = 0, 0.0, 0.0, 0
        for qi in queries:
            q = w.queries[qi]
            dq = torch.from_numpy(q).cuda()
            d_out = torch.empty(db.n_seqs, dtype=torch.int32, device="cuda")
            db.search_mode_async(dq, w.matrix, 10, 2, mode, d_out)      # warm
            torch.cuda.synchronize()
            db.stats()
            db.set_option(sw.SW_OPT_TIMING, 1)
            ms_tot += _event_ms(lambda: db.search_mode_async(dq, w.matrix, 10, 2, mode, d_out))
            st = db.stats()
            db.set_option(sw.SW_OPT_TIMING, 0)
            inter_ms += st["ms_inter"]
            inter_cells += st["inter_cells"]
            cells += len(q) * w.n_residues
        achieved = inter_cells * MODE_OPS_PER_CELL / (inter_ms / 1e3) / 1e12 if inter_ms else None
        out[mode] = {"gcups": cells / ms_tot / 1e6, "ms": ms_tot,
                     "queries": [len(w.queries[i]) for i in queries],
                     "roofline": {"bound": "alu", "kernel": "k_mode_inter", "achieved": achieved,
                                  "peak": PEAK_I32_TOPS, "unit": "Tops/s (int32)",
                                  "frac": achieved / PEAK_I32_TOPS if achieved else None,
                                  "ops_per_cell": MODE_OPS_PER_CELL}}
    log("modes: %s" % out)
    return out


def plain_small_leg(reps=50):
    """The small plain configuration (1 query of 144 residues vs 2,000
    sequences): per-search latency, device-resident and through host buffers."""
    import numpy as np
    import torch
    import paper_2203_11100_amd as sw
    import swinputs
    w = swinputs.config("plain-small")
    q = w.queries[0]
    with sw.Database(w.residues, w.offsets) as db:
        dq = torch.from_numpy(q).cuda()
        d_out = torch.empty(db.n_seqs, dtype=torch.int32, device="cuda")
        for _ in range(3):
            db.search_async(dq, w.matrix, 10, 2, d_out)
        torch.cuda.synchronize()
        dev = [_event_ms(lambda: db.search_async(dq, w.matrix, 10, 2, d_out))
               for _ in range(reps)]
        host = []
        for _ in range(reps):
            t0 = time.perf_counter()
            db.search(q, w.matrix, 10, 2)
            host.append((time.perf_counter() - t0) * 1e3)
    r = {"p50_ms": float(np.percentile(dev, 50)), "p99_ms": float(np.percentile(dev, 99)),
         "host_p50_ms": float(np.percentile(host, 50)),
         "host_p99_ms": float(np.percentile(host, 99)),
         "gcups": len(q) * w.n_residues / float(np.percentile(dev, 50)) / 1e6,
         "workload": w.recipe}
    log("plain-small: %s" % r)
    return r


def long_mix_leg(scale, steps=2):
    """The long-sequence mix: 10 queries (1,000..10,000) vs 50,000 sequences
    of which 1,000 are 10,000..35,000 long, single searches and one batch."""
    import numpy as np
    import torch
    import paper_2203_11100_amd as sw
    import swinputs
    w = swinputs.config("long-mix", scale=scale)
    cells = w.cells()
    with sw.Database(w.residues, w.offsets) as db:
        dqs = [torch.from_numpy(q).cuda() for q in w.queries]
        outs = [torch.empty(db.n_seqs, dtype=torch.int32, device="cuda") for _ in w.queries]

        def step():
            for dq, do in zip(dqs, outs):
                db.search_async(dq, w.matrix, 10, 2, do)
        step()
        torch.cuda.synchronize()
        db.stats()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        st = db.stats()
        n_rescored = int(st["n_rescored"])
        cat = torch.from_numpy(np.concatenate(w.queries)).cuda()
        qoffs = np.zeros(len(w.queries) + 1, np.int64)
        np.cumsum([len(q) for q in w.queries], out=qoffs[1:])
        bout = torch.empty((len(w.queries), db.n_seqs), dtype=torch.int32, device="cuda")
        db.search_batch_async(cat, qoffs, w.matrix, 10, 2, bout)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        db.search_batch_async(cat, qoffs, w.matrix, 10, 2, bout)
        torch.cuda.synchronize()
        dtb = time.perf_counter() - t0
        planted = bout[len(w.queries) - 1][torch.from_numpy(w.planted).cuda()].cpu().numpy()
    r = {"value": cells / dt / 1e9, "unit": "GCUPS", "ms_per_step": dt * 1e3,
         "batched_gcups": cells / dtb / 1e9, "batched_ms": dtb * 1e3, "cells": cells,
         "n_rescored_last_query": n_rescored, "planted_scores": [int(x) for x in planted],
         "workload": w.recipe}
    log("long mix: %s" % r)
    return r


def batched_leg(db, scale, replays=3):
    """220 queries in one batched search, first with the schedule fitted to
    the pairs, then with the one the autotuner picks for these query
    lengths; each form's first call plans and captures the graph (untimed),
    then the mean of `replays` timed replays."""
    import numpy as np
    import torch
    import swinputs
    wb = swinputs.config("batched", scale=scale)
    cells = wb.cells()
    log("batched: %d queries, %.3e cells" % (len(wb.queries), cells))
    cat = torch.from_numpy(np.concatenate(wb.queries)).cuda()
    qoffs = np.zeros(len(wb.queries) + 1, np.int64)
    np.cumsum([len(q) for q in wb.queries], out=qoffs[1:])
    out = torch.empty((len(wb.queries), db.n_seqs), dtype=torch.int32, device="cuda")

    def timed():
        db.search_batch_async(cat, qoffs, wb.matrix, wb.gap_open, wb.gap_extend, out)
        torch.cuda.synchronize()
        times = []
        for _ in range(max(1, replays)):
            t0 = time.perf_counter()
            db.search_batch_async(cat, qoffs, wb.matrix, wb.gap_open, wb.gap_extend, out)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        return sum(times) / len(times), times

    dt_fit, times_fit = timed()
    log("batched (fitted): %.3f s, %.0f GCUPS" % (dt_fit, cells / dt_fit / 1e9))
    t0 = time.perf_counter()
    rep = db.autotune([len(q) for q in wb.queries])
    tune_s = time.perf_counter() - t0
    dt, times = timed()
    db.autotune([0])                  # back to the fitted schedules for the other legs
    db.stats()
    del out
    log("batched (autotuned in %.1f s): %.3f s mean of %d replays, %.0f GCUPS"
        % (tune_s, dt, len(times), cells / dt / 1e9))
    return {"value": cells / dt / 1e9, "unit": "GCUPS", "ms_per_step": dt * 1e3,
            "replays_ms": [t * 1e3 for t in times],
            "fitted": {"value": cells / dt_fit / 1e9, "ms_per_step": dt_fit * 1e3,
                       "replays_ms": [t * 1e3 for t in times_fit]},
            "autotune": {"seconds": tune_s,
                         "buckets": [{"query_len": b["query_len"], "batch_chosen": b["batch_chosen"],
                                      "batch_gcups": b["batch_gcups"]}
                                     for b in rep["buckets"]]},
            "n_queries": len(wb.queries), "cells_per_step": cells,
            "form": "one batched search (paired queries, persistent kernel, HIP graph replay) "
                    "with the autotuned schedule, mean of %d replays; `fitted` is the same with "
                    "the schedule fitted to the pairs" % len(times)}


def served_leg(db, scale, n_requests, qps, slots=4, max_batch=16, timeout_s=None):
    import numpy as np
    import swinputs
    from paper_2203_11100_amd import serve
    ws = swinputs.config("served", scale=scale, n_requests=n_requests, qps=qps)
    srv = serve.Server(db, ws.matrix, ws.gap_open, ws.gap_extend, max_slots=slots,
                       max_batch=max_batch, request_timeout=timeout_s)
    srv.ex.warm(5000)
    log("served: %d requests at %.0f QPS on %d slots ..." % (n_requests, qps, srv.n_slots))
    reqs = srv.run(ws.queries, ws.arrivals)
    srv.close()
    s = serve.summarize(reqs, ws.n_residues)
    log("served: %s" % s)
    s.update({"qps": qps, "slots": srv.n_slots, "max_batch": max_batch, "unit_latency": "ms",
              "request_memory_bytes": srv.request_memory, "peak_request_bytes": srv.peak_bytes,
              "timeout_s": timeout_s,
              "arrivals": "Poisson, query lengths log-normal (median 400, sigma 0.8, "
                          "clip 30..5000)"})
    return s


def served_sweep(db, scale, n_requests, qps_points=(10, 25, 75), saturate=400.0):
    """The served form at the other offered loads, and a saturation point
    (arrivals far faster than the device) whose GCUPS is the capacity."""
    out = []
    for qps in list(qps_points) + [saturate]:
        s = served_leg(db, scale, n_requests, qps)
        out.append({k: s.get(k) for k in ("qps", "requests", "served", "p50_ms", "p99_ms",
                                          "gcups", "mean_batch", "slots")})
    return out


if __name__ == "__main__":
    main()
