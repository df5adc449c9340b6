"""Workload driver for hardware-counter runs (rocprofv3 --pmc).

Runs, in one process:
  1. a plain device-to-device copy of COPY_MIB MiB (torch), the calibration
     kernel of known traffic: COPY_MIB MiB read and COPY_MIB MiB written;
  2. a benchmark workload's searches for the chosen queries (default: all;
     --workload plain, the 20-query plain workload, long-mix, its 10
     queries against the long-sequence mix, or plain-small, one 144-residue
     query against 2,000 sequences), with the database already
     resident; with --long-only, the plain queries against a database of only
     the plain database's long sequences (2,048 residues or more), so the
     long-sequence kernel runs alone.  --timing adds each search's kernel
     times (HIP events) to the printed record.  --mode global or semiglobal
     runs those alignment modes' searches instead of local ones.

Under `rocprofv3 --pmc FETCH_SIZE` (then `--pmc WRITE_SIZE`, one counter
block per run) each dispatch gets its counter value; dividing a search
kernel's value by the copy kernel's value per MiB converts it into bytes.

    python pmc.py [--workload plain|long-mix|plain-small] [--queries 0,19] [--copy-mib 1024]
                  [--long-only] [--repeat N] [--timing] [--mode local|global|semiglobal]
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

COPY_MIB = 1024


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--queries", default="all")
    ap.add_argument("--copy-mib", type=int, default=COPY_MIB)
    ap.add_argument("--long-only", action="store_true")
    ap.add_argument("--repeat", type=int, default=1)
    ap.add_argument("--workload", default="plain", choices=("plain", "long-mix", "plain-small"))
    ap.add_argument("--timing", action="store_true")
    ap.add_argument("--mode", default="local", choices=("local", "global", "semiglobal"))
    args = ap.parse_args()
    import numpy as np
    import torch
    import paper_2203_11100_amd as sw
    import swinputs

    n = args.copy_mib << 20
    a = torch.ones(n // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    w = swinputs.config(args.workload)
    idx = range(len(w.queries)) if args.queries == "all" else [int(x) for x in args.queries.split(",")]
    res, offs = w.residues, w.offsets
    if args.long_only:
        lens = np.diff(offs)
        keep = np.nonzero(lens >= sw.SW_DEFAULT_LONG_THRESHOLD)[0]
        res = np.concatenate([res[offs[i]:offs[i + 1]] for i in keep])
        offs = np.zeros(len(keep) + 1, np.int64)
        np.cumsum(lens[keep], out=offs[1:])
    with sw.Database(res, offs) as db:
        if args.timing:
            db.set_option(sw.SW_OPT_TIMING, 1)
        out = torch.empty(db.n_seqs, dtype=torch.int32, device="cuda")
        info = []
        for _ in range(args.repeat):
            for i in idx:
                q = torch.from_numpy(w.queries[i]).cuda()
                if args.mode == "local":
                    db.search_async(q, w.matrix, w.gap_open, w.gap_extend, out)
                else:
                    db.search_mode_async(q, w.matrix, w.gap_open, w.gap_extend, args.mode, out)
                torch.cuda.synchronize()
                st = db.stats()
                info.append({"query": i, "m": len(w.queries[i]), "inter_cells": st["inter_cells"],
                             "intra_cells": st["intra_cells"], "long_items": st["long_items"],
                             "long_overlap": st["long_overlap"], "rows": st["rows"],
                             "waves": st["waves"]})
                if args.timing:
                    info[-1].update({k: round(float(st[k]), 3) for k in
                                     ("ms_total", "ms_inter", "ms_intra", "ms_rescore")})
    print(json.dumps({"copy_mib": args.copy_mib, "workload": args.workload, "mode": args.mode,
                      "long_only": args.long_only,
                      "n_seqs": int(len(offs) - 1), "n_residues": int(offs[-1]),
                      "searches": info}), flush=True)


if __name__ == "__main__":
    main()
