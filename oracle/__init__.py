"""CPU oracle for Smith-Waterman/Gotoh database search scores.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only the test suite, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code, tables or helpers with the GPU
path.

What it computes (paper section 2.2: Smith-Waterman local alignment by
dynamic programming; section 4.1: BLOSUM62 with gap penalties 10(2)): for a
query a and each database sequence b, the best local alignment score

    SW(a, b) = max(0, max over chains of matched pairs
                         sum S(a_i, b_j) - sum of gap costs),
    gap cost w(k) = o + (k - 1) * e  for a gap of k >= 1 residues.

The end of the best alignment (search tools report where a hit lies) is
the last matched pair of an optimal chain; of several, the smallest in
database-then-query order, as 0-based residue indices ((-1, -1) for a
score of 0): sw_bruteforce_end, sw_gotoh_end and cpu.score_end/search_end.

Two other alignment modes of the same scoring scheme, global (every
residue of both sequences aligned, end gaps charged) and semi-global (the
whole query aligned inside the database sequence, whose overhangs are free),
are maxima over chains with different end costs and no floor at 0:
sw_bruteforce_mode, sw_gotoh_mode and cpu.score_mode/search_mode.

The alignment itself (an M/I/D string placed at its first residues, scored
by alignment_score from the same definition) is recovered by walking the
H/E/F tables back from that end: sw_gotoh_traceback.

Three implementations, each written from that definition:
  * sw_bruteforce  - enumerates every chain (tiny inputs only);
  * sw_gotoh       - Gotoh's H/E/F recurrence in plain Python;
  * cpu.search     - the same recurrence in plain scalar C (oracle/sw_oracle.c),
                     threaded over database sequences; the timed CPU baseline
                     and the parity source for full-size workloads.
"""
from .sw_ref import (GLOBAL, SEMIGLOBAL, alignment_score, gap_cost, sw_bruteforce,
                     sw_bruteforce_end, sw_bruteforce_mode, sw_bruteforce_table, sw_gotoh,
                     sw_gotoh_end, sw_gotoh_mode, sw_gotoh_traceback)

__all__ = ["GLOBAL", "SEMIGLOBAL", "alignment_score", "gap_cost", "sw_bruteforce",
           "sw_bruteforce_end", "sw_bruteforce_mode", "sw_bruteforce_table", "sw_gotoh",
           "sw_gotoh_end", "sw_gotoh_mode", "sw_gotoh_traceback"]
