"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

Co-schedule pruning by PUR / MUR (Kernelet, Section 4.3 "Co-scheduling
Space Pruning"):
  PUR = instructions executed / (time * frequency * peak IPC)
  MUR = (DRAM reads + DRAM writes) / (time * frequency * peak memory
        requests per cycle)
A pair of kernels is not promising when the two have close PUR and close
MUR.  Reading: a pair is pruned when |dPUR| < alpha_p AND |dMUR| < alpha_m
(strict).  The sentence in Section 4.3 says "or", but the pruned-pair counts
of the paper's C2050 table (tb:pruningTableC2050) are reproduced by "and"
and not by "or" (the tests pin this).  When every pair is pruned, both
thresholds are halved (up to four times) and after that every pair is kept.
"""
from __future__ import annotations

import itertools


def pur(instructions, time_s, freq_hz, peak_ipc):
    return instructions / (time_s * freq_hz * peak_ipc)


def mur(dram_reads, dram_writes, time_s, freq_hz, peak_mpc):
    return (dram_reads + dram_writes) / (time_s * freq_hz * peak_mpc)


def pruned(a, b, alpha_p, alpha_m):
    """a, b: (PUR, MUR).  True when the pair is pruned."""
    return abs(a[0] - b[0]) < alpha_p and abs(a[1] - b[1]) < alpha_m


def count_pruned(chars, alpha_p, alpha_m):
    """Number of the C(n,2) pairs pruned (chars: list of (PUR, MUR))."""
    return sum(pruned(a, b, alpha_p, alpha_m)
               for a, b in itertools.combinations(chars, 2))


def surviving_pairs(chars, alpha_p, alpha_m, max_relax=4):
    """Indices (i, j), i < j, of the pairs kept; relax when none survive."""
    pairs = list(itertools.combinations(range(len(chars)), 2))
    ap, am = alpha_p, alpha_m
    for _ in range(max_relax + 1):
        keep = [(i, j) for i, j in pairs
                if not pruned(chars[i], chars[j], ap, am)]
        if keep or not pairs:
            return keep
        ap, am = ap / 2.0, am / 2.0
    return pairs
