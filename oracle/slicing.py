"""CPU ORACLE -- TEST INFRASTRUCTURE ONLY.

Slicing plans and index rectification (Kernelet, Section 2.2 "Problem
Definition" and Section 4.1 "Kernel Slicing"):
  * a kernel is k thread blocks with ids 0..k-1;
  * a slice is a contiguous range of block ids; a slicing plan is the
    sequence of slices covering 0..k-1;
  * index rectification: a slice launched with a small grid adds its offset
    to the built-in block index and recovers the block's position in the
    ORIGINAL grid.  Reading for 2-D/3-D grids: row-major linearisation
    id = x + gx (y + gy z).
"""
from __future__ import annotations


def plan(k: int, s: int):
    """Slices [o, o + n) of size s (last one shorter) covering 0..k-1."""
    if s <= 0:
        raise ValueError("slice size must be positive")
    return [(o, min(s, k - o)) for o in range(0, k, s)]


def rectify(offset: int, local: int, grid):
    """Original (x, y, z) block index of local block `local` of the slice
    starting at `offset`, for original grid (gx, gy, gz)."""
    gx, gy, gz = grid
    lin = offset + local
    return lin % gx, (lin // gx) % gy, lin // (gx * gy)


def matrix_add_blocks(n=256, tile=16, slice_blocks=8):
    """The paper's MatrixAdd slicing example: n x n matrices, tile x tile
    threads per block, slices of `slice_blocks` blocks.  Returns the list
    of (row, col) elements written, in launch order."""
    g = n // tile
    out = []
    for off, cnt in plan(g * g, slice_blocks):
        for local in range(cnt):
            bx, by, _ = rectify(off, local, (g, g, 1))
            for ty in range(tile):
                for tx in range(tile):
                    out.append((by * tile + ty, bx * tile + tx))
    return out


# ------------------------------------------------------------- placement
# Slices run as low-occupancy kernels (Section 4.1): a co-schedule of two
# kernels at b1 and b2 blocks per multiprocessor means that at no moment
# does a multiprocessor hold more than b_i blocks of kernel i, and that the
# two kernels share multiprocessors.  These functions read that off a
# record of where and when each workgroup ran: its compute unit and the
# times of its first and last instruction.  Readings: a workgroup occupies
# its CU over the closed interval [t0, t1]; two workgroups whose intervals
# only touch (one's t1 equals the other's t0) do not overlap, since the
# clock ticks far slower than a workgroup hand-over.


def cu_key(hw_id: int, xcc_id: int):
    """A compute unit's identity from the HW_ID and XCC_ID hardware
    registers: (XCC, shader engine, shader array, CU), from XCC_ID bits 3:0
    and HW_ID bits 15:13, 12 and 11:8."""
    return (xcc_id & 0xF, (hw_id >> 13) & 0x7, (hw_id >> 12) & 0x1, (hw_id >> 8) & 0xF)


def max_concurrent(intervals):
    """Largest number of closed intervals [t0, t1] covering one instant,
    ends before starts at equal times (brute force over every start)."""
    best = 0
    for s, _ in intervals:
        # every interval alive at instant s: started at or before s and
        # ending after s (an interval ending exactly at s has left)
        n = sum(1 for a, b in intervals if a <= s and (b > s or (a == s and b == s)))
        best = max(best, n)
    return best


def placement(records):
    """records: iterable of (kernel, cu, t0, t1), one per workgroup.
    Returns {kernel: largest number of its workgroups resident at once on
    any one CU}, and the set of CUs per kernel."""
    by = {}
    for k, cu, t0, t1 in records:
        by.setdefault((k, cu), []).append((t0, t1))
    peak, cus = {}, {}
    for (k, cu), iv in by.items():
        peak[k] = max(peak.get(k, 0), max_concurrent(iv))
        cus.setdefault(k, set()).add(cu)
    return peak, cus


def coresident_cus(records, k1, k2):
    """CUs on which a workgroup of k1 and one of k2 were resident at the same
    instant."""
    by = {}
    for k, cu, t0, t1 in records:
        if k in (k1, k2):
            by.setdefault(cu, {}).setdefault(k, []).append((t0, t1))
    out = set()
    for cu, d in by.items():
        if k1 not in d or k2 not in d:
            continue
        if any(a0 < b1 and b0 < a1 for a0, a1 in d[k1] for b0, b1 in d[k2]):
            out.add(cu)
    return out
