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
