"""Load-balanced tiling of a grid of eigenvalue-count estimates.  Test infrastructure only.

Section 6 names several search domains of one problem as the outermost level of parallelism and
load balance -- subdomains with about the same number of eigenvalues -- as the open problem; it
gives no algorithm.  This is the plain statement of the one the library uses (cells of a gx x gy
grid, counts[ix, iy]; negative estimates count as zero):

1. total = sum of the counts; T = max(1, ceil(total / target)) tiles are aimed at, in
   k = min(gx, ceil(sqrt(T))) vertical slabs.
2. Slab boundary i (1 <= i < k) is the column edge b in [b_(i-1) + 1, gx - (k - i)] whose prefix
   count (sum over columns < b) is closest to i * total / k, the smaller b on ties; b_0 = 0,
   b_k = gx.
3. Each slab is cut bottom to top: a tile grows row by row and is closed before a row that would
   take a nonempty tile above target.

Tiles are listed slab by slab, bottom to top, as (ix0, ix1, iy0, iy1) half-open cell ranges, with
their summed counts.
"""
from __future__ import annotations

import math

import numpy as np


def partition_grid(counts, target):
    c = np.maximum(np.asarray(counts, dtype=np.float64), 0.0)
    gx, gy = c.shape
    # column totals, then running sums over the columns (sums taken left to right, bottom to top)
    col = []
    for ix in range(gx):
        t = 0.0
        for iy in range(gy):
            t += float(c[ix, iy])
        col.append(t)
    run = [0.0]
    for ix in range(gx):
        run.append(run[-1] + col[ix])
    total = run[gx]
    T = max(1, math.ceil(total / target))
    k = min(gx, max(1, math.ceil(math.sqrt(T))))

    def prefix(b):
        return run[b]

    bounds = [0]
    for i in range(1, k):
        goal = total * i / k
        cands = range(bounds[-1] + 1, gx - (k - i) + 1)
        bounds.append(min(cands, key=lambda e: (abs(prefix(e) - goal), e)))
    bounds.append(gx)
    tiles, sums = [], []
    for i in range(k):
        lo, hi = bounds[i], bounds[i + 1]
        start, acc = 0, 0.0
        for iy in range(gy):
            row = 0.0
            for ix in range(lo, hi):
                row += float(c[ix, iy])
            if iy > start and acc > 0 and acc + row > target:
                tiles.append((lo, hi, start, iy))
                sums.append(acc)
                start, acc = iy, 0.0
            acc += row
        tiles.append((lo, hi, start, gy))
        sums.append(acc)
    return tiles, sums
