"""Load-balanced tiling of a count grid (multi-domain runs): the oracle against properties that any
valid tiling has, then the library (C-ABI, host only) against the oracle, tile for tile."""
import numpy as np
import pytest

import paper_1404_2891_amd as fm
from oracle.partition import partition_grid


def check_tiling(tiles, sums, counts, target):
    gx, gy = counts.shape
    owner = -np.ones((gx, gy), dtype=int)
    for t, (ix0, ix1, iy0, iy1) in enumerate(tiles):
        assert 0 <= ix0 < ix1 <= gx and 0 <= iy0 < iy1 <= gy
        assert np.all(owner[ix0:ix1, iy0:iy1] == -1), "tiles overlap"
        owner[ix0:ix1, iy0:iy1] = t
        block = np.maximum(counts[ix0:ix1, iy0:iy1], 0)
        assert abs(block.sum() - sums[t]) < 1e-9 * (1 + block.sum())
        # a tile above target is a single row of its slab (the row alone exceeds it)
        if sums[t] > target + 1e-9:
            assert iy1 - iy0 == 1
    assert np.all(owner >= 0), "tiles do not cover the grid"


@pytest.mark.parametrize("seed", range(12))
def test_oracle_tiles_cover_disjointly_and_balance(seed):
    g = np.random.default_rng(seed)
    gx, gy = g.integers(1, 10, size=2)
    counts = g.gamma(0.7, 3.0, size=(gx, gy)) - (0.3 if seed % 3 == 0 else 0.0)
    target = float(g.uniform(2, 20))
    tiles, sums = partition_grid(counts, target)
    check_tiling(tiles, sums, counts, target)
    total = np.maximum(counts, 0).sum()
    k = min(gx, int(np.ceil(np.sqrt(max(1, np.ceil(total / target))))))
    assert len({(t[0], t[1]) for t in tiles}) == k


def test_oracle_special_cases():
    # uniform counts: equal slabs and equal tiles
    tiles, sums = partition_grid(np.ones((8, 8)), 16.0)
    assert len(tiles) == 4 and all(s == 16.0 for s in sums)
    assert sorted({(t[0], t[1]) for t in tiles}) == [(0, 4), (4, 8)]
    # everything fits one tile
    tiles, sums = partition_grid(np.full((3, 5), 0.5), 100.0)
    assert tiles == [(0, 3, 0, 5)] and sums == [7.5]
    # empty estimates (all <= 0): one tile over the whole grid
    tiles, sums = partition_grid(-np.ones((4, 2)), 5.0)
    assert tiles == [(0, 4, 0, 2)] and sums == [0.0]
    # one heavy cell becomes a row of its own
    c = np.zeros((1, 5))
    c[0, 2] = 50
    c[0, [0, 1, 3, 4]] = 1
    tiles, _ = partition_grid(c, 10.0)
    assert tiles == [(0, 1, 0, 2), (0, 1, 2, 3), (0, 1, 3, 5)]


@pytest.mark.parametrize("seed", range(20))
def test_library_partition_matches_oracle(seed):
    g = np.random.default_rng(100 + seed)
    gx, gy = g.integers(1, 12, size=2)
    counts = g.gamma(0.8, 4.0, size=(gx, gy)) - 0.2
    if seed % 4 == 0:
        counts = np.round(counts)       # integer-valued estimates: ties in the slab choice
    target = float(g.uniform(1, 30))
    tiles, sums = fm.partition_grid(counts, target)
    ot, os_ = partition_grid(counts, target)
    assert [tuple(int(v) for v in t) for t in tiles] == [tuple(t) for t in ot]
    assert np.array_equal(sums, np.array(os_))


def test_library_partition_rejects_bad_arguments():
    import ctypes
    nt = ctypes.c_int(0)
    c = np.ones((2, 2))
    L = fm.lib()
    assert L.feast_partition_grid(0, 2, c.ctypes.data, 1.0, 4, ctypes.byref(nt), None, None) == -1
    assert L.feast_partition_grid(2, 2, c.ctypes.data, 0.0, 4, ctypes.byref(nt), None, None) == -4
    assert L.feast_partition_grid(2, 2, c.ctypes.data, 1.0, 0, ctypes.byref(nt), None, None) == \
        fm.binding.FEAST_EUNSUPPORTED and nt.value == 4
