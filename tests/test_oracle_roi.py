"""Oracle ROI selection (Sec. 3.3, flexible scientific workflow) against an
independent numpy computation on the oracle's own progressive decode: per-block
or per-slice maximum / value range, threshold or top fraction."""
import math

import numpy as np
import pytest

from paper_2509_01626_amd import fields


def _brute(grid, s, B, unit, stat):
    """Statistic per unit from the level grid `grid` (stride s)."""
    nz, ny, nx = grid.shape
    if unit == 0:
        # full-resolution block of a grid point = (index * s) // B
        bz = (np.arange(nz) * s) // B
        by = (np.arange(ny) * s) // B
        bx = (np.arange(nx) * s) // B
        nb = (bz[-1] + 1, by[-1] + 1, bx[-1] + 1)
        out = []
        for i in range(nb[0]):
            for j in range(nb[1]):
                for k in range(nb[2]):
                    sub = grid[np.ix_(bz == i, by == j, bx == k)].astype(np.float64)
                    out.append(sub.max() if stat == 0 else sub.max() - sub.min())
        return np.array(out)
    ax = unit - 1
    g = np.moveaxis(grid.astype(np.float64), ax, 0).reshape(grid.shape[ax], -1)
    return g.max(axis=1) if stat == 0 else g.max(axis=1) - g.min(axis=1)


def _select(st, rule, value):
    if rule == 0:
        return np.nonzero(st > value)[0]
    k = min(len(st), math.ceil(value * len(st)))
    order = sorted(range(len(st)), key=lambda u: (-st[u], u))
    return np.array(sorted(order[:k]))


@pytest.mark.parametrize("unit", [0, 1, 2, 3])
@pytest.mark.parametrize("stat", [0, 1])
def test_roi_matches_numpy(oracle, unit, stat):
    x = fields.bumps((45, 38, 52), seed=31, n_bumps=10)
    comp = oracle.compress(x, oracle.EB_REL, 1e-3, oracle.config(block=8))
    inf = oracle.info(comp)
    for level in (1, inf.levels):
        s = 1 << (inf.levels - level)
        grid = oracle.decompress_level(comp, level)
        want_stats = _brute(grid, s, inf.block, unit, stat)
        for rule, value in ((0, float(np.median(want_stats))), (1, 0.1), (1, 1.0)):
            sel, st = oracle.roi_select(comp, level, unit, stat, rule, value)
            assert np.array_equal(st, want_stats), (unit, stat, level)
            assert np.array_equal(sel, _select(want_stats, rule, value)), (unit, stat, level, rule)


def test_roi_top_fraction_ties_prefer_low_index(oracle):
    x = np.zeros((16, 16, 16), dtype=np.float32)   # every block has the same max
    comp = oracle.compress(x, oracle.EB_ABS, 0.1, oracle.config(block=4))
    sel, st = oracle.roi_select(comp, 2, 0, 0, 1, 0.25)
    assert list(sel) == list(range(16))            # 64 blocks, top 16 by index
    assert np.all(st == 0.0)


def test_roi_finds_the_planted_peak(oracle):
    x = fields.bumps((32, 32, 32), seed=3, n_bumps=4) * 0.01
    x[20, 9, 27] = 50.0                            # one extreme value (block (5, 2, 6))
    comp = oracle.compress(x, oracle.EB_REL, 1e-4, oracle.config(block=4))
    inf = oracle.info(comp)
    sel, _ = oracle.roi_select(comp, inf.levels, 0, 0, 0, 25.0)
    assert list(sel) == [(5 * 8 + 2) * 8 + 6]
