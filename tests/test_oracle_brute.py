"""The oracle's level loops against the independent recursive brute force on
every small shape: symbols and reconstructions must agree bit for bit."""
import itertools

import numpy as np
import pytest

from tests import brute

SIZES = [1, 2, 3, 4, 5, 7, 8, 9]


def _field(dims, seed):
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(*[np.arange(n) for n in dims], indexing="ij")
    smooth = np.sin(0.7 * x + 0.3) * np.cos(0.45 * y) + 0.2 * z
    return (smooth + 0.05 * rng.standard_normal(dims)).astype(np.float32)


@pytest.mark.parametrize("B,L", [(2, 1), (4, 2), (4, 1), (8, 3), (8, 2)])
def test_brute_force_matches_oracle(oracle, B, L):
    cases = list(itertools.product(SIZES, repeat=3))
    rng = np.random.default_rng(B * 10 + L)
    pick = rng.choice(len(cases), size=40, replace=False)
    for k, ci in enumerate(pick):
        dims = cases[ci]
        x = _field(dims, int(ci))
        for mode, eb, R in [(1, 1e-2, 512), (0, 3e-3, 512), (1, 1e-3, 4)]:
            cfg = oracle.config(block=B, levels=L, radius=R)
            s1, r1, l1 = oracle.symbols(x, mode, eb, cfg)
            s2, r2, l2 = brute.brute_symbols(x, mode, eb, B, L, R=R)
            assert np.array_equal(l1, l2), dims
            assert np.array_equal(s1, s2), (dims, mode, eb, R)
            assert np.array_equal(r1.view(np.uint32), r2.view(np.uint32)), (dims, mode, eb)


def test_brute_force_outliers_and_ratio(oracle):
    """Small radius forces outliers; a non-default ratio changes the level
    bounds. Both sides must still agree."""
    for dims in [(9, 9, 9), (5, 8, 3)]:
        x = _field(dims, 7) * 40
        for ratio in (1.0, 3.7):
            cfg = oracle.config(block=8, levels=3, radius=3, eb_ratio=ratio)
            s1, r1, _ = oracle.symbols(x, 0, 0.01, cfg)
            s2, r2, _ = brute.brute_symbols(x, 0, 0.01, 8, 3, R=3, ratio=ratio)
            assert np.any(s1 == 0)
            assert np.array_equal(s1, s2)
            assert np.array_equal(r1, r2)
