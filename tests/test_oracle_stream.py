"""The oracle's byte stream read back by the independent reader: header
fields, level sections, lane streams and outliers must give exactly the
brute-force symbols of every point."""
import numpy as np
import pytest

from tests import brute


@pytest.mark.parametrize("dims,B,L,mode,eb,R", [
    ((9, 7, 8), 4, 2, 1, 1e-2, 512),
    ((5, 9, 3), 8, 3, 0, 2e-3, 16),
    ((8, 8, 8), 2, 1, 1, 1e-3, 512),
    ((1, 1, 17), 8, 3, 1, 1e-2, 512),
    ((3, 12, 10), 8, 2, 0, 1e-4, 4),
])
def test_independent_reader(oracle, dims, B, L, mode, eb, R):
    rng = np.random.default_rng(sum(dims))
    x = (np.cumsum(rng.standard_normal(dims), axis=2)).astype(np.float32)
    cfg = oracle.config(block=B, levels=L, radius=R)
    comp = oracle.compress(x, mode, eb, cfg)
    st = brute.read_stream(comp)
    want, rec, lvl = brute.brute_symbols(x, mode, eb, B, L, R=R)
    assert st["dims"] == dims and st["B"] == B and st["L"] == L and st["R"] == R
    assert st["eb_abs"] == brute.resolve_eb(x, mode, eb)
    assert np.array_equal(st["sym"][lvl > 0], want[lvl > 0])
    assert np.array_equal(st["anchors"], x[:: 1 << L, :: 1 << L, :: 1 << L].ravel())
    for q, v in st["outliers"].items():
        assert want[q] == 0 and np.float32(v) == x[q]
    assert len(st["outliers"]) == int(np.sum(want == 0))
