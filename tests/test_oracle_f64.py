"""Float64 fields (the paper's WarpX data are double precision, Sec. 4.1,
Table 2): the same format with value type 1 in the header, the predictor and
quantizer evaluated in double, anchors and outliers stored as 8-byte values.

Pins: the independent recursive brute force in float64 with an exact rational
error-bound test; stencil exactness for cubic polynomials at magnitudes that
float32 cannot hold; the error bound below float32 resolution (a float32
evaluation anywhere in the path would turn nearly every point into an
outlier); progressive and region invariants; header and section widths."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from paper_2509_01626_amd import fields
from tests import brute

F64 = np.float64


def _field(dims, seed, scale=1.0, offset=0.0):
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(*[np.arange(n) for n in dims], indexing="ij")
    smooth = np.sin(0.7 * x + 0.3) * np.cos(0.45 * y) + 0.2 * z
    return offset + scale * (smooth + 0.05 * rng.standard_normal(dims))


@pytest.mark.parametrize("B,L", [(2, 1), (4, 2), (8, 3), (8, 2)])
def test_f64_brute_force_matches_oracle(oracle, B, L):
    cases = list(itertools.product([1, 2, 3, 5, 8, 9], repeat=3))
    rng = np.random.default_rng(100 + B * 10 + L)
    for ci in rng.choice(len(cases), size=16, replace=False):
        dims = cases[ci]
        # offset 1 with fine detail: float32 would round away what the bounds keep
        x = _field(dims, int(ci), scale=1e-4, offset=1.0)
        for mode, eb, R in [(1, 1e-3, 512), (0, 3e-9, 512), (1, 1e-5, 4)]:
            cfg = oracle.config(block=B, levels=L, radius=R)
            s1, r1, l1 = oracle.symbols(x, mode, eb, cfg, dtype=F64)
            s2, r2, l2 = brute.brute_symbols(x, mode, eb, B, L, R=R, dtype=F64)
            assert np.array_equal(l1, l2), dims
            assert np.array_equal(s1, s2), (dims, mode, eb, R)
            assert np.array_equal(r1.view(np.uint64), r2.view(np.uint64)), (dims, mode, eb)


def test_f64_cubic_exact_beyond_float32(oracle):
    """Eqs. 6-8 reproduce cubic polynomials exactly. With integer coefficients
    and values near 2^36 every stencil sum is exact in double but not in
    float32, so the double predictor must return the sample itself."""
    n = 32
    z, y, x = np.meshgrid(*[np.arange(n, dtype=F64)] * 3, indexing="ij")
    v = (2.0 ** 36 + 7 * x ** 3 - 3 * x * y * z + 5 * y * y - 11 * z + 1)
    assert np.any(v.astype(np.float32).astype(F64) != v)
    for s in (1, 2):
        for q in [(7, 7, 7), (7, 9, 11), (8, 7, 9), (7, 8, 8), (8, 8, 7), (9, 9, 8)]:
            p = tuple(c * s for c in q)
            got = oracle.predict(v, p, s, dtype=F64)
            assert got == v[p], (p, s, got - v[p])
    # the float32 predictor on the same samples cannot be exact everywhere
    v32 = v.astype(np.float32)
    assert any(oracle.predict(v32, (7 * s, 9 * s, 11 * s), s) != v[7 * s, 9 * s, 11 * s]
               for s in (1, 2))


def test_f64_bound_below_float32_resolution(oracle):
    """A smooth field around 1 with detail far below float32's spacing (6e-8):
    every point stays within the bound (checked exactly) and most points are
    coded, not stored verbatim."""
    x = 1.0 + 1e-9 * fields.spectral((40, 48, 56), 5 / 3, seed=3).astype(F64)
    x = x + 1e-12 * np.random.default_rng(3).standard_normal(x.shape)
    eb = 1e-11
    comp = oracle.compress(x, oracle.EB_ABS, eb, oracle.config(block=16), dtype=F64)
    inf = oracle.info(comp)
    assert inf.dtype == 1
    full = oracle.decompress(comp)
    assert full.dtype == F64
    d = np.abs(full - x)
    assert float(d.max()) <= eb * (1 + 1e-6)
    # exact check on the points closest to the bound
    for i in np.argsort(d.ravel())[-50:]:
        assert abs(Fraction(float(full.flat[i])) - Fraction(float(x.flat[i]))) <= Fraction(eb)
    sym, _, _ = oracle.symbols(x, oracle.EB_ABS, eb, oracle.config(block=16), dtype=F64)
    outl = int((sym == 0).sum())
    assert outl < 0.01 * x.size, outl
    assert len(comp) < x.nbytes / 3


def test_f64_header_widths_and_type_checks(oracle):
    x = _field((17, 20, 33), 4, scale=3.0, offset=-1.0)
    cfg = oracle.config(block=8)
    comp = oracle.compress(x, oracle.EB_REL, 1e-4, cfg, dtype=F64)
    comp32 = oracle.compress(x, oracle.EB_REL, 1e-4, cfg)
    b = np.frombuffer(comp, dtype=np.uint8)
    assert int(b[52:56].view(np.uint32)[0]) == 1
    assert int(np.frombuffer(comp32, dtype=np.uint8)[52:56].view(np.uint32)[0]) == 0
    assert len(comp) <= oracle.compress_bound(x.shape, cfg, dtype=F64)
    # anchors: the stride-B grid, verbatim, 8 bytes each
    off = int(b[96:104].view(np.uint64)[0])
    n = int(b[104:112].view(np.uint64)[0])
    anchors = x[::8, ::8, ::8].ravel()
    assert n == anchors.size
    assert np.array_equal(b[off:off + 8 * n].view(F64), anchors)
    # outliers are stored verbatim as doubles
    _, E2, INV = oracle.level_bounds(1.0, 2.5, 3)
    assert E2[3] > 0 and INV[3] > 0
    # each decode entry point rejects a stream of the other value type
    assert oracle.decode_status(comp) == oracle.ERR_ARG
    assert oracle.decode_status(comp, "level", level=1) == oracle.ERR_ARG
    assert oracle.decode_status(comp, "region", level=2, lo=[0, 0, 0],
                                hi=[4, 4, 4]) == oracle.ERR_ARG
    assert oracle.decode_status(comp32, dtype=F64) == oracle.ERR_ARG
    assert oracle.decode_status(comp, dtype=F64) == oracle.OK
    # a value type other than 0 or 1 is a corrupt stream
    bad = bytearray(comp)
    bad[52] = 2
    assert oracle.decode_status(bytes(bad), dtype=F64) == oracle.ERR_CORRUPT


def test_f64_outliers_verbatim(oracle):
    """Small radius forces outliers; every outlier point decodes to the input
    double bit for bit."""
    x = _field((9, 16, 12), 6, scale=50.0)
    cfg = oracle.config(block=8, radius=3)
    sym, _, _ = oracle.symbols(x, oracle.EB_ABS, 1e-3, cfg, dtype=F64)
    assert int((sym == 0).sum()) > 50
    full = oracle.decompress(oracle.compress(x, oracle.EB_ABS, 1e-3, cfg, dtype=F64))
    m = sym <= 0  # outliers and anchors
    assert np.array_equal(full[m].view(np.uint64), x[m].view(np.uint64))
    assert float(np.abs(full - x).max()) <= 1e-3


@pytest.mark.parametrize("dims,B", [((33, 40, 29), 16), ((1, 70, 90), 8)])
def test_f64_progressive_and_region(oracle, dims, B):
    x = _field(dims, 9, scale=1e3)
    comp = oracle.compress(x, oracle.EB_REL, 1e-6, oracle.config(block=B), dtype=F64)
    inf = oracle.info(comp)
    full = oracle.decompress(comp)
    assert float(np.abs(full - x).max()) <= inf.eb_abs
    for lv in range(inf.levels + 1):
        s = 1 << (inf.levels - lv)
        assert np.array_equal(oracle.decompress_level(comp, lv), full[::s, ::s, ::s])
    rng = np.random.default_rng(1)
    for _ in range(6):
        lo = [int(rng.integers(0, n)) for n in dims]
        hi = [int(rng.integers(a + 1, n + 1)) for a, n in zip(lo, dims)]
        lv = int(rng.integers(0, inf.levels + 1))
        s = 1 << (inf.levels - lv)
        got = oracle.decompress_region(comp, lo, hi, lv)
        first = [-(-a // s) * s for a in lo]
        want = full[first[0]:hi[0]:s, first[1]:hi[1]:s, first[2]:hi[2]:s]
        assert np.array_equal(got, want), (lo, hi, lv)


def test_f64_float32_exact_data_decodes_like_float32(oracle):
    """Integer data with eb = 0.5 (2e = 1) and cubic-exact content: every
    prediction, difference and reconstruction is an exact small dyadic number
    in both precisions, so the two value types must code the same symbols."""
    n = 20
    z, y, x = np.meshgrid(*[np.arange(n, dtype=F64)] * 3, indexing="ij")
    v = (x * x - 2 * y + 3 * z + 1).astype(F64)
    cfg = oracle.config(block=8, levels=1)
    s64, r64, _ = oracle.symbols(v, oracle.EB_ABS, 0.5, cfg, dtype=F64)
    s32, r32, _ = oracle.symbols(v, oracle.EB_ABS, 0.5, cfg)
    assert np.array_equal(s64, s32)
    assert np.array_equal(r64, r32.astype(F64))
