"""Invariants of the oracle: error bound, progressive and region equalities,
decode-unit savings, determinism, and error handling."""
import numpy as np
import pytest

from paper_2509_01626_amd import fields


def _cfgs(oracle):
    return [oracle.config(block=8), oracle.config(block=16), oracle.config(block=4, levels=1),
            oracle.config(block=16, levels=3, radius=16)]


@pytest.mark.parametrize("dims", [(33, 20, 27), (16, 16, 16), (1, 9, 40), (7, 1, 1), (2, 3, 2)])
@pytest.mark.parametrize("eb", [1e-2, 1e-3, 1e-5])
def test_error_bound_everywhere(oracle, dims, eb):
    """|x - x'| <= eb_abs at every point, at every error bound and shape."""
    x = fields.bumps(dims, seed=sum(dims), n_bumps=6)
    for cfg in _cfgs(oracle):
        comp = oracle.compress(x, 1, eb, cfg)
        y = oracle.decompress(comp)
        eb_abs = oracle.info(comp).eb_abs
        assert np.all(np.abs(x.astype(np.float64) - y.astype(np.float64)) <= eb_abs)


def test_progressive_equals_full_subsample(oracle):
    """Decoding only up to level l gives exactly the full decode restricted to
    the stride-2^(L-l) grid (Sec. 3.3, progressive decompression)."""
    x = fields.spectral((40, 36, 45), alpha=5 / 3, seed=2)
    for cfg in _cfgs(oracle):
        comp = oracle.compress(x, 1, 1e-3, cfg)
        full = oracle.decompress(comp)
        L = oracle.info(comp).levels
        for l in range(L + 1):
            s = 1 << (L - l)
            lv = oracle.decompress_level(comp, l)
            assert np.array_equal(lv.view(np.uint32), full[::s, ::s, ::s].view(np.uint32))
        if L >= 1:
            # level 0 is the anchors, stored verbatim
            s0 = 1 << L
            assert np.array_equal(oracle.decompress_level(comp, 0), x[::s0, ::s0, ::s0])


def test_region_equals_full_restriction(oracle):
    """A region decode equals the same region of the full (or level) decode
    (Sec. 3.3, random-access decompression)."""
    rng = np.random.default_rng(5)
    x = fields.spectral((37, 41, 30), alpha=5 / 3, seed=4)
    for cfg in _cfgs(oracle):
        comp = oracle.compress(x, 1, 1e-3, cfg)
        L = oracle.info(comp).levels
        full = oracle.decompress(comp)
        for _ in range(12):
            lo = [int(rng.integers(0, n)) for n in x.shape]
            hi = [int(rng.integers(a + 1, n + 1)) for a, n in zip(lo, x.shape)]
            l = int(rng.integers(0, L + 1))
            s = 1 << (L - l)
            r = oracle.decompress_region(comp, lo, hi, l)
            first = [-(-a // s) * s for a in lo]
            want = full[first[0]:hi[0]:s, first[1]:hi[1]:s, first[2]:hi[2]:s]
            assert np.array_equal(r, want), (lo, hi, l)


def test_slice_decodes_three_of_seven_subblocks(oracle):
    """An even 2-D slice at full resolution needs only the three finest-level
    sub-blocks that lie in its plane (Sec. 3.3); the prediction at coarser
    levels still needs its neighbourhood."""
    x = fields.bumps((32, 32, 32), seed=1, n_bumps=8)
    comp = oracle.compress(x, 1, 1e-3, oracle.config(block=8))
    L = oracle.info(comp).levels
    oracle.decompress_region(comp, (10, 0, 0), (11, 32, 32), L)
    u = oracle.units_decoded()
    assert sorted(c for c in range(1, 8) if u[L, c] > 0) == [1, 2, 3]
    assert u[L, 1] == u[L, 2] == u[L, 3] == 16  # one z-layer of 4x4 blocks
    # A box decode touches every class of the blocks it covers.
    oracle.decompress_region(comp, (9, 9, 9), (12, 12, 12), L)
    u = oracle.units_decoded()
    assert all(u[L, c] == 1 for c in range(1, 8))
    # Full decode touches every unit.
    oracle.decompress(comp)
    u = oracle.units_decoded()
    assert all(u[L, c] == 64 for c in range(1, 8))


def test_determinism(oracle):
    x = fields.spectral((24, 24, 24), alpha=5 / 3, seed=9)
    cfg = oracle.config(block=8)
    assert oracle.compress(x, 1, 1e-3, cfg) == oracle.compress(x, 1, 1e-3, cfg)


def test_error_codes(oracle):
    x = fields.bumps((12, 12, 12), seed=3, n_bumps=4)
    cfg = oracle.config(block=8)
    assert oracle.compress_status(x, 1, 0.0, cfg) == oracle.ERR_ARG
    assert oracle.compress_status(x, 1, -1.0, cfg) == oracle.ERR_ARG
    assert oracle.compress_status(x, 2, 1e-3, cfg) == oracle.ERR_ARG
    assert oracle.compress_status(x, 1, 1e-3, oracle.config(block=12)) == oracle.ERR_ARG
    assert oracle.compress_status(x, 1, 1e-3, oracle.config(block=8, levels=4)) == oracle.ERR_ARG
    assert oracle.compress_status(x, 1, 1e-3, oracle.config(block=128)) == oracle.ERR_ARG
    assert oracle.compress_status(x, 1, 1e-3, oracle.config(block=8, radius=2048)) == oracle.ERR_ARG
    assert oracle.compress_status(x, 1, 1e-3, oracle.config(block=8, radius=1024)) == oracle.OK
    bad = x.copy()
    bad[3, 4, 5] = np.nan
    assert oracle.compress_status(bad, 1, 1e-3, cfg) == oracle.ERR_NONFINITE
    bad[3, 4, 5] = np.inf
    assert oracle.compress_status(bad, 0, 1e-3, cfg) == oracle.ERR_NONFINITE
    assert oracle.compress_status(x, 1, 1e-3, cfg, cap=100) == oracle.ERR_BUFFER
    comp = oracle.compress(x, 1, 1e-3, cfg)
    assert oracle.decode_status(comp) == oracle.OK
    # Truncation, bad magic, corrupted payload.
    assert oracle.decode_status(comp[:-4]) == oracle.ERR_CORRUPT
    assert oracle.decode_status(comp[:100]) == oracle.ERR_CORRUPT
    assert oracle.decode_status(b"XXXX" + comp[4:]) == oracle.ERR_CORRUPT
    # Region outside the domain and a level above L.
    assert oracle.decode_status(comp, "region", 3, (0, 0, 0), (13, 5, 5)) == oracle.ERR_ARG
    assert oracle.decode_status(comp, "region", 3, (5, 0, 0), (5, 5, 5)) == oracle.ERR_ARG
    assert oracle.decode_status(comp, "level", 9) == oracle.ERR_ARG


def test_corrupt_payload_never_crashes(oracle):
    """Random byte flips anywhere in the stream give OK or an error code."""
    x = fields.spectral((20, 20, 20), alpha=5 / 3, seed=1)
    comp = bytearray(oracle.compress(x, 1, 1e-3, oracle.config(block=8)))
    rng = np.random.default_rng(0)
    seen = set()
    for _ in range(200):
        c = bytearray(comp)
        i = int(rng.integers(0, len(c)))
        c[i] ^= 1 << int(rng.integers(0, 8))
        st = oracle.decode_status(bytes(c))
        assert st in (oracle.OK, oracle.ERR_CORRUPT, oracle.ERR_ARG, oracle.ERR_BUFFER)
        seen.add(st)
    assert oracle.ERR_CORRUPT in seen


def test_constant_field_relative(oracle):
    """Relative bound on a constant field (zero range) falls back to eb*|value|
    and reproduces the field exactly."""
    x = np.full((10, 11, 12), 3.5, dtype=np.float32)
    comp = oracle.compress(x, 1, 1e-3, oracle.config(block=8))
    assert oracle.info(comp).eb_abs == 1e-3 * 3.5
    assert np.array_equal(oracle.decompress(comp), x)
    z = np.zeros((5, 5, 5), dtype=np.float32)
    comp = oracle.compress(z, 1, 1e-3, oracle.config(block=4))
    assert oracle.info(comp).eb_abs == 1e-3
    assert np.array_equal(oracle.decompress(comp), z)


def test_single_point_and_anchor_only(oracle):
    x = np.array([[[2.5]]], dtype=np.float32)
    comp = oracle.compress(x, 0, 0.1, oracle.config(block=4))
    assert np.array_equal(oracle.decompress(comp), x)
    x = fields.bumps((1, 1, 9), seed=0, n_bumps=2)
    comp = oracle.compress(x, 0, 1e-4, oracle.config(block=8))
    y = oracle.decompress(comp)
    assert np.all(np.abs(y - x) <= 1e-4)
