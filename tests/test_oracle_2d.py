"""2-D fields (Sec. 3.1: the partition and prediction in the plane use the
sub-blocks b, c, d with Eqs. 3, 4, 6 and 7). A 2-D field is the 3-D format
with nz = 1: no point has an odd z, so the level points split into the three
in-plane classes, and the diagonal class uses the 2-D cubic (Eq. 7)."""
import numpy as np

from paper_2509_01626_amd import fields


def test_2d_classes_are_the_three_planar_subblocks(oracle):
    x = fields.bumps((1, 40, 56), seed=5, n_bumps=6)
    sym, _, lvl = oracle.symbols(x, oracle.EB_REL, 1e-3, oracle.config(block=8))
    L = int(lvl.max())
    anchors = ((40 - 1) // 8 + 1) * ((56 - 1) // 8 + 1)
    assert int((sym < 0).sum()) == anchors
    for l in range(1, L + 1):
        s = 1 << (L - l)
        y, x_ = np.nonzero(lvl[0] == l)
        cls = 2 * ((y // s) % 2) + (x_ // s) % 2   # in-plane parity class
        assert np.all((y % s == 0) & (x_ % s == 0))
        assert set(np.unique(cls)) <= {1, 2, 3} and len(y) > 0


def test_2d_cubic_exact_in_the_plane(oracle):
    """Eq. 7 (and Eq. 6 along each axis) reproduce polynomials of total degree
    <= 3 in (y, x) exactly at interior points."""
    ny, nx = 32, 32
    yy, xx = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                         indexing="ij")
    # integer coefficients: every value and every stencil sum is exact in float32
    v = (xx ** 3 - 2 * xx * yy * yy + 5 * yy * yy - 3 * xx + 4).reshape(1, ny, nx)
    v = v.astype(np.float32)
    for s in (1, 2):
        for p0 in [(0, 7, 7), (0, 9, 11), (0, 6, 7), (0, 7, 6)]:
            p = (0, p0[1] * s, p0[2] * s)
            assert oracle.predict(v, p, s) == v[p], (p, s)


def test_2d_roundtrip_bound_and_progressive(oracle):
    x = fields.spectral((1, 96, 80), 5 / 3, seed=8)
    for eb in (1e-2, 1e-3):
        comp = oracle.compress(x, oracle.EB_REL, eb, oracle.config(block=16))
        inf = oracle.info(comp)
        full = oracle.decompress(comp)
        assert float(np.abs(full.astype(np.float64) - x).max()) <= inf.eb_abs
        for lv in range(inf.levels + 1):
            s = 1 << (inf.levels - lv)
            assert np.array_equal(oracle.decompress_level(comp, lv), full[::s, ::s, ::s])
