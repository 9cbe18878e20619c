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
@pytest.mark.parametrize("coding", [1, 2])
def test_independent_reader(oracle, dims, B, L, mode, eb, R, coding):
    rng = np.random.default_rng(sum(dims))
    x = (np.cumsum(rng.standard_normal(dims), axis=2)).astype(np.float32)
    cfg = oracle.config(block=B, levels=L, radius=R, coding=coding)
    comp = oracle.compress(x, mode, eb, cfg)
    st = brute.read_stream(comp)
    want, rec, lvl = brute.brute_symbols(x, mode, eb, B, L, R=R)
    assert st["dims"] == dims and st["B"] == B and st["L"] == L and st["R"] == R
    assert st["coding"] == coding
    assert st["eb_abs"] == brute.resolve_eb(x, mode, eb)
    assert np.array_equal(st["sym"][lvl > 0], want[lvl > 0])
    assert np.array_equal(st["anchors"], x[:: 1 << L, :: 1 << L, :: 1 << L].ravel())
    for q, v in st["outliers"].items():
        assert want[q] == 0 and np.float32(v) == x[q]
    assert len(st["outliers"]) == int(np.sum(want == 0))


def zero_chunks(sym, lvl, B, L, R):
    """(chunks whose symbols are all R, all chunks, symbols those chunks
    cover), counted from the per-point symbols: a chunk is the points of one
    sub-block with fixed (v_z, v_x), i.e. one class row along y inside one
    block."""
    dims = sym.shape
    nz = nall = cover = 0
    for l in range(1, L + 1):
        s = 1 << (L - l)
        nb = [-(-n // B) for n in dims]
        for bz in range(nb[0]):
            for by in range(nb[1]):
                for bx in range(nb[2]):
                    blk = tuple(slice(bb * B, min((bb + 1) * B, n), s)
                                for bb, n in zip((bz, by, bx), dims))
                    sb, lb = sym[blk], lvl[blk]
                    for oz in (0, 1):
                        for oy in (0, 1):
                            for ox in (0, 1):
                                if oz + oy + ox == 0:
                                    continue
                                cs = sb[oz::2, oy::2, ox::2]
                                assert np.all(lb[oz::2, oy::2, ox::2] == l)
                                if cs.size == 0:
                                    continue
                                allr = np.all(cs == R, axis=1)
                                nz += int(allr.sum())
                                nall += allr.size
                                cover += int(allr.sum()) * cs.shape[1]
    return nz, nall, cover


@pytest.mark.parametrize("dims,B", [((17, 24, 20), 8), ((12, 33, 16), 16), ((1, 40, 40), 8)])
def test_zero_chunk_tokens(oracle, dims, B):
    """Smooth data: most chunks are all-centre. The reader sees exactly one
    token per all-centre chunk (counted independently from the brute-force
    symbols), the decoded symbols are unchanged, the code is an optimal prefix
    code for the token counts, and the stage is lossless: both codings
    reconstruct the same values while the coded lanes are shorter."""
    z, y, x_ = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in dims], indexing="ij")
    x = (np.sin(0.11 * x_ + 0.07 * y) + 0.05 * z + 1e-4 * np.cos(3.1 * x_ * y)).astype(
        np.float32)
    L = int(np.log2(B))
    R = 512
    want, _, lvl = brute.brute_symbols(x, 1, 1e-2, B, L)
    nz, nall, cover = zero_chunks(want, lvl, B, L, R)
    assert nz > 0.3 * nall
    comp = oracle.compress(x, 1, 1e-2, oracle.config(block=B, coding=2))
    plain = oracle.compress(x, 1, 1e-2, oracle.config(block=B, coding=1))
    st = brute.read_stream(comp)
    assert st["zero_tokens"] == nz
    assert np.array_equal(st["sym"][lvl > 0], want[lvl > 0])
    assert brute.read_stream(plain)["zero_tokens"] == 0
    assert np.array_equal(oracle.decompress(comp).view(np.uint32),
                          oracle.decompress(plain).view(np.uint32))
    assert st["lane_bits"] < brute.read_stream(plain)["lane_bits"]
    # token counts: every symbol outside zero chunks, plus one token per chunk
    tok = np.bincount(want[lvl > 0].ravel(), minlength=2 * R + 1).astype(np.int64)
    tok[R] -= cover
    tok[2 * R] = nz
    lens = np.array(st["lens"], dtype=np.int64)
    assert np.array_equal(lens > 0, tok > 0)
    assert int((lens * tok).sum()) == st["lane_bits"]
    assert int((lens * tok).sum()) == brute.optimal_prefix_cost(tok[tok > 0].tolist())
