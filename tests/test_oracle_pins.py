"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something that is not the oracle: the
coefficients printed in the paper, polynomial exactness, closed-form level
counts, an independent optimal-code cost, an independent 1-D subdivision.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_weights():
    rows = {}
    with open(os.path.join(GOLDEN, "stencil_weights.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            eq, offs, w = line.split()
            rows.setdefault(eq, {})[tuple(int(o) for o in offs.split(","))] = Fraction(w)
    return rows


# (dims, predicted point at stride 1, odd axes) that select each equation.
# Scaled by the stride s for the multi-stride check below.
CASES = {
    "eq6": ((16, 16, 16), (6, 6, 7), (2,)),
    "eq7": ((16, 16, 16), (6, 7, 7), (1, 2)),
    "eq8": ((16, 16, 16), (7, 7, 7), (0, 1, 2)),
    "eq3": ((16, 16, 3), (6, 6, 1), (2,)),
    "eq4": ((16, 16, 16), (6, 1, 1), (1, 2)),
    "eq5": ((16, 16, 16), (1, 1, 1), (0, 1, 2)),
}


@pytest.mark.parametrize("eq", sorted(CASES))
@pytest.mark.parametrize("s", [1, 2, 4])
def test_stencil_impulse_response_matches_paper(oracle, eq, s):
    """Putting a unit value at one coarse point and zero elsewhere must give
    exactly the weight the paper prints for that point (Sec. 3.1, Eqs. 3-8);
    every other coarse point of the neighbourhood has weight zero."""
    weights = load_weights()[eq]
    dims0, p0, axes = CASES[eq]
    dims = tuple(d * s if d > 3 else (d - 1) * s + 1 for d in dims0)
    p = tuple(c * s for c in p0)
    assert all((p[d] // s) % 2 == (1 if d in axes else 0) for d in range(3))
    total = Fraction(0)
    # Probe every coarse point within 3 strides along the odd axes.
    rng = [-3, -1, 1, 3]
    probes = [()]
    for _ in axes:
        probes = [q + (o,) for q in probes for o in rng]
    for offs in probes:
        q = list(p)
        for d, o in zip(axes, offs):
            q[d] += o * s
        if any(c < 0 or c >= n for c, n in zip(q, dims)):
            continue
        rec = np.zeros(dims, dtype=np.float32)
        rec[tuple(q)] = 1.0
        got = Fraction(oracle.predict(rec, p, s))
        want = weights.get(offs, Fraction(0))
        assert got == want, (eq, s, offs, got, want)
        total += got
    assert total == 1


def _poly_field(dims, f):
    z, y, x = np.meshgrid(*[np.arange(n, dtype=np.int64) for n in dims], indexing="ij")
    v = f(z, y, x)
    assert np.abs(v).max() < 2**20
    return v.astype(np.float32)


@pytest.mark.parametrize("s", [1, 2])
def test_cubic_stencils_exact_for_cubics(oracle, s):
    """Eq. 6 is exact for cubics along its axis; Eqs. 7 and 8 average cubic
    interpolations along diagonals, so they are exact for every polynomial of
    total degree <= 3 (its restriction to a line is a cubic)."""
    dims = (16 * s, 16 * s, 16 * s)
    polys = [
        lambda z, y, x: x**3 - 2 * x**2 + 5,
        lambda z, y, x: z * y * x + y**3 - 3 * x * x + 7 * z,
        lambda z, y, x: (z - y) ** 3 + 4 * x * y - 11,
    ]
    for f in polys:
        v = _poly_field(dims, f)
        for p0 in [(6, 6, 7), (6, 7, 6), (7, 6, 6), (6, 7, 7), (7, 6, 7), (7, 7, 6), (7, 7, 7),
                   (8, 9, 11), (9, 9, 9)]:
            p = tuple(c * s for c in p0)
            assert oracle.predict(v, p, s) == v[p], (p, s)


def test_boundary_rules_exact_for_linear(oracle):
    """Every boundary rule (quadratic, linear, extrapolation, nested fallback)
    reproduces linear functions; only the copy rule does not, and it is used
    only when an axis is no longer than twice the stride."""
    f = lambda z, y, x: 3 * z - 2 * y + 5 * x + 7
    for dims in [(9, 10, 11), (12, 7, 5), (5, 5, 5)]:
        v = _poly_field(dims, f)
        for s in (1, 2):
            for p in np.ndindex(*dims):
                odd = [(p[d] // s) % 2 == 1 and p[d] % s == 0 for d in range(3)]
                if not all(p[d] % s == 0 for d in range(3)) or not any(odd):
                    continue
                if any(odd[d] and dims[d] <= 2 * s for d in range(3)):
                    continue
                assert oracle.predict(v, p, s) == v[p], (dims, s, p)


@pytest.mark.parametrize("dims,B,L", [((40, 37, 33), 8, 3), ((33, 17, 65), 16, 4),
                                      ((20, 20, 20), 4, 2), ((17, 33, 9), 8, 2)])
def test_zero_codes_on_constant_and_linear_fields(oracle, dims, B, L):
    """Constant and linear fields are predicted exactly everywhere, so every
    non-anchor symbol is the zero-residual symbol R (axes longer than 2^L)."""
    R = 512
    cfg = oracle.config(block=B, levels=L)
    for f in [lambda z, y, x: 0 * z + 42, lambda z, y, x: 3 * z - 2 * y + 5 * x + 7,
              lambda z, y, x: -7 * z + 11 * y - x]:
        v = _poly_field(dims, f)
        sym, rec, lvl = oracle.symbols(v, 0, 0.25, cfg)
        assert np.all(sym[lvl > 0] == R)
        assert np.array_equal(rec, v)


def test_level_counts_closed_form(oracle):
    """Per-level point counts equal |G_l| - |G_{l-1}| with |G_l| the product of
    floor((n-1)/s_l)+1, and the paper's fractions hold (Sec. 3.2, Sec. 4.4)."""
    fr = {}
    with open(os.path.join(GOLDEN, "level_fractions.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, a, b = line.split()
                fr[k] = Fraction(int(a), int(b))
    for dims, B, L in [((64, 64, 64), 16, 4), ((19, 23, 30), 8, 3), ((64, 64, 64), 4, 2)]:
        x = np.zeros(dims, dtype=np.float32)
        _, _, lvl = oracle.symbols(x, 0, 1.0, oracle.config(block=B, levels=L))
        G = [int(np.prod([(n - 1) // (1 << (L - l)) + 1 for n in dims])) for l in range(L + 1)]
        for l in range(L + 1):
            want = G[0] if l == 0 else G[l] - G[l - 1]
            assert int(np.sum(lvl == l)) == want
        if dims == (64, 64, 64):
            N = 64**3
            assert Fraction(int(np.sum(lvl == L)), N) == fr["finest_level"]
            if L == 2:
                assert Fraction(int(np.sum(lvl == 0)), N) == fr["coarsest_3level"]
    # Survey table for the 64^3, B=16 configuration.
    x = np.zeros((64, 64, 64), dtype=np.float32)
    _, _, lvl = oracle.symbols(x, 0, 1.0, oracle.config(block=16))
    assert [int(np.sum(lvl == l)) for l in range(5)] == [64, 448, 3584, 28672, 229376]
    # Four levels with stride-8 anchors: 511/512 of the points are not anchors.
    _, _, lvl3 = oracle.symbols(x, 0, 1.0, oracle.config(block=16, levels=3))
    assert Fraction(int(np.sum(lvl3 > 0)), 64**3) == fr["outside_coarsest_4level"]


def test_level_bounds_ratio(oracle):
    """The finer level's bound is the ratio (2.5 in the paper) times the
    coarser level's (Sec. 3.1, Optimization 5)."""
    e, E2, INV = oracle.level_bounds(1e-3, 2.5, 5)
    assert e[5] == 1e-3
    assert abs(e[5] / e[4] - 2.5) < 1e-15
    assert abs(e[4] / e[3] - 2.5) < 1e-15
    assert e[3] == e[2] == e[1]
    for l in range(1, 6):
        assert E2[l] == np.float32(2 * e[l])
        assert INV[l] == np.float32(1 / (2 * e[l]))


# ---------------------------------------------------------------------------
# Huffman
# ---------------------------------------------------------------------------

def _kraft(lens):
    return sum(Fraction(1, 2 ** int(l)) for l in lens if l > 0)


@pytest.mark.parametrize("seed", range(8))
def test_huffman_optimal_and_complete(oracle, seed):
    """Without the length limit the code lengths are optimal (equal total cost
    to an independent Huffman merge) and complete (Kraft sum 1)."""
    rng = np.random.default_rng(seed)
    n = 1024
    k = int(rng.integers(2, 200))
    counts = np.zeros(n, dtype=np.uint64)
    idx = rng.choice(n, size=k, replace=False)
    counts[idx] = rng.geometric(0.05, size=k).astype(np.uint64) * rng.integers(1, 50, size=k)
    lens = oracle.huffman_lengths(counts, 30)
    assert _kraft(lens) == 1
    assert np.all((lens > 0) == (counts > 0))
    cost = int(np.sum(lens.astype(np.int64) * counts.astype(np.int64)))
    assert cost == brute.optimal_prefix_cost(counts)


def test_huffman_length_limit(oracle):
    """Fibonacci counts force depth ~ n; the limit rebuilds with halved counts
    until every code fits in 12 bits, keeping a complete prefix code."""
    fib = [1, 1]
    while len(fib) < 40:
        fib.append(fib[-1] + fib[-2])
    counts = np.zeros(1024, dtype=np.uint64)
    counts[:40] = fib
    lens = oracle.huffman_lengths(counts, 12)
    assert lens.max() <= 12
    assert _kraft(lens) == 1
    assert np.all((lens > 0) == (counts > 0))
    unl = oracle.huffman_lengths(counts, 60)
    assert unl.max() > 12


def test_huffman_length_limit_worked_examples(oracle):
    """Hand-worked lengths for counts that need one and two halvings to fit
    the 12-bit limit (tests/golden/huffman_length_limit.txt)."""
    n = 0
    with open(os.path.join(GOLDEN, "huffman_length_limit.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            a, b = line.split(";")
            counts = np.array([int(v) for v in a.split()], dtype=np.uint64)
            want = [int(v) for v in b.split()]
            assert list(oracle.huffman_lengths(counts, 12)) == want, (list(counts), want)
            n += 1
    assert n == 3


def _first_fitting_halving(oracle, counts, lmax):
    """k and ceil(c / 2^k) for the first k whose unlimited code fits lmax."""
    c = counts.astype(np.uint64)
    k = 0
    while oracle.huffman_lengths(c, 64).max() > lmax:
        c = np.where(c > 0, (c + 1) >> np.uint64(1), c).astype(np.uint64)
        k += 1
        assert k < 64
    return k, c


@pytest.mark.parametrize("seed", range(6))
def test_huffman_length_limit_is_halving_rebuild(oracle, seed):
    """The limited lengths are the unlimited lengths of ceil(c / 2^k) at the
    first k that fits (the rule restated: k halvings, each c -> ceil(c/2)),
    on skewed random histograms that exceed 12 bits."""
    rng = np.random.default_rng(100 + seed)
    counts = np.zeros(1024, dtype=np.uint64)
    m = int(rng.integers(20, 60))
    idx = rng.choice(1024, size=m, replace=False)
    counts[idx] = np.floor(1.6 ** rng.uniform(0, 45, size=m)).astype(np.uint64) + 1
    k, c = _first_fitting_halving(oracle, counts, 12)
    assert k >= 1, "the case must exercise the limit"
    # repeated ceil halving equals one division by 2^k, rounded up
    assert np.array_equal(c, (counts + np.uint64((1 << k) - 1)) >> np.uint64(k))
    assert np.array_equal(oracle.huffman_lengths(counts, 12), oracle.huffman_lengths(c, 64))


def test_huffman_degenerate(oracle):
    counts = np.zeros(16, dtype=np.uint64)
    assert np.all(oracle.huffman_lengths(counts) == 0)
    counts[5] = 1000
    lens = oracle.huffman_lengths(counts)
    assert lens[5] == 1 and lens.sum() == 1
    counts[9] = 1
    lens = oracle.huffman_lengths(counts)
    assert lens[5] == 1 and lens[9] == 1


def test_huffman_tie_rule_worked_examples(oracle):
    """Hand-worked code lengths for inputs with ties (the construction rule
    picks one of several optimal codes)."""
    with open(os.path.join(GOLDEN, "huffman_ties.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            a, b = line.split(";")
            counts = np.array([int(v) for v in a.split()], dtype=np.uint64)
            want = [int(v) for v in b.split()]
            assert list(oracle.huffman_lengths(counts)) == want, (list(counts), want)


def test_canonical_codes_prefix_free(oracle):
    """Canonical codes: increasing in (length, symbol) order, and no code is a
    prefix of another."""
    rng = np.random.default_rng(3)
    counts = rng.integers(0, 1000, size=300).astype(np.uint64)
    lens = oracle.huffman_lengths(counts)
    codes = oracle.canonical_codes(lens)
    used = [i for i in range(300) if lens[i]]
    order = sorted(used, key=lambda i: (lens[i], i))
    vals = [(int(codes[i]) << (12 - int(lens[i]))) for i in order]
    assert vals == sorted(vals) and len(set(vals)) == len(vals)
    strs = {format(int(codes[i]), f"0{int(lens[i])}b") for i in used}
    for a in strs:
        for b in strs:
            assert a == b or not b.startswith(a)


# ---------------------------------------------------------------------------
# Special case: every code zero -> hierarchical interpolation of the anchors
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,L", [(65, 4), (50, 4), (37, 3), (9, 3), (130, 5)])
def test_all_zero_codes_is_dd_subdivision(oracle, n, L):
    """With an error bound far above the data, every code is the zero-residual
    symbol and the decoder returns pure hierarchical interpolation of the
    anchors; in 1-D that is the Deslauriers-Dubuc 4-point subdivision (with the
    format's end rules), computed here independently."""
    rng = np.random.default_rng(n)
    x = rng.standard_normal((1, 1, n)).astype(np.float32)
    cfg = oracle.config(block=1 << L, levels=L)
    comp = oracle.compress(x, 0, 1e30, cfg)
    y = oracle.decompress(comp)
    sym, _, lvl = oracle.symbols(x, 0, 1e30, cfg)
    assert np.all(sym[lvl > 0] == 512)
    want = brute.subdivide_1d(x[0, 0, :: 1 << L], n, L)
    assert np.array_equal(y[0, 0], want)
