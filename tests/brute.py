"""Independent brute-force model of the STZ predictor/quantizer for tiny inputs.

Written separately from the C++ oracle, in a different shape: instead of level
loops over blocks and classes, every point's reconstruction is defined
recursively from the reconstructions of the coarser points its stencil reads
(Sec. 3.1-3.2 of the paper: a point depends only on the previous, coarser
level). The evaluation order follows the format (it is part of the format),
using numpy float32 (or float64) scalars, which round every operation to
nearest even and never fuse a multiply with an add. For float64 data the
error-bound test is done in exact rational arithmetic.

Also holds:
  * an independent 1-D hierarchical subdivision (Deslauriers-Dubuc 4-point
    scheme in the interior), used to pin the special case where every code is
    zero;
  * an independent optimal prefix-code cost (heap merge of the two lightest
    weights) for pinning the Huffman code lengths.
"""
import heapq
from fractions import Fraction
from functools import lru_cache

import numpy as np

F = np.float32


def level_strides(L):
    return {l: 1 << (L - l) for l in range(L + 1)}


def point_level(p, L):
    """Smallest level whose grid contains p (level 0 = stride 2^L anchors)."""
    for l in range(L + 1):
        s = 1 << (L - l)
        if all(c % s == 0 for c in p):
            return l
    raise AssertionError


def flags(n, c, s):
    return (c + s <= n - 1, c - 3 * s >= 0, c + 3 * s <= n - 1)


def one_axis(flag, s, f, F=F):
    """Nested fallback rule along one axis (linear / extrapolate / copy)."""
    p1, m3, _ = flag
    if p1:
        return (f(-s) + f(s)) * F(0.5)
    if m3:
        return (F(3.0) * f(-s) - f(-3 * s)) * F(0.5)
    return f(-s)


def stencil(val, dims, p, s, F=F):
    """Prediction of point p at stride s; val(q) returns the coarse value at q.
    F is the value type (numpy float32 or float64 scalar)."""
    odd = [d for d in range(3) if (p[d] // s) % 2 == 1]
    fl = [flags(dims[d], p[d], s) for d in odd]

    def at(offs):
        q = list(p)
        for d, o in zip(odd, offs):
            q[d] += o
        return val(tuple(q))

    if len(odd) == 1:
        p1, m3, p3 = fl[0]
        if p1 and m3 and p3:
            return (F(9.0) * (at([-s]) + at([s])) - (at([-3 * s]) + at([3 * s]))) * F(0.0625)
        if p1 and p3:
            return ((F(3.0) * at([-s]) + F(6.0) * at([s])) - at([3 * s])) * F(0.125)
        if p1 and m3:
            return ((F(6.0) * at([-s]) + F(3.0) * at([s])) - at([-3 * s])) * F(0.125)
        if p1:
            return (at([-s]) + at([s])) * F(0.5)
        if m3:
            return (F(3.0) * at([-s]) - at([-3 * s])) * F(0.5)
        return at([-s])
    full = all(a and b and c for a, b, c in fl)
    if full:
        k = len(odd)
        signs = [(-1, -1), (-1, 1), (1, -1), (1, 1)] if k == 2 else [
            (a, b, c) for a in (-1, 1) for b in (-1, 1) for c in (-1, 1)]
        inner = None
        outer = None
        for sg in signs:
            vi = at([g * s for g in sg])
            vo = at([3 * g * s for g in sg])
            inner = vi if inner is None else inner + vi
            outer = vo if outer is None else outer + vo
        scale = F(0.03125) if k == 2 else F(0.015625)
        return (F(9.0) * inner - outer) * scale

    def nest(i, offs):
        if i == len(odd):
            return at(offs)
        return one_axis(fl[i], s, lambda o: nest(i + 1, offs + [o]), F)

    return nest(0, [])


def level_bounds(eb_abs, ratio, L):
    e = {}
    for l in range(1, L + 1):
        if l == L:
            e[l] = eb_abs
        elif l == L - 1:
            e[l] = eb_abs / ratio
        else:
            e[l] = (eb_abs / ratio) / ratio
    E2 = {l: F(2.0 * e[l]) for l in e}
    INV = {l: F(1.0 / (2.0 * e[l])) for l in e}
    return e, E2, INV


def resolve_eb(x, mode, eb):
    if mode == 0:
        return eb
    mn = float(np.min(x))
    mx = float(np.max(x))
    rng = mx - mn
    if rng > 0:
        return eb * rng
    return eb * (abs(mn) if abs(mn) > 0 else 1.0)


def brute_symbols(x, mode, eb, B, L, R=512, ratio=2.5, dtype=np.float32):
    """Per-point (symbol, reconstruction, level); symbol -1 marks anchors."""
    F = np.dtype(dtype).type
    x = np.asarray(x, dtype=dtype)
    dims = x.shape
    eb_abs = resolve_eb(x, mode, eb)
    e, E2, INV = level_bounds(eb_abs, ratio, L)
    if F is np.float64:
        E2 = {l: F(2.0 * e[l]) for l in e}
        INV = {l: F(1.0 / (2.0 * e[l])) for l in e}
    assert 1 <= L and (1 << L) <= B

    @lru_cache(maxsize=None)
    def rec(p):
        return solve(p)[1]

    @lru_cache(maxsize=None)
    def solve(p):
        lv = point_level(p, L)
        xv = F(x[p])
        if lv == 0:
            return -1, xv
        s = 1 << (L - lv)
        pred = F(stencil(rec, dims, p, s, F))
        diff = xv - pred
        t = np.rint(diff * INV[lv])
        if abs(t) <= F(R - 1):
            q = int(t)
            xr = pred + F(q) * E2[lv]
            if abs(Fraction(float(xv)) - Fraction(float(xr))) <= Fraction(e[lv]):
                return q + R, F(xr)
        return 0, xv

    sym = np.empty(dims, dtype=np.int32)
    out = np.empty(dims, dtype=dtype)
    lvl = np.empty(dims, dtype=np.int32)
    for p in np.ndindex(*dims):
        a, b = solve(p)
        sym[p] = a
        out[p] = b
        lvl[p] = point_level(p, L)
    return sym, out, lvl


def subdivide_1d(anchors, n, L):
    """Hierarchical 1-D interpolation of anchor values at stride 2^L up to
    stride 1 on [0, n): the Deslauriers-Dubuc 4-point rule (-1, 9, 9, -1)/16
    in the interior; near the ends the format's boundary rules (quadratic
    through the three available neighbours, linear, linear extrapolation,
    copy)."""
    v = np.full(n, np.nan, dtype=np.float32)
    v[:: 1 << L] = anchors
    for l in range(1, L + 1):
        s = 1 << (L - l)
        for i in range(s, n, 2 * s):
            has_p1 = i + s <= n - 1
            has_m3 = i - 3 * s >= 0
            has_p3 = i + 3 * s <= n - 1
            a = v[i - 3 * s] if has_m3 else None
            b = v[i - s]
            c = v[i + s] if has_p1 else None
            d = v[i + 3 * s] if has_p3 else None
            if has_p1 and has_m3 and has_p3:
                v[i] = (F(9.0) * (b + c) - (a + d)) * F(0.0625)
            elif has_p1 and has_p3:
                v[i] = ((F(3.0) * b + F(6.0) * c) - d) * F(0.125)
            elif has_p1 and has_m3:
                v[i] = ((F(6.0) * b + F(3.0) * c) - a) * F(0.125)
            elif has_p1:
                v[i] = (b + c) * F(0.5)
            elif has_m3:
                v[i] = (F(3.0) * b - a) * F(0.5)
            else:
                v[i] = b
    return v


def optimal_prefix_cost(counts):
    """Minimum total bits of any prefix code for these counts (Huffman's
    merge with a heap): the sum of all merged weights."""
    h = [int(c) for c in counts if c > 0]
    if len(h) <= 1:
        return sum(h)
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a = heapq.heappop(h)
        b = heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


# ---------------------------------------------------------------------------
# Independent stream reader (format specification, written separately from
# the oracle's decoder): parses the header, level sections, lane streams and
# outlier lists and returns the per-point symbols and outlier values.
# ---------------------------------------------------------------------------
import struct


def _a16(v):
    return (v + 15) // 16 * 16


def read_stream(comp):
    b = bytes(comp)
    magic, version = struct.unpack_from("<II", b, 0)
    assert magic == 0x315A5453 and version == 1
    nz, ny, nx = struct.unpack_from("<QQQ", b, 8)
    B, L, R, lmax, mode, vtype = struct.unpack_from("<IIIIII", b, 32)
    eb, eb_abs, ratio = struct.unpack_from("<ddd", b, 56)
    total, clo, ao, na = struct.unpack_from("<QQQQ", b, 80)
    (coding,) = struct.unpack_from("<I", b, 112)
    assert total == len(b) and clo == 512 and lmax == 12
    assert vtype in (0, 1) and coding in (1, 2)
    vf, vw = ("<f8", 8) if vtype == 1 else ("<f4", 4)
    # code alphabet: symbols 0..2R-1, and token 2R (a chunk of centre symbols)
    # when the zero-chunk stage is on
    Z = 2 * R if coding == 2 else None
    lens = list(b[clo:clo + 2 * R + (coding == 2)])
    # canonical codes: (length, symbol) order, consecutive integers per length
    book = {}
    code = 0
    prev = 0
    for ln, sym in sorted((l, s) for s, l in enumerate(lens) if l > 0):
        code <<= ln - prev
        book[format(code, f"0{ln}b")] = sym
        code += 1
        prev = ln
    dims = (nz, ny, nx)
    anchors = np.frombuffer(b, dtype=vf, count=na, offset=ao)
    sym = np.full(dims, -1, dtype=np.int32)
    outv = {}
    nz_tokens = 0
    lane_bits = 0
    pos = _a16(ao + vw * na)
    for l in range(1, L + 1):
        off, nu, nl, nsym, words, nout = struct.unpack_from("<6Q", b, 128 + 48 * (l - 1))
        assert off == pos
        uw = np.frombuffer(b, "<u4", nu + 1, off)
        o2 = off + _a16(4 * (nu + 1))
        uo = np.frombuffer(b, "<u4", nu + 1, o2)
        o3 = o2 + _a16(4 * (nu + 1))
        lane = np.frombuffer(b, "<u2", nl, o3)
        lane_bits += int(lane.astype(np.int64).sum())
        o4 = o3 + _a16(2 * nl)
        pay = np.frombuffer(b, "<u4", words, o4)
        o5 = o4 + _a16(4 * words)
        outl = np.frombuffer(b, vf, nout, o5)
        pos = o5 + _a16(vw * nout)
        bits = "".join(format(int(w), "032b") for w in pay)
        s = 1 << (L - l)
        ui = 0
        li = 0
        nb = [-(-n // B) for n in dims]
        for bz in range(nb[0]):
            for by in range(nb[1]):
                for bx in range(nb[2]):
                    U = [-(-min(B, dims[d] - bb * B) // s) for d, bb in enumerate((bz, by, bx))]
                    for c in range(1, 8):
                        o = ((c >> 2) & 1, (c >> 1) & 1, c & 1)
                        M = [U[d] // 2 if o[d] else (U[d] + 1) // 2 for d in range(3)]
                        p = int(uw[ui]) * 32
                        vals = {}
                        for j in range(M[2]):
                            end = p + int(lane[li + j])
                            for vz in range(M[0]):
                                for vy in range(M[1]):
                                    cur = ""
                                    while cur not in book:
                                        cur += bits[p]
                                        p += 1
                                        assert len(cur) <= 12
                                    if book[cur] == Z:
                                        assert vy == 0
                                        nz_tokens += 1
                                        for k in range(M[1]):
                                            vals[(vz, k, j)] = R
                                        break
                                    vals[(vz, vy, j)] = book[cur]
                            assert p == end
                        assert -(-p // 32) == int(uw[ui + 1]) or M[0] * M[1] * M[2] == 0
                        oi = int(uo[ui])
                        for vz in range(M[0]):
                            for vy in range(M[1]):
                                for vx in range(M[2]):
                                    q = tuple(bb * B + s * (2 * v + oo) for bb, v, oo in
                                              zip((bz, by, bx), (vz, vy, vx), o))
                                    sym[q] = vals[(vz, vy, vx)]
                                    if sym[q] == 0:
                                        outv[q] = float(outl[oi])
                                        oi += 1
                        assert oi == int(uo[ui + 1])
                        li += M[2]
                        ui += 1
        assert ui == nu and li == nl
    assert pos == total
    return dict(dims=dims, B=B, L=L, R=R, eb_abs=eb_abs, anchors=anchors, sym=sym, outliers=outv,
                coding=coding, zero_tokens=nz_tokens, lens=lens, lane_bits=lane_bits)
