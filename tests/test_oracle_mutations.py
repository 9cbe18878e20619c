"""Mutation check of the oracle's pins (CPU only, slow).

Each mutation plants one plausible mistake in a copy of the oracle source (a
wrong stencil weight or sign, an availability flag off by a point, a wrong
bound ratio, class or lane order, bit order, Huffman tie or halving rule,
dependency-cone width, quantizer radius or dequantization step), builds it
as a separate library and runs the oracle's CPU pin tests against it
(STZ_ORACLE_LIB). Every mutation must make at least one pin fail; a mutation
that survives names a pin that is missing.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "stz_oracle.cpp")

PIN_TESTS = ["tests/test_oracle_pins.py", "tests/test_oracle_brute.py",
             "tests/test_oracle_stream.py", "tests/test_oracle_invariants.py",
             "tests/test_oracle_2d.py", "tests/test_oracle_f64.py", "tests/test_oracle_roi.py"]

# name -> [(exact text, replacement)]; every text must occur exactly once.
MUTATIONS = {
    "eq6 inner weight 9 -> 8": [
        ("return ((T(9) * (Bv + Cv)) - (A + Dv)) * T(0.0625);",
         "return ((T(8) * (Bv + Cv)) - (A + Dv)) * T(0.0625);")],
    "eq7 scale 1/32 -> 1/16": [
        ("return ((T(9) * in) - out) * T(0.03125);", "return ((T(9) * in) - out) * T(0.0625);")],
    "eq8 outer sign": [
        ("return ((T(9) * in) - out) * T(0.015625);",
         "return ((T(9) * in) + out) * T(0.015625);")],
    "quadratic low-edge weight": [
        ("return ((T(3) * Bv + T(6) * Cv) - Dv) * T(0.125);",
         "return ((T(3) * Bv + T(6) * Cv) - Dv) * T(0.25);")],
    # (pd is an odd multiple of s, so pd >= 2s would equal pd >= 3s)
    "M3 flag strict": [("f.M3 = pd >= 3 * s;", "f.M3 = pd > 3 * s;")],
    "P3 flag one point short": [
        ("f.P3 = pd + 3 * s <= g.n[d] - 1;", "f.P3 = pd + 3 * s <= g.n[d] - 2;")],
    "coarse bound ratio applied once": [
        ("e = (eb_abs / ratio) / ratio;", "e = eb_abs / ratio;")],
    "default ratio 2.0": [
        ("double ratio = d.eb_ratio != 0.0 ? d.eb_ratio : 2.5;",
         "double ratio = d.eb_ratio != 0.0 ? d.eb_ratio : 2.0;")],
    "class parity z <-> x": [
        ("u.o[0] = (c >> 2) & 1;", "u.o[0] = c & 1;"),
        ("u.o[2] = c & 1;", "u.o[2] = (c >> 2) & 1;")],
    "lane order reversed": [
        ("uint16_t sy = syms[l][sym_base + (vz * u.M[1] + vy) * u.M[2] + j];",
         "uint16_t sy = syms[l][sym_base + (vz * u.M[1] + vy) * u.M[2] + (u.M[2] - 1 - j)];")],
    "bit order LSB first": [
        ("(*words)[w] |= 1u << (31 - (pos & 31));", "(*words)[w] |= 1u << (pos & 31);")],
    "Huffman ties to the node queue": [("wt[li] <= wt[ii]", "wt[li] < wt[ii]")],
    "length-limit halving floor(c/2), at least 1": [
        ("if (w[i]) w[i] = (w[i] + 1) >> 1;",
         "if (w[i]) w[i] = std::max<uint64_t>(1, w[i] >> 1);")],
    "dependency cone 2s": [
        ("const uint64_t r = 3 * g.stride(k);", "const uint64_t r = 2 * g.stride(k);")],
    "quantizer radius R-2": [
        ("if (std::fabs(t) <= (T)(R - 1)) {", "if (std::fabs(t) <= (T)(R - 2)) {")],
    "dequantization step e instead of 2e": [
        ("T prod = (T)(sym - P.c.R) * E2;", "T prod = (T)(sym - P.c.R) * (E2 * T(0.5));")],
}


def _mutant_source(edits):
    with open(SRC) as f:
        src = f.read()
    for old, new in edits:
        assert src.count(old) == 1, f"mutation target not unique or missing: {old!r}"
        src = src.replace(old, new)
    return src


def _survives(name, edits, tmp):
    """True when every pin test passes against the mutated oracle."""
    d = os.path.join(tmp, str(abs(hash(name))))
    os.makedirs(d, exist_ok=True)
    cpp = os.path.join(d, "stz_oracle.cpp")
    so = os.path.join(d, "liboracle.so")
    with open(cpp, "w") as f:
        f.write(_mutant_source(edits))
    subprocess.run(["g++", "-O1", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-shared",
                    "-fPIC", "-o", so, cpp], check=True)
    env = dict(os.environ, STZ_ORACLE_LIB=so)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu and not slow",
                        "-p", "no:cacheprovider"] + PIN_TESTS,
                       cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       timeout=900)
    return r.returncode == 0


@pytest.mark.slow
def test_every_mutation_fails_a_pin():
    for edits in MUTATIONS.values():  # targets still present, before any build
        _mutant_source(edits)
    with tempfile.TemporaryDirectory() as tmp:
        with ThreadPoolExecutor(max_workers=4) as ex:
            res = dict(zip(MUTATIONS, ex.map(lambda kv: _survives(kv[0], kv[1], tmp),
                                             MUTATIONS.items())))
    survivors = [k for k, v in res.items() if v]
    assert not survivors, f"mutations no pin detects: {survivors}"


def test_mutation_targets_present():
    """Cheap guard (not slow): every mutation still applies to the current
    oracle source."""
    for edits in MUTATIONS.values():
        _mutant_source(edits)
