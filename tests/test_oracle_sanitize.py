"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only,
slow): the oracle's pin tests against a sanitized build of the oracle, and a
byte-flip fuzz of its decoders (tests/sanitize/oracle_fuzz.cpp). Any
sanitizer finding aborts the run and fails the test."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
       "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
PIN_TESTS = ["tests/test_oracle_pins.py", "tests/test_oracle_brute.py",
             "tests/test_oracle_stream.py", "tests/test_oracle_invariants.py",
             "tests/test_oracle_2d.py", "tests/test_oracle_f64.py", "tests/test_oracle_roi.py"]


def _runtime(name):
    p = subprocess.run(["g++", f"-print-file-name={name}"], stdout=subprocess.PIPE, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_decoder_fuzz_under_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_fuzz")
        subprocess.run(["g++"] + SAN + ["-o", exe,
                                        os.path.join(ROOT, "tests", "sanitize", "oracle_fuzz.cpp")],
                       check=True)
        r = subprocess.run([exe, "40"], stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                           text=True, timeout=600)
        assert r.returncode == 0, r.stdout[-4000:]
        assert r.stdout.startswith("ok:"), r.stdout[-4000:]


@pytest.mark.slow
def test_pins_against_sanitized_oracle():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("sanitizer runtimes not found")
    with tempfile.TemporaryDirectory() as tmp:
        so = os.path.join(tmp, "liboracle_san.so")
        subprocess.run(["g++"] + SAN + ["-shared", "-fPIC", "-o", so,
                                        os.path.join(ROOT, "oracle", "stz_oracle.cpp")],
                       check=True)
        pre = " ".join(p for p in (asan, ubsan, os.environ.get("LD_PRELOAD", "")) if p)
        env = dict(os.environ, STZ_ORACLE_LIB=so, LD_PRELOAD=pre,
                   ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m",
                            "not gpu and not slow", "-p", "no:cacheprovider"] + PIN_TESTS,
                           cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                           text=True, timeout=900)
        assert r.returncode == 0, r.stdout[-4000:]
