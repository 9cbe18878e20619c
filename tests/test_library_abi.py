"""The C-ABI library loads and exports every function include/stz.h declares
(no compute calls; runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "stz.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(stz_[a-z_]+)\s*\(", src)))


def test_header_declares_boundary():
    names = declared_functions()
    for n in ["stz_compress", "stz_decompress", "stz_decompress_level", "stz_decompress_region",
              "stz_compress_bound", "stz_info", "stz_status_string"]:
        assert n in names


def test_library_exports_all_declared():
    from paper_2509_01626_amd import build
    if build.stale():
        pytest.skip("library not built or older than its sources (run __graft_entry__.build())")
    lib = ctypes.CDLL(build.LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_compress_bound_matches_oracle(oracle):
    """Host-only entry point: same worst-case bound formula on both sides."""
    from paper_2509_01626_amd import build, stz
    if build.stale():
        pytest.skip("library not built")
    for shape, B, L in [((64, 64, 64), 16, 0), ((33, 17, 5), 8, 2), ((1, 1, 1), 2, 1),
                        ((512, 512, 512), 32, 0)]:
        a = stz.stz_compress_bound(shape, stz.config(block=B, levels=L))
        b = oracle.compress_bound(shape, oracle.config(block=B, levels=L))
        assert a >= b > 0
    assert stz.stz_compress_bound((4, 4, 4), stz.config(block=12)) == 0
    assert stz.lib().stz_status_string(-4) == b"corrupt stream"
