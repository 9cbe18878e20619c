"""Build the HIP library libstz.so for gfx950 in-tree.

Device code is compiled without floating-point contraction, fast-math or
denormal flushing (the format fixes the float32 operation sequence), and with
packed-fp32 instruction selection disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libstz.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in
           ("stz_api.hip", "stz_compress.hip", "stz_codebook.hip", "stz_decode.hip",
            "stz_profile.hip")]
HEADERS = [os.path.join(ROOT, "include", "stz.h")] + [
    os.path.join(HERE, "csrc", f) for f in ("stz_internal.h", "stz_device.h", "stz_slab.h")]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc] + FLAGS + ["-I", os.path.join(ROOT, "include"), "-o", LIB + ".tmp"] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def stale():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(f) > t for f in SOURCES + HEADERS)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
