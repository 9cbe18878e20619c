"""Build the HIP library libstz.so for gfx950 in-tree.

Device code is compiled without floating-point contraction, fast-math or
denormal flushing (the format fixes the float32 operation sequence), and with
packed-fp32 instruction selection disabled.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

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


OBJDIR = os.path.join(HERE, "_build")


def build(verbose=False):
    """Compile every source to an object in parallel, then link the library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    cflags = [f for f in FLAGS if f != "-shared"]
    objs = [os.path.join(OBJDIR, os.path.basename(f) + ".o") for f in SOURCES]
    cmds = [[hipcc] + cflags + ["-I", os.path.join(ROOT, "include"), "-c", "-o", o, f]
            for f, o in zip(SOURCES, objs)]
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as ex:
        for r in ex.map(lambda c: subprocess.run(c, check=True), cmds):
            pass
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
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
