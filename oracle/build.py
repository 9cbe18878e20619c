"""Build the CPU oracle shared library (test infrastructure only).

The oracle is plain C++ compiled with contraction into fused multiply-add and
fast-math disabled, so its float32 arithmetic is the IEEE sequence written in
the source.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "stz_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
        "-Wall", "-Wextra", "-shared", "-fPIC", "-o", LIB, SRC,
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
