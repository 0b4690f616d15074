"""Build the CPU oracle shared library (test infrastructure only).

    python oracle/build_oracle.py

Compiles oracle/rt_oracle.cpp with g++ into oracle/liboracle_rt.so.  The
flags keep IEEE binary64 semantics: no fused multiply-add contraction and no
fast-math, so the oracle's arithmetic is exactly the written expression order.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rt_oracle.cpp")
LIB = os.path.join(HERE, "liboracle_rt.so")


def build(verbose: bool = False) -> str:
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
