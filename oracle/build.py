"""Compile the plain-C oracle into ``oracle/liboracle.so``.

Test infrastructure: only the test suite, the smoke check and the CPU-baseline
leg of the benchmark use the library this builds.

The flags keep the arithmetic as written: no fast-math, no FMA contraction,
portable x86-64 code (the library travels to other hosts), OpenMP over
independent output columns only.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "chfsi_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O3", "-std=c99", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-D_POSIX_C_SOURCE=200809L",
        "-o", LIB + ".tmp", SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
