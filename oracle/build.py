"""Build the C oracle into oracle/liboracle.so (test infrastructure only).

Flags: -O2 with FMA contraction and fast-math off, so every operation of the
oracle is one IEEE-754 round-to-nearest-even operation in its stated
precision; OpenMP parallelises rows inside one colour, which cannot change a
bit because points of one colour never read each other.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rbgs_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
          "-fno-fast-math", "-fno-unsafe-math-optimizations", "-fopenmp"]


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc; returns the path of the shared library."""
    cmd = ["gcc", *CFLAGS, SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
