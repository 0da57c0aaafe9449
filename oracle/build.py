"""Build liboracle4.so from oracle4.c (plain C, no FMA contraction, OpenMP).

Test infrastructure: the library is loaded only by the tests, the smoke check
and the CPU-baseline leg of the benchmark.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle4.c")
LIB = os.path.join(HERE, "liboracle4.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-std=c99", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose: bool = False, src: str = SRC, lib: str = LIB) -> str:
    tmp = lib + ".tmp"
    cmd = ["gcc", *CFLAGS, src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
