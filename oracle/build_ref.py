"""Builds the CPU oracle ``oracle/libptalm_ref.so`` with gcc (plain C + OpenMP).

Portable flags only (no -march=native): the library built here also runs on
the benchmark host.  No fast-math: IEEE round-to-nearest throughout.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ptalm_ref.c")
OUT = os.path.join(HERE, "libptalm_ref.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", OUT + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
