"""Compile the FP64 CPU oracle (test infrastructure) into oracle/_nbody_oracle.so with gcc.

Plain IEEE double arithmetic: no -ffast-math, no -ffp-contract=fast, so every operation is the
one the source writes.  OpenMP parallelises the loops over i only.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nbody_oracle.c")
LIB = os.path.join(HERE, "_nbody_oracle.so")


def build(verbose: bool = False, src: str = SRC, lib: str = LIB) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-Wno-maybe-uninitialized", "-o", lib + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
