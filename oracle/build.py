"""Build the oracle's shared library (test infrastructure only).

Compiles ``aap_oracle.c`` with gcc at -O2, without FP contraction and
without fast-math, so every double operation is the rounded IEEE operation
written in the source.  OpenMP only spreads independent particles over
threads; results do not depend on the thread count.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "aap_oracle.c")
LIB = os.path.join(HERE, "liborc.so")


def build_oracle(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [
        "gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off",
        "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-Wall",
        "-o", tmp, SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_oracle(verbose=True))
