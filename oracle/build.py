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
# AAP_ORACLE_LIB selects another build of the same source (the sanitizer
# check loads liborc_san.so this way)
LIB = os.environ.get("AAP_ORACLE_LIB") or os.path.join(HERE, "liborc.so")
LIB_SAN = os.path.join(HERE, "liborc_san.so")

# AddressSanitizer + UndefinedBehaviorSanitizer check build: every error
# aborts the process (load it with gcc's libasan preloaded)
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
             "-fno-omit-frame-pointer", "-g"]


def build_oracle(verbose: bool = False, sanitize: bool = False) -> str:
    out = LIB_SAN if sanitize else os.path.join(HERE, "liborc.so")
    tmp = out + ".tmp"
    cmd = [
        "gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off",
        "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-Wall",
    ] + (SAN_FLAGS if sanitize else []) + ["-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_oracle(verbose=True))
