"""Build libaap.so in-tree for gfx950 with hipcc.

Flags:
  * ``-ffp-contract=off``: the binary64 decision arithmetic (cell ids and the
    neighbour test) must be the rounded operations written in the source;
  * ``-target-feature -packed-fp32-ops``: no packed FP32 instructions.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libaap.so")
LIB_SAN = os.path.join(HERE, "libaap_san.so")
SOURCES = [os.path.join(CSRC, f) for f in ("aap_kernels.hip", "aap_api.hip", "aap_surrogate.hip")]

# Host-side AddressSanitizer + UndefinedBehaviorSanitizer check build of the
# host runtime (the device code is built as usual): each -fsanitize= applies
# to the host compilation only.  Load it with clang's ASan runtime preloaded.
HOST_SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host",
                  "-fno-omit-frame-pointer", "-shared-libsan"]


def hipcc_command(out, sanitize=False):
    return [
        "hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-ffp-contract=off",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    ] + (HOST_SAN_FLAGS if sanitize else []) + ["-o", out] + SOURCES


def build_library(verbose=False, sanitize=False):
    out = LIB_SAN if sanitize else LIB
    tmp = out + ".tmp"
    cmd = hipcc_command(tmp, sanitize)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build_library(verbose="-v" in sys.argv or True)
