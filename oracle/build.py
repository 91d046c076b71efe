"""Build the FP64 CPU oracle (test infrastructure) into ``oracle/_lbm_oracle.so``.

Plain ``gcc -O2`` with OpenMP over lattice rows; no vector intrinsics and no
fast-math, so that every arithmetic step is the one written in the source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["lbm_oracle.c"]
TARGET = os.path.join(HERE, "_lbm_oracle.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-std=c11",
           "-Wall", "-Wextra", "-shared", "-fPIC", "-o", TARGET + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(TARGET + ".tmp", TARGET)
    return TARGET


def build_sanitized(target: str, verbose: bool = False) -> str:
    """The same source with AddressSanitizer and UndefinedBehaviorSanitizer
    (host code only; load it with the ASan runtime preloaded)."""
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", target] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return target


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
