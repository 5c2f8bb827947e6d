"""Compile the FP64 sgemm oracle (test infrastructure) with the system C compiler.

The oracle is plain C: ``gcc -O2 -ffp-contract=off`` so that no fused
multiply-add changes its rounding, threaded with pthreads over output rows.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sgemm_oracle.c")
LIB = os.path.join(HERE, "liboracle_sgemm.so")


def build(verbose: bool = False) -> str:
    cmd = [
        os.environ.get("CC", "gcc"), "-std=c11", "-O2", "-ffp-contract=off",
        "-fno-fast-math", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra",
        "-o", LIB + ".tmp", SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
