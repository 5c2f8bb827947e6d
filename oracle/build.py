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


# The sanitizer build (tests only): AddressSanitizer and UndefinedBehavior-
# Sanitizer, gcc's runtimes, loaded into a process that preloads libasan.
ASAN_LIB = os.path.join(os.path.dirname(HERE), "_build", "asan", "liboracle_sgemm_asan.so")


def asan_runtime() -> str:
    """Path of the gcc ASan runtime the sanitizer build needs preloaded."""
    out = subprocess.run([os.environ.get("CC", "gcc"), "-print-file-name=libasan.so"], capture_output=True, text=True)
    return os.path.realpath(out.stdout.strip())


def build(verbose: bool = False, sanitize: bool = False) -> str:
    lib = ASAN_LIB if sanitize else LIB
    os.makedirs(os.path.dirname(lib), exist_ok=True)
    cmd = [
        os.environ.get("CC", "gcc"), "-std=c11", "-O2", "-ffp-contract=off",
        "-fno-fast-math", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra",
        *(["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]
          if sanitize else []),
        "-o", lib + ".tmp", SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
