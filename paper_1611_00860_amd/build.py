"""Build libhpvm_sgemm.so: the gfx950 kernels and the C-ABI host layer.

Every ``csrc/*.hip`` file is compiled with hipcc for gfx950 only, every
``csrc/*.cpp`` file (host-only C++: the CPU lowering) with the host compiler,
and all are linked into one shared library under ``lib/``.  Packed FP32
instructions are turned off (``-packed-fp32-ops``); hipcc's host pass warns
that it does not know that feature, which is harmless.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libhpvm_sgemm.so")
OBJDIR = os.path.join(ROOT, "_build")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


# The sanitizer build (tests only): AddressSanitizer on the host code of
# every source (argument checks, handle registries, plan and tracker
# bookkeeping); device code is built as usual.  The ASan runtime is the one
# of the ROCm clang that compiles the host code; the library is loaded into
# a process that preloads it.
ASAN_DIR = os.path.join(OBJDIR, "asan")
ASAN_LIB = os.path.join(ASAN_DIR, "libhpvm_sgemm_asan.so")
ASAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
CLANGXX = "/opt/rocm/llvm/bin/clang++"


def asan_runtime() -> str:
    """Path of the ASan runtime the sanitizer build needs preloaded."""
    out = subprocess.run([CLANGXX, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = out.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        found = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        path = found[0] if found else ""
    return path


def _compile(src: str, verbose: bool, objdir: str = OBJDIR, extra=()) -> str:
    obj = os.path.join(objdir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *extra, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    if err.strip() and verbose:
        print(err, file=sys.stderr)
    return obj


CXX = os.environ.get("CXX", "g++")
CXXFLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", INCLUDE, "-I", CSRC]


def _compile_host(src: str, verbose: bool, objdir: str = OBJDIR, sanitize: bool = False) -> str:
    """Host-only C++ (the CPU lowering): compiled by the host compiler."""
    obj = os.path.join(objdir, os.path.basename(src) + ".o")
    cmd = [CLANGXX, *CXXFLAGS, "-fsanitize=address", "-fno-omit-frame-pointer"] if sanitize else [CXX, *CXXFLAGS]
    cmd += ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"{CXX} failed on {src}:\n{res.stderr}")
    return obj


def sources() -> list:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip"))) + sorted(glob.glob(os.path.join(CSRC, "*.cpp")))


def build(verbose: bool = False, jobs: int | None = None, sanitize: bool = False) -> str:
    """Compile every kernel source for gfx950 and link the library; returns its
    path.  sanitize: the AddressSanitizer build of the host code, as ASAN_LIB."""
    objdir = ASAN_DIR if sanitize else OBJDIR
    lib = ASAN_LIB if sanitize else LIB
    os.makedirs(objdir, exist_ok=True)
    os.makedirs(os.path.dirname(lib), exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 2) // 2))

    def one(src):
        if src.endswith(".cpp"):
            return _compile_host(src, verbose, objdir, sanitize)
        return _compile(src, verbose, objdir, ASAN_HOST if sanitize else ())

    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(one, srcs))
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *(ASAN_HOST if sanitize else ()), "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
