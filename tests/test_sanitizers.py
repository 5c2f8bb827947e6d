"""The CPU suites again, with AddressSanitizer on the host code.

The library's host side (argument checks, handle registries, plan, stream
and tracker bookkeeping, the CPU lowering) is rebuilt with ASan on its host
code only, and the C-ABI and CPU-lowering tests run against it in a process
that preloads ROCm clang's ASan runtime.  The oracle is rebuilt with gcc's
ASan and UBSan and its pin tests run the same way.  No GPU is touched: the
ABI tests stop every call before a kernel launch.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

pytestmark = pytest.mark.slow

SANITIZER_ERRORS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def _stale(lib, sources):
    return not os.path.exists(lib) or os.path.getmtime(lib) < max(os.path.getmtime(s) for s in sources)


def _run(cmd, env):
    out = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    text = out.stdout + out.stderr
    return out.returncode, text


def _env(preload, **extra):
    env = dict(os.environ)
    env.pop("HPVM_FAULT_INJECT", None)
    env["LD_PRELOAD"] = preload
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env.update(extra)
    return env


def test_host_library_under_asan():
    from paper_1611_00860_amd import build

    inc = os.path.join(ROOT, "include", "hpvm_sgemm.h")
    srcs = build.sources() + [inc] + [os.path.join(build.CSRC, f) for f in os.listdir(build.CSRC)]
    if _stale(build.ASAN_LIB, srcs):
        build.build(sanitize=True)
    rt = build.asan_runtime()
    assert rt and os.path.exists(rt), "ROCm clang's ASan runtime is missing"
    env = _env(rt, HPVM_SGEMM_LIB=build.ASAN_LIB)
    # the sanitized build is the one loaded, and the ASan runtime is live
    probe = ("import ctypes, os, paper_1611_00860_amd as hp; lib = hp.load(); "
             "assert lib._name == os.environ['HPVM_SGEMM_LIB'], lib._name; ctypes.CDLL(None).__asan_init")
    rc, text = _run([sys.executable, "-c", probe], env)
    assert rc == 0, text[-3000:]
    rc, text = _run([sys.executable, "-m", "pytest", "tests/test_abi.py", "tests/test_cpu_lowering.py", "-q",
                     "-m", "not gpu", "-p", "no:cacheprovider"], env)
    assert rc == 0 and not any(e in text for e in SANITIZER_ERRORS), text[-5000:]


def test_oracle_under_asan_and_ubsan():
    from oracle import build

    if _stale(build.ASAN_LIB, [build.SRC]):
        build.build(sanitize=True)
    rt = build.asan_runtime()
    assert rt and os.path.exists(rt), "gcc's ASan runtime is missing"
    env = _env(rt, HPVM_ORACLE_LIB=build.ASAN_LIB)
    probe = ("import ctypes, os, oracle; lib = oracle._load(); "
             "assert lib._name == os.environ['HPVM_ORACLE_LIB'], lib._name; ctypes.CDLL(None).__asan_init")
    rc, text = _run([sys.executable, "-c", probe], env)
    assert rc == 0, text[-3000:]
    rc, text = _run([sys.executable, "-m", "pytest", "tests/test_oracle_pins.py", "-q", "-p", "no:cacheprovider"],
                    env)
    assert rc == 0 and not any(e in text for e in SANITIZER_ERRORS), text[-5000:]
