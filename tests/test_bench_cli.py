"""bench.py's command-line contract, checked without a GPU: arguments that it
must refuse are refused before any device work, with a message and exit
status 2."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_unknown_variant_is_refused():
    r = run_bench("--variants", "precision,nonesuch")
    assert r.returncode == 2
    assert "nonesuch" in r.stderr
