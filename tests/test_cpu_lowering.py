"""Parity of the CPU (vector) lowering of the sgemm graph with the FP64 oracle.

The CPU lowering is a separate target on host memory (no GPU needed).
Integer inputs are exact in FP32, so every tile, thread count and shape must
agree with the oracle bit for bit; random inputs are held to the FP32 bar
and to a componentwise accumulation bound.
"""
import numpy as np
import pytest

import oracle
import paper_1611_00860_amd as hp
from paper_1611_00860_amd import inputs

U32 = 2.0 ** -24
SHAPES = [(300, 260, 200), (129, 257, 77), (1, 1, 1), (64, 520, 48), (17, 33, 513)]


def padded(x, pad):
    r, c = x.shape
    buf = np.full((r, c + pad), np.nan, dtype=np.float32)
    buf[:, :c] = x
    return buf[:, :c]


@pytest.mark.parametrize("m,n,k", SHAPES)
def test_cpu_integers_bit_exact_every_tile(m, n, k):
    A, B, C = inputs.sgemm_operands(m, n, k, seed=m + 3 * k, dist="int")
    ref = oracle.sgemm(A, B, C, 1.0, -1.0)
    for tile in hp.cpu_menu():
        for threads in (1, 3):
            got = padded(C, 4)
            hp.sgemm_cpu(padded(A, 2), padded(B, 1), got, 1.0, -1.0, tile=tile, threads=threads)
            assert np.array_equal(got, ref), (tile, threads)


def test_cpu_random_within_fp32_bounds():
    m, n, k = 320, 288, 456
    A, B, C = inputs.sgemm_operands(m, n, k, seed=2)
    ref = oracle.sgemm(A, B, C, 1.5, 0.5)
    got = C.copy()
    hp.sgemm_cpu(A, B, got, 1.5, 0.5)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-5
    # componentwise: FP32 accumulation over k terms, then the epilogue
    ab = np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64))
    bound = 1.5 * 2 * (k + 2) * U32 * ab + 2 * U32 * np.abs(0.5 * C.astype(np.float64)) + 1e-30
    assert np.all(np.abs(got - ref) <= bound)


def test_cpu_thread_count_does_not_change_bits():
    A, B, C = inputs.sgemm_operands(333, 400, 300, seed=5, dist="loguniform")
    outs = []
    for threads in (1, 2, 7):
        got = C.copy()
        hp.sgemm_cpu(A, B, got, 1.0, 1.0, threads=threads)
        outs.append(got)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_cpu_special_cases():
    A, B, C = inputs.sgemm_operands(50, 40, 30, seed=6, dist="int")
    # alpha == 0: C <- beta C without reading A or B (NULL)
    got = C.copy()
    hp.sgemm_cpu(None, None, got, 0.0, 2.0, k=30)
    assert np.array_equal(got, 2.0 * C.astype(np.float64))
    # beta == 0: NaN in C is never read
    got = np.full_like(C, np.nan)
    hp.sgemm_cpu(A, B, got, 1.0, 0.0)
    assert np.array_equal(got, oracle.sgemm(A, B, None, 1.0, 0.0))
    # k == 0
    got = C.copy()
    hp.sgemm_cpu(np.zeros((50, 0), np.float32), np.zeros((0, 40), np.float32), got, 1.0, 0.5)
    assert np.array_equal(got, 0.5 * C.astype(np.float64))
    # m == 0: nothing to do
    hp.sgemm_cpu(np.zeros((0, 30), np.float32), B, np.zeros((0, 40), np.float32), 1.0, 1.0)


def test_cpu_validation():
    A, B, C = inputs.sgemm_operands(16, 16, 16, seed=7)
    with pytest.raises(hp.HpvmError) as ei:
        hp.sgemm_cpu(A, B, C, tile=(32, 32, 32, 8, 32, 1))
    assert ei.value.status == -2
    with pytest.raises(hp.HpvmError) as ei:
        hp.sgemm_cpu(A, B, C, threads=-1)
    assert ei.value.status == -1
    with pytest.raises(hp.HpvmError) as ei:  # C overlapping A
        hp.sgemm_cpu(A, B, A, 1.0, 0.0)
    assert ei.value.status == -1
    assert hp.cpu_isa() in ("avx512f", "avx2", "x86-64")
