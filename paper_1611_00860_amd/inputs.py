"""Seeded synthetic inputs for the sgemm workloads.

This module holds no sgemm arithmetic: it only draws matrices and scalars.
Both the GPU path's tests/benchmark and the FP64 oracle's tests take their
inputs from here, so the two sides see the same numbers.

Generator: ``numpy.random.default_rng(seed)`` (PCG64).  Values are drawn in
float64 and cast to float32.  Draw order is A, B, C (each row-major), then the
upstream gradient G where one is needed.

Distributions:
* ``uniform``      -- i.i.d. uniform on [-1, 1].
* ``loguniform``   -- magnitude 2**U(-8, 8) (U uniform), times an independent
                      random sign; all magnitudes are drawn first, then signs.
* ``int``          -- integers uniform on [-8, 8]; with k <= 2**18 every
                      product sum stays an exact float32/bfloat16 integer.
* ``dyadic``       -- multiples of 2**-8 in [-1, 1]; a perturbation by
                      2**-10 stays exact in float32, which keeps finite
                      differences exact.

The paper measures sgemm on Parboil's input sets; those are not available
here, and these synthetic matrices stand in for them.
"""
from __future__ import annotations

import math

import numpy as np

DISTRIBUTIONS = ("uniform", "loguniform", "int", "dyadic")


def draw(rng: np.random.Generator, shape, dist: str = "uniform") -> np.ndarray:
    """One float32 array of ``shape`` from distribution ``dist``."""
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, size=shape).astype(np.float32)
    if dist == "loguniform":
        mag = np.exp2(rng.uniform(-8.0, 8.0, size=shape))
        sign = np.where(rng.integers(0, 2, size=shape) == 0, -1.0, 1.0)
        return (mag * sign).astype(np.float32)
    if dist == "int":
        return rng.integers(-8, 9, size=shape).astype(np.float32)
    if dist == "dyadic":
        return (rng.integers(-256, 257, size=shape) / 256.0).astype(np.float32)
    raise ValueError(f"unknown distribution {dist!r}")


def sgemm_operands(m: int, n: int, k: int, seed: int, dist: str = "uniform",
                   c_dist: str | None = None, pad: int = 0):
    """A (m x k), B (k x n), C (m x n) float32, row-major.

    ``pad`` > 0 returns views into arrays whose leading dimension is larger by
    ``pad`` elements (lda = k + pad, ldb = ldc = n + pad); the padding holds
    NaN so that a read outside the logical matrix poisons the result.
    """
    rng = np.random.default_rng(seed)
    A = draw(rng, (m, k), dist)
    B = draw(rng, (k, n), dist)
    C = draw(rng, (m, n), c_dist or dist)
    if pad:
        A, B, C = (_padded(X, pad) for X in (A, B, C))
    return A, B, C


def _padded(X: np.ndarray, pad: int) -> np.ndarray:
    r, c = X.shape
    big = np.full((r, c + pad), np.nan, dtype=np.float32)
    big[:, :c] = X
    return big[:, :c]


def grouped_problem(count: int = 512, seed: int = 3, lo: int = 32, hi: int = 2048,
                    multiple: int = 16):
    """Shapes and scalars of a grouped batch of independent sgemms.

    M, N, K are each drawn log-uniformly from [lo, hi] and rounded to a
    multiple of ``multiple``; alpha ~ U[0.5, 2], beta ~ U[0, 1].  Matrices are
    drawn afterwards, per instance in order (A, B, C), uniform on [-1, 1].
    Returns (dims[count, 3] int64, alpha[count] float32, beta[count] float32,
    rng) -- the rng is positioned to draw the matrices next.
    """
    rng = np.random.default_rng(seed)
    dims = np.empty((count, 3), dtype=np.int64)
    for col in range(3):
        x = np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))
        dims[:, col] = np.clip(np.round(x / multiple) * multiple, lo, hi)
    alpha = rng.uniform(0.5, 2.0, size=count).astype(np.float32)
    beta = rng.uniform(0.0, 1.0, size=count).astype(np.float32)
    return dims, alpha, beta, rng


def grouped_operands(dims, rng, dist: str = "uniform"):
    """Per-instance (A, B, C) lists for ``grouped_problem``'s shapes."""
    As, Bs, Cs = [], [], []
    for m, n, k in dims:
        As.append(draw(rng, (int(m), int(k)), dist))
        Bs.append(draw(rng, (int(k), int(n)), dist))
        Cs.append(draw(rng, (int(m), int(n)), dist))
    return As, Bs, Cs


def backward_operands(m: int, n: int, k: int, seed: int = 4, dist: str = "uniform"):
    """A, B, C_in, then the upstream gradient G = dL/dC_out, all float32."""
    rng = np.random.default_rng(seed)
    A = draw(rng, (m, k), dist)
    B = draw(rng, (k, n), dist)
    C = draw(rng, (m, n), dist)
    G = draw(rng, (m, n), dist)
    return A, B, C, G
