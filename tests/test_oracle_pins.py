"""Pins for the FP64 oracle: facts fixed by mathematics, not by the oracle itself.

Each test would fail for a plausible slip in the oracle (a dropped alpha or
beta term, a wrong sign, a swapped index, lda/ldb confusion, a transposed
operand, a broken bfloat16 rounder).  None of them needs a GPU.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1611_00860_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U64 = 2.0 ** -53


def gamma(n, u=U64):
    return n * u / (1 - n * u)


def exact(A, B, C, alpha, beta):
    """alpha * A @ B + beta * C in exact rational arithmetic (tiny inputs only)."""
    m, k = A.shape
    n = B.shape[1]
    out = [[None] * n for _ in range(m)]
    for i in range(m):
        for j in range(n):
            s = sum((Fraction(float(A[i, p])) * Fraction(float(B[p, j])) for p in range(k)),
                    Fraction(0))
            v = Fraction(float(alpha)) * s
            if beta != 0:
                v += Fraction(float(beta)) * Fraction(float(C[i, j]))
            out[i][j] = v
    return out


def abs_scale(A, B, C, alpha, beta):
    """|alpha| |A||B| + |beta| |C| in float64 (the size against which error is bounded)."""
    s = abs(float(alpha)) * (np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64)))
    if beta != 0:
        s = s + abs(float(beta)) * np.abs(C.astype(np.float64))
    return s


# --------------------------------------------------------------------------- #
# Worked examples and brute force                                              #
# --------------------------------------------------------------------------- #
def test_worked_example_golden():
    with open(os.path.join(GOLDEN, "sgemm_worked_example.json")) as f:
        g = json.load(f)
    A = np.array(g["A"], dtype=np.float32)
    B = np.array(g["B"], dtype=np.float32)
    C = np.array(g["C"], dtype=np.float32)
    out = oracle.sgemm(A, B, C, g["alpha"], g["beta"])
    assert out.tolist() == g["expected"]


@pytest.mark.parametrize("m,n,k,pad", [(1, 1, 1, 0), (2, 3, 4, 0), (5, 4, 3, 2), (3, 5, 7, 3),
                                       (4, 1, 6, 1), (1, 6, 2, 0)])
def test_bruteforce_rational_random(m, n, k, pad):
    A, B, C = inputs.sgemm_operands(m, n, k, seed=100 + m * 31 + n * 7 + k, pad=pad)
    rng = np.random.default_rng(m + n + k)
    alpha, beta = (np.float32(v) for v in rng.uniform(-2, 2, size=2))
    out = oracle.sgemm(A, B, C, alpha, beta)
    ref = exact(A, B, C, alpha, beta)
    bound = gamma(k + 3) * abs_scale(A, B, C, alpha, beta)
    for i in range(m):
        for j in range(n):
            err = abs(Fraction(out[i, j]) - ref[i][j])
            assert err <= Fraction(bound[i, j]) + Fraction(1, 2 ** 1074), (i, j)


@pytest.mark.parametrize("m,n,k", [(3, 4, 5), (7, 2, 9), (8, 8, 8)])
def test_bruteforce_integers_exact(m, n, k):
    A, B, C = inputs.sgemm_operands(m, n, k, seed=7, dist="int", pad=1)
    out = oracle.sgemm(A, B, C, 3.0, -2.0)
    ref = exact(A, B, C, 3.0, -2.0)
    assert all(Fraction(out[i, j]) == ref[i][j] for i in range(m) for j in range(n))


def test_numpy_crosscheck_within_higham_bound():
    m, n, k = 37, 53, 61
    A, B, C = inputs.sgemm_operands(m, n, k, seed=11, dist="loguniform")
    alpha, beta = np.float32(0.75), np.float32(-1.25)
    out = oracle.sgemm(A, B, C, alpha, beta)
    ref = float(alpha) * (A.astype(np.float64) @ B.astype(np.float64)) + float(beta) * C.astype(np.float64)
    # both sides round in FP64 in different orders: each is within gamma_{k+2}
    bound = 2 * gamma(k + 3) * abs_scale(A, B, C, alpha, beta)
    assert np.all(np.abs(out - ref) <= bound)


def test_threads_do_not_change_bits():
    A, B, C = inputs.sgemm_operands(29, 31, 47, seed=5)
    one = oracle.sgemm(A, B, C, 1.5, 0.5, threads=1)
    many = oracle.sgemm(A, B, C, 1.5, 0.5, threads=7)
    assert np.array_equal(one, many)


# --------------------------------------------------------------------------- #
# Invariants                                                                   #
# --------------------------------------------------------------------------- #
def test_alpha_zero_gives_beta_c_and_ignores_ab():
    A, B, C = inputs.sgemm_operands(9, 11, 13, seed=3)
    A[2, 3] = np.nan
    B[4, 5] = np.inf
    out = oracle.sgemm(A, B, C, 0.0, 0.375)
    assert np.array_equal(out, 0.375 * C.astype(np.float64))


def test_beta_zero_never_reads_c():
    A, B, C = inputs.sgemm_operands(6, 5, 4, seed=4)
    C[:] = np.nan
    out = oracle.sgemm(A, B, C, 1.0, 0.0)
    assert np.all(np.isfinite(out))
    out2 = oracle.sgemm(A, B, None, 1.0, 0.0)
    assert np.array_equal(out, out2)


def test_identity_b():
    m, k = 12, 10
    A, _, C = inputs.sgemm_operands(m, k, k, seed=21)
    eye = np.eye(k, dtype=np.float32)
    alpha, beta = 1.75, -0.5
    out = oracle.sgemm(A, eye, C, alpha, beta)
    ref = alpha * A.astype(np.float64) + beta * C.astype(np.float64)
    assert np.array_equal(out, ref)


def test_k_zero_gives_beta_c():
    C = inputs.sgemm_operands(4, 6, 1, seed=2)[2]
    A = np.zeros((4, 0), dtype=np.float32)
    B = np.zeros((0, 6), dtype=np.float32)
    out = oracle.sgemm(A, B, C, 2.0, 0.25)
    assert np.array_equal(out, 0.25 * C.astype(np.float64))


def test_linearity_in_alpha_and_beta():
    A, B, C = inputs.sgemm_operands(15, 17, 19, seed=8)
    a1, a2 = 0.625, 1.125  # dyadic, a1 + a2 exact
    f12 = oracle.sgemm(A, B, C, a1 + a2, 0.0)
    f1 = oracle.sgemm(A, B, C, a1, 0.0)
    f2 = oracle.sgemm(A, B, C, a2, 0.0)
    scale = abs_scale(A, B, C, a1 + a2, 0.0)
    assert np.all(np.abs(f12 - (f1 + f2)) <= 4 * U64 * scale)
    # beta enters linearly and only through C
    g = oracle.sgemm(A, B, C, 1.0, 0.5) - oracle.sgemm(A, B, C, 1.0, 0.0)
    assert np.all(np.abs(g - 0.5 * C.astype(np.float64)) <= 4 * U64 * abs_scale(A, B, C, 1.0, 0.5))


def test_transpose_identity_bit_exact():
    A, B, C = inputs.sgemm_operands(7, 9, 11, seed=12)
    out = oracle.sgemm(A, B, C, 1.25, 0.75)
    At = np.ascontiguousarray(A.T)
    Bt = np.ascontiguousarray(B.T)
    Ct = np.ascontiguousarray(C.T)
    outt = oracle.sgemm(Bt, At, Ct, 1.25, 0.75)
    assert np.array_equal(out, outt.T)


def test_entries_equal_full_result():
    A, B, C = inputs.sgemm_operands(33, 21, 40, seed=9, pad=3)
    rng = np.random.default_rng(1)
    rows = rng.integers(0, 33, size=50)
    cols = rng.integers(0, 21, size=50)
    for mode in ("fp32", "bf16", "bf16x3"):
        full = oracle.sgemm(A, B, C, 0.5, 2.0, mode=mode)
        ent = oracle.sgemm_entries(A, B, C, 0.5, 2.0, rows, cols, mode=mode)
        assert np.array_equal(ent, full[rows, cols]), mode


# --------------------------------------------------------------------------- #
# bfloat16 rounding (split-aware modes)                                        #
# --------------------------------------------------------------------------- #
def _torch_bf16(x):
    torch = pytest.importorskip("torch")
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32))
    return t.to(torch.bfloat16).to(torch.float32).numpy()


def test_bf16_round_matches_library_conversion():
    rng = np.random.default_rng(0)
    bits = rng.integers(0, 2 ** 32, size=400_000, dtype=np.uint64).astype(np.uint32)
    # every exponent, plus exact ties, plus the largest finite values
    ties = (rng.integers(0, 2 ** 16, size=20_000, dtype=np.uint32) << 16) | np.uint32(0x8000)
    special = np.array([0x00000000, 0x80000000, 0x7F7FFFFF, 0x7F7F8000, 0x7F7F7FFF,
                        0xFF7F8000, 0x00000001, 0x00008000, 0x00018000, 0x007FFFFF,
                        0x7F800000, 0xFF800000, 0x3F808000, 0x3F818000], dtype=np.uint32)
    allbits = np.concatenate([bits, ties, special])
    x = allbits.view(np.float32)
    finite = np.isfinite(x)
    ours = oracle.bf16_round(x)
    ref = _torch_bf16(x)
    assert np.array_equal(np.isnan(ours), np.isnan(ref))
    keep = ~np.isnan(ref)
    assert np.array_equal(ours[keep].view(np.uint32), ref[keep].view(np.uint32))
    assert finite.sum() > 0


def test_bf16_round_hand_cases():
    cases = {
        0x3F808000: 0x3F800000,  # tie, even neighbour below
        0x3F818000: 0x3F820000,  # tie, even neighbour above
        0x3F808001: 0x3F810000,  # just above the tie
        0x7F7F8000: 0x7F800000,  # tie at the top rounds to +inf
        0x7F7F7FFF: 0x7F7F0000,  # just below: largest finite bfloat16
        0x80008000: 0x80000000,  # tie in the subnormals: -0
    }
    x = np.array(list(cases), dtype=np.uint32).view(np.float32)
    y = oracle.bf16_round(x).view(np.uint32)
    assert y.tolist() == list(cases.values())


def test_bf16_split_properties():
    rng = np.random.default_rng(3)
    x = inputs.draw(rng, (100_000,), "loguniform")
    hi, lo = oracle.bf16_split(x)
    assert np.all(hi.view(np.uint32) & 0xFFFF == 0)
    assert np.all(lo.view(np.uint32) & 0xFFFF == 0)
    x64 = x.astype(np.float64)
    assert np.all(np.abs(x64 - hi) <= 2.0 ** -8 * np.abs(x64))
    assert np.all(np.abs(x64 - (hi.astype(np.float64) + lo)) <= 2.0 ** -16 * np.abs(x64))
    assert np.array_equal(hi, _torch_bf16(x))
    assert np.array_equal(lo, _torch_bf16(x - hi))


def test_modes_agree_on_bf16_representable_inputs():
    A, B, C = inputs.sgemm_operands(10, 12, 14, seed=6, dist="int")
    outs = [oracle.sgemm(A, B, C, 1.0, 1.0, mode=m) for m in ("fp32", "bf16", "bf16x3")]
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_split_modes_bruteforce():
    A, B, C = inputs.sgemm_operands(3, 4, 5, seed=14)
    hiA, loA = (x.astype(np.float64) for x in oracle.bf16_split(A))
    hiB, loB = (x.astype(np.float64) for x in oracle.bf16_split(B))
    out16 = oracle.sgemm(A, B, C, 1.0, 0.0, mode="bf16")
    out3 = oracle.sgemm(A, B, C, 1.0, 0.0, mode="bf16x3")
    for i in range(3):
        for j in range(4):
            e16 = sum(Fraction(hiA[i, p]) * Fraction(hiB[p, j]) for p in range(5))
            e3 = sum(Fraction(hiA[i, p]) * Fraction(hiB[p, j]) + Fraction(hiA[i, p]) *
                     Fraction(loB[p, j]) + Fraction(loA[i, p]) * Fraction(hiB[p, j])
                     for p in range(5))
            assert abs(Fraction(out16[i, j]) - e16) <= Fraction(1e-15)
            assert abs(Fraction(out3[i, j]) - e3) <= Fraction(1e-15)


def test_bf16x3_representation_error_is_near_fp32():
    """hi*hi + hi*lo + lo*hi is accurate to about 2**-16 per product."""
    A, B, C = inputs.sgemm_operands(64, 64, 256, seed=2)
    ref = oracle.sgemm(A, B, C, 1.0, 0.0)
    out3 = oracle.sgemm(A, B, C, 1.0, 0.0, mode="bf16x3")
    out16 = oracle.sgemm(A, B, C, 1.0, 0.0, mode="bf16")
    rel3 = np.linalg.norm(out3 - ref) / np.linalg.norm(ref)
    rel16 = np.linalg.norm(out16 - ref) / np.linalg.norm(ref)
    assert rel3 < 1e-5
    assert 1e-4 < rel16 < 1e-2


# --------------------------------------------------------------------------- #
# Gradient                                                                     #
# --------------------------------------------------------------------------- #
def _loss(A, B, C, G, alpha, beta):
    """<G, C_out> with C_out from the oracle forward; exact for dyadic inputs."""
    out = oracle.sgemm(A, B, C, alpha, beta, threads=1)
    return float(np.sum(G.astype(np.float64) * out))


def test_gradient_central_differences_16():
    """L = <G, alpha A B + beta C> is linear in each argument: differences are exact."""
    n = 16
    A, B, C, G = inputs.backward_operands(n, n, n, seed=4, dist="dyadic")
    alpha, beta = np.float32(0.7), np.float32(0.3)
    h = 2.0 ** -10
    g = oracle.sgemm_grad(A, B, C, G, alpha, beta, threads=1)
    rng = np.random.default_rng(0)

    def fd_matrix(name, X, positions):
        out = []
        for (r, c) in positions:
            Xp = X.copy()
            Xm = X.copy()
            Xp[r, c] += np.float32(h)
            Xm[r, c] -= np.float32(h)
            assert float(Xp[r, c]) - float(X[r, c]) == h  # perturbation is exact
            args_p = {"A": A, "B": B, "C": C}
            args_m = dict(args_p)
            args_p[name] = Xp
            args_m[name] = Xm
            lp = _loss(args_p["A"], args_p["B"], args_p["C"], G, alpha, beta)
            lm = _loss(args_m["A"], args_m["B"], args_m["C"], G, alpha, beta)
            out.append((lp - lm) / (2 * h))
        return np.array(out)

    pos = [tuple(rng.integers(0, n, size=2)) for _ in range(12)]
    for name, X, key in (("A", A, "dA"), ("B", B, "dB"), ("C", C, "dC_in")):
        fd = fd_matrix(name, X, pos)
        ana = np.array([g[key][r, c] for r, c in pos])
        np.testing.assert_allclose(fd, ana, rtol=1e-12, atol=1e-12)
    # scalars: alpha +- h and beta +- h are exact in float32 for these values
    ap, am = np.float32(alpha + np.float32(h)), np.float32(alpha - np.float32(h))
    fd_a = (_loss(A, B, C, G, ap, beta) - _loss(A, B, C, G, am, beta)) / (float(ap) - float(am))
    bp, bm = np.float32(beta + np.float32(h)), np.float32(beta - np.float32(h))
    fd_b = (_loss(A, B, C, G, alpha, bp) - _loss(A, B, C, G, alpha, bm)) / (float(bp) - float(bm))
    assert math.isclose(fd_a, g["dalpha"], rel_tol=1e-12, abs_tol=1e-12)
    assert math.isclose(fd_b, g["dbeta"], rel_tol=1e-12, abs_tol=1e-12)


def test_gradient_identities():
    A, B, C, G = inputs.backward_operands(13, 9, 11, seed=4)
    alpha, beta = 0.7, 0.3
    g = oracle.sgemm_grad(A, B, C, G, alpha, beta)
    A64, B64, G64 = (x.astype(np.float64) for x in (A, B, G))
    # dalpha = <A, G B^T> = <A B, G>
    assert math.isclose(g["dalpha"], float(np.sum(A64 * (G64 @ B64.T))), rel_tol=1e-12)
    assert math.isclose(g["dbeta"], float(np.sum(G64 * C.astype(np.float64))), rel_tol=1e-12)
    np.testing.assert_allclose(g["dA"], alpha * G64 @ B64.T, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(g["dB"], alpha * A64.T @ G64, rtol=1e-12, atol=1e-12)
    assert np.array_equal(g["dC_in"], beta * G64)
    rows = np.array([0, 5, 12])
    cols = np.array([10, 0, 3])
    np.testing.assert_allclose(oracle.grad_entries("dA", A, B, G, alpha, rows, cols),
                               g["dA"][rows, cols], rtol=1e-13)
    rows = np.array([0, 5, 10])
    cols = np.array([8, 0, 3])
    np.testing.assert_allclose(oracle.grad_entries("dB", A, B, G, alpha, rows, cols),
                               g["dB"][rows, cols], rtol=1e-13)


# ---------------------------------------------------------------------------
# The one-to-one consumer node (the dependent pair that node fusion merges).
# ---------------------------------------------------------------------------
def test_consumer_worked_example():
    """Worked by hand from each function's definition."""
    X = np.array([[-2.5, 0.0, 3.25], [0.5, -0.0, 7.0]])
    bias = np.array([1.0, -1.0, 0.5], dtype=np.float32)
    expect = {
        "none": [[-2.5, 0.0, 3.25], [0.5, -0.0, 7.0]],
        "relu": [[0.0, 0.0, 3.25], [0.5, 0.0, 7.0]],         # v > 0 ? v : 0
        "bias": [[-1.5, -1.0, 3.75], [1.5, -1.0, 7.5]],      # v + bias[column]
        "bias_relu": [[0.0, 0.0, 3.75], [1.5, 0.0, 7.5]],
        "clamp": [[-1.0, 0.0, 2.0], [0.5, -0.0, 2.0]],       # into [-1, 2]
    }
    for op, want in expect.items():
        got = oracle.consumer(X, op, bias=bias, lo=-1.0, hi=2.0)
        assert got.tolist() == want, op


def test_consumer_invariants():
    rng = np.random.default_rng(11)
    X = rng.uniform(-4, 4, (37, 29))
    X[0, :5] = [0.0, -0.0, np.inf, -np.inf, 1e-300]
    bias = (rng.integers(-64, 64, 29) / 8.0).astype(np.float32)
    relu = oracle.consumer(X, "relu")
    # relu(x) - relu(-x) == x exactly, relu >= 0, and it never mixes columns
    assert np.array_equal(relu - oracle.consumer(-X, "relu"), X + 0.0)
    assert np.all(relu >= 0)
    # clamp into [0, inf) is relu; clamp into (-inf, inf) is the identity
    assert np.array_equal(oracle.consumer(X, "clamp", lo=0.0, hi=np.inf), relu)
    assert np.array_equal(oracle.consumer(X, "clamp"), X)
    c = oracle.consumer(X, "clamp", lo=-1.0, hi=0.5)
    assert c.min() == -1.0 and c.max() == 0.5
    inside = (X >= -1.0) & (X <= 0.5)
    assert np.array_equal(c[inside], X[inside])
    # bias adds column j's value to column j (dyadic: exact), bias+relu composes
    D = rng.integers(-1000, 1000, (37, 29)) / 64.0
    assert np.array_equal(oracle.consumer(D, "bias", bias=bias) - D, np.broadcast_to(bias, D.shape))
    assert np.array_equal(oracle.consumer(X, "bias_relu", bias=bias),
                          oracle.consumer(oracle.consumer(X, "bias", bias=bias), "relu"))
    assert np.array_equal(oracle.consumer(X, "bias", bias=np.zeros(29, np.float32)), X)
    # NaN: relu gives 0, bias and clamp keep it
    N = np.array([[np.nan, 1.0]])
    assert oracle.consumer(N, "relu")[0, 0] == 0.0
    assert np.isnan(oracle.consumer(N, "bias", bias=np.ones(2, np.float32))[0, 0])
    assert np.isnan(oracle.consumer(N, "clamp", lo=-1.0, hi=1.0)[0, 0])
    with pytest.raises(ValueError):
        oracle.consumer(X, 7)
