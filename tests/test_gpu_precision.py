"""GPU parity of the BF16 and bf16x3 lowerings (needs an MI355X).

Two references: the exact FP64 oracle (the bar: normwise error <= 1e-2 for
BF16, <= 1e-5 for bf16x3) and the oracle's split-aware mode, which applies
the same bfloat16 rounding / hi-lo split to the inputs and then sums exactly;
against it only the kernel's FP32 accumulation error remains, bounded
componentwise.
"""
import numpy as np
import pytest

import oracle
from paper_1611_00860_amd import inputs
from gpu_util import componentwise_bound, normwise, to_dev, to_host

pytestmark = pytest.mark.gpu

BAR = {"bf16": 1e-2, "bf16x3": 1e-5}


def run(hp, A, B, C, alpha, beta, prec, tile=None, pad=0, misalign=False):
    import torch

    dA, dB, dC = (to_dev(x, pad, misalign) for x in (A, B, C))
    hp.sgemm(dA, dB, dC, alpha, beta, prec=prec, tile=tile)
    torch.cuda.synchronize()
    return to_host(dC)


SHAPES = [(300, 260, 200), (257, 129, 77), (1, 1, 1), (64, 520, 48)]


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
@pytest.mark.parametrize("m,n,k", SHAPES)
def test_integers_bit_exact_all_tiles(gpu, prec, m, n, k):
    A, B, C = inputs.sgemm_operands(m, n, k, seed=m * 3 + k, dist="int")
    ref = oracle.sgemm(A, B, C, 1.0, 1.0)
    for tile in gpu.tile_menu(prec):
        print(f"case: {prec} int {m}x{n}x{k} tile {tile}", flush=True)
        got = run(gpu, A, B, C, 1.0, 1.0, prec, tile=tile, pad=4)
        assert np.array_equal(got, ref), tile


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
@pytest.mark.parametrize("dist", ["uniform", "loguniform"])
def test_random_against_exact_and_split_aware(gpu, prec, dist):
    m, n, k = 320, 288, 456
    A, B, C = inputs.sgemm_operands(m, n, k, seed=2, dist=dist)
    alpha, beta = 1.0, 0.5
    exact = oracle.sgemm(A, B, C, alpha, beta)
    split = oracle.sgemm(A, B, C, alpha, beta, mode=prec)
    terms = 3 * k if prec == "bf16x3" else k
    bound = componentwise_bound(A, B, C, alpha, beta, terms, extra=2.0 ** -7 if prec == "bf16" else 0)
    for tile in gpu.tile_menu(prec):
        print(f"case: {prec} {dist} tile {tile}", flush=True)
        got = run(gpu, A, B, C, alpha, beta, prec, tile=tile)
        assert normwise(got, exact) <= BAR[prec], tile
        assert np.all(np.abs(got - split) <= bound), tile


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
def test_unaligned_and_padded(gpu, prec):
    A, B, C = inputs.sgemm_operands(190, 150, 130, seed=9, dist="int")
    ref = oracle.sgemm(A, B, C, 1.0, -2.0)
    for tile in gpu.tile_menu(prec):
        got = run(gpu, A, B, C, 1.0, -2.0, prec, tile=tile, pad=1, misalign=True)
        assert np.array_equal(got, ref), tile


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
def test_staged_equals_fused_bitwise(gpu, prec):
    """Same tile shape, same bf16 operands, same MFMA order: identical bits."""
    import torch

    A, B, C = inputs.sgemm_operands(700, 600, 333, seed=21)
    menu = gpu.tile_menu(prec)
    pairs = [(f, s) for f in menu for s in menu if f[5] == 2 and s[5] == 3 and f[:5] == s[:5]]
    assert pairs
    for fused, staged in pairs:
        dA, dB = to_dev(A), to_dev(B)
        c1, c2 = to_dev(C), to_dev(C)
        gpu.sgemm(dA, dB, c1, 1.5, 0.5, prec=prec, tile=fused)
        gpu.sgemm(dA, dB, c2, 1.5, 0.5, prec=prec, tile=staged)
        torch.cuda.synchronize()
        assert torch.equal(c1, c2), (fused, staged)


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
def test_beta_zero_ignores_nan_c(gpu, prec):
    A, B, C = inputs.sgemm_operands(100, 90, 80, seed=3)
    C[:] = np.nan
    got = run(gpu, A, B, C, 1.0, 0.0, prec)
    ref = oracle.sgemm(A, B, None, 1.0, 0.0)
    assert np.all(np.isfinite(got)) and normwise(got, ref) <= BAR[prec]


# ---------------------------------------------------------------------------
# 8192^3 in the default launch configuration: sampled entries.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dist", ["uniform", "loguniform"])
def test_full_size_8192_sampled(gpu, dist):
    import torch

    n = 8192
    A, B, C = inputs.sgemm_operands(n, n, n, seed=2, dist=dist)
    dA, dB = to_dev(A), to_dev(B)
    rng = np.random.default_rng(17)
    rows = np.concatenate([rng.integers(0, n, 600), [0, n - 1]])
    cols = np.concatenate([rng.integers(0, n, 600), [n - 1, 0]])
    for prec in ("bf16", "bf16x3"):
        print(f"case: {prec} 8192^3 {dist}", flush=True)
        dC = torch.empty((n, n), device="cuda", dtype=torch.float32)
        gpu.sgemm(dA, dB, dC, 1.0, 0.0, prec=prec)
        torch.cuda.synchronize()
        got = dC[torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()].cpu().numpy()
        del dC
        exact = oracle.sgemm_entries(A, B, None, 1.0, 0.0, rows, cols)
        split = oracle.sgemm_entries(A, B, None, 1.0, 0.0, rows, cols, mode=prec)
        assert normwise(got, exact) <= BAR[prec], prec
        ab = (np.abs(A[rows].astype(np.float64)) * np.abs(B[:, cols].T.astype(np.float64))).sum(axis=1)
        terms = 3 * n if prec == "bf16x3" else n
        bound = 2 * (terms + 2) * 2.0 ** -24 * ab * (1 + 2.0 ** -7)
        assert np.all(np.abs(got - split) <= bound), prec


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
@pytest.mark.parametrize("m,n,k", [(1536, 1536, 1024), (4096, 4096, 256)])
def test_default_tile_is_staged_for_large_products(gpu, prec, m, n, k):
    """With no tile and no autotuned entry, a product of at least 2^31
    multiply-adds runs a staged tile (through a workspace): the first one
    when it gives at least 256 tiles, else 128 x 128 x 64 with 64 x 32
    leaves -- the same bits as naming that tile, and within the precision's
    bound."""
    import torch

    gpu.autotune_clear()
    A, B, C = inputs.sgemm_operands(m, n, k, seed=37)
    first = [t for t in gpu.tile_menu(prec) if t[5] == 3][0]
    whole = -(-m // first[0]) * -(-n // first[1]) >= 256
    staged = first if whole else (128, 128, 64, 64, 32, 3)
    assert whole == (m == 4096)
    print(f"case: default tile {prec} {m}x{n}x{k}", flush=True)
    C1, C2 = to_dev(C), to_dev(C)
    gpu.sgemm(to_dev(A), to_dev(B), C1, 1.0, 0.5, prec=prec)
    gpu.sgemm(to_dev(A), to_dev(B), C2, 1.0, 0.5, prec=prec, tile=staged)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
    ref = oracle.sgemm(A, B, C, 1.0, 0.5)
    assert normwise(to_host(C1), ref) <= (1e-2 if prec == "bf16" else 1e-5)
