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


# The last two run the DMA-fed tiles (at least one tile each way, k a whole
# number of slabs, n a multiple of 4): edge tiles moved inward, then whole.
SHAPES = [(300, 260, 200), (257, 129, 77), (1, 1, 1), (64, 520, 48), (300, 260, 96), (512, 384, 64)]


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
    bound = componentwise_bound(A, B, C, alpha, beta, terms)
    for tile in gpu.tile_menu(prec):
        print(f"case: {prec} {dist} tile {tile}", flush=True)
        got = run(gpu, A, B, C, alpha, beta, prec, tile=tile)
        assert normwise(got, exact) <= BAR[prec], tile
        assert np.all(np.abs(got - split) <= bound), tile


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
@pytest.mark.parametrize("m,n,k", [(512, 512, 4096), (1024, 512, 2048)])
def test_split_contraction(gpu, prec, m, n, k):
    """Products that 128 x 128 tiles leave CUs idle on take the DMA-fed
    tile's split contraction by default (with a workspace): integers exact,
    random inputs within the bound of the split-aware oracle, and the same
    bits as naming the tile."""
    d = gpu.describe(m, n, k, prec, workspace_bytes=1 << 30)
    assert d["splits"] > 1, d
    A, B, C = inputs.sgemm_operands(m, n, k, seed=31, dist="int")
    print(f"case: {prec} split {m}x{n}x{k} int, {d['splits']} slices", flush=True)
    assert np.array_equal(run(gpu, A, B, C, 2.0, -1.0, prec), oracle.sgemm(A, B, C, 2.0, -1.0))
    A, B, C = inputs.sgemm_operands(m, n, k, seed=32)
    print(f"case: {prec} split {m}x{n}x{k} uniform", flush=True)
    got = run(gpu, A, B, C, 1.0, 0.5, prec)
    assert np.array_equal(got, run(gpu, A, B, C, 1.0, 0.5, prec, tile=d["tile"]))
    assert normwise(got, oracle.sgemm(A, B, C, 1.0, 0.5)) <= BAR[prec]
    split = oracle.sgemm(A, B, C, 1.0, 0.5, mode=prec)
    bound = componentwise_bound(A, B, C, 1.0, 0.5, 3 * k if prec == "bf16x3" else k)
    assert np.all(np.abs(got - split) <= bound)


# ---------------------------------------------------------------------------
# The conversion itself, bit for bit.  With one nonzero column of A (or row
# of B) meeting ones, every output is a single product x * 1, exact in FP32:
# BF16 must give the oracle's round-to-nearest-even bf16(x), bf16x3 must give
# hi + lo of the oracle's split (also exact in FP32).  Truncating instead of
# rounding, rounding ties away from zero, or losing the lo part fails here.
# ---------------------------------------------------------------------------
def special_values(count, seed):
    """float32 values that decide a conversion: ties (to an even and to an
    odd neighbour), one bit either side of a tie, subnormals, the largest
    finite values (some round to infinity), zeros, then random bit patterns
    over the whole finite range, both signs."""
    bits = [0x3F808000, 0x3F818000, 0x3F808001, 0x3F807FFF, 0x3F818001, 0x3F817FFF,  # ties near 1
            0x40490FDB, 0x3EAAAAAB, 0x3DCCCCCD, 0x42F6E979, 0x4B7FFFFF, 0x4B800001,  # pi, 1/3, 0.1, 123.456, ...
            0x00000001, 0x00008000, 0x00018000, 0x00017FFF, 0x007FFFFF, 0x00400000,  # subnormals
            0x00808000, 0x00818000, 0x0080FFFF,                                       # smallest normals
            0x7F7FFFFF, 0x7F7F7FFF, 0x7F7F8000, 0x7F7E8000, 0x7F7F0000,               # largest finite
            0x00000000, 0x3F800000, 0x3F7FFFFF, 0x33800000, 0x33800001]
    bits += [b | 0x80000000 for b in bits]
    rng = np.random.default_rng(seed)
    rnd = rng.integers(0, 0x7F800000, count - len(bits), dtype=np.int64)
    rnd |= rng.integers(0, 2, rnd.shape[0], dtype=np.int64) << 31
    return np.concatenate([np.array(bits, dtype=np.uint32), rnd.astype(np.uint32)]).view(np.float32)


def conversion_expected(prec, x):
    if prec == "bf16":
        return oracle.bf16_round(x).astype(np.float64)
    hi, lo = oracle.bf16_split(x)
    # values whose hi rounds to infinity get lo = -hi: their sum is NaN, as
    # the products' sum is on the GPU
    with np.errstate(invalid="ignore"):
        return hi.astype(np.float64) + lo.astype(np.float64)


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
@pytest.mark.parametrize("k,p,w", [(1, 0, 72), (40, 0, 72), (40, 39, 72), (200, 131, 72), (32, 5, 260),
                                   (64, 63, 260)])
@pytest.mark.parametrize("side", ["A", "B"])
def test_conversion_is_rne_bit_exact_all_tiles(gpu, prec, k, p, w, side):
    """w = 260 with k a whole number of slabs: the DMA-fed tiles convert
    FP32 fragments read from LDS (the other sizes take their fallback)."""
    import torch

    vals = special_values(700, seed=k + p)
    if side == "A":  # column p of A holds the values, row p of B is ones
        m, n = vals.shape[0], w
        A = np.zeros((m, k), np.float32)
        A[:, p] = vals
        B = np.zeros((k, n), np.float32)
        B[p, :] = 1.0
        expect = np.repeat(conversion_expected(prec, vals)[:, None], n, axis=1)
    else:  # row p of B holds the values, column p of A is ones
        m, n = w, vals.shape[0]
        A = np.zeros((m, k), np.float32)
        A[:, p] = 1.0
        B = np.zeros((k, n), np.float32)
        B[p, :] = vals
        expect = np.repeat(conversion_expected(prec, vals)[None, :], m, axis=0)
    dA, dB = to_dev(A), to_dev(B)
    for tile in gpu.tile_menu(prec):
        print(f"case: {prec} conversion side {side} k {k} p {p} tile {tile}", flush=True)
        dC = torch.full((m, n), float("nan"), device="cuda")
        gpu.sgemm(dA, dB, dC, 1.0, 0.0, prec=prec, tile=tile)
        torch.cuda.synchronize()
        got = to_host(dC)
        assert np.array_equal(np.isnan(got), np.isnan(expect)), tile
        bad = ~np.isnan(expect) & (got != expect)
        assert not bad.any(), (tile, vals[np.nonzero(bad.any(axis=1 if side == "A" else 0))[0][:5]])


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
@pytest.mark.parametrize("m,n,k", [(768, 512, 320), (520, 300, 96)])
def test_every_lowering_gives_the_same_bits(gpu, prec, m, n, k):
    """Every lowering of a precision sums the same bf16 products of each
    output in the same order (16-k steps in k order, bf16x3 as lo*hi, hi*lo,
    hi*hi): converting in the DMA-fed loop's fragment reads, in the
    register-staged copy into LDS, or in a pass before the GEMM gives the
    same bits on random inputs."""
    import torch

    A, B, C = inputs.sgemm_operands(m, n, k, seed=23)
    dA, dB = to_dev(A), to_dev(B)
    menu = gpu.tile_menu(prec)
    ref = None
    for tile in menu:
        print(f"case: {prec} {m}x{n}x{k} tile {tile}", flush=True)
        c = to_dev(C)
        gpu.sgemm(dA, dB, c, 1.5, 0.5, prec=prec, tile=tile)
        torch.cuda.synchronize()
        if ref is None:
            ref = c
        assert torch.equal(c, ref), tile


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
def test_default_tile_for_large_products(gpu, prec, m, n, k):
    """With no tile and no autotuned entry, a product of at least 2^31
    multiply-adds runs, for BF16, a staged tile (through a workspace): the
    first one when it gives at least 256 tiles, else 128 x 128 x 64 with
    64 x 32 leaves; bf16x3 the same when 256 x 256 tiles would not cover the
    CUs, else the menu's first (DMA-fed) tile, which converts in its own
    load path.  The same bits as naming that tile, and within the
    precision's bound."""
    import torch

    gpu.autotune_clear()
    A, B, C = inputs.sgemm_operands(m, n, k, seed=37)
    first = [t for t in gpu.tile_menu(prec) if t[5] == 3][0]
    whole = -(-m // first[0]) * -(-n // first[1]) >= 256
    staged = first if whole else (128, 128, 64, 64, 32, 3)
    assert whole == (m == 4096)
    expect = gpu.tile_menu(prec)[0] if (whole and prec == "bf16x3") else staged
    assert gpu.describe(m, n, k, prec, workspace_bytes=1 << 40)["tile"] == expect
    print(f"case: default tile {prec} {m}x{n}x{k}", flush=True)
    C1, C2 = to_dev(C), to_dev(C)
    gpu.sgemm(to_dev(A), to_dev(B), C1, 1.0, 0.5, prec=prec)
    gpu.sgemm(to_dev(A), to_dev(B), C2, 1.0, 0.5, prec=prec, tile=expect)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
    ref = oracle.sgemm(A, B, C, 1.0, 0.5)
    assert normwise(to_host(C1), ref) <= (1e-2 if prec == "bf16" else 1e-5)
