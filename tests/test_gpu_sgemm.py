"""GPU parity of the sgemm lowerings against the FP64 oracle (needs an MI355X)."""
import numpy as np
import pytest

import oracle
from paper_1611_00860_amd import inputs
from gpu_util import componentwise_bound, normwise, to_dev, to_host

pytestmark = pytest.mark.gpu

LITERAL = (32, 32, 32, 1, 1, 1)


def run(hp, A, B, C, alpha, beta, prec="fp32", tile=None, pad=0, misalign=False):
    import torch

    dA, dB, dC = (to_dev(x, pad, misalign) for x in (A, B, C))
    hp.sgemm(dA, dB, dC, alpha, beta, prec=prec, tile=tile)
    torch.cuda.synchronize()
    return to_host(dC)


# ---------------------------------------------------------------------------
# Literal lowering: 128^3, alpha = 1, beta = 0.5, internal tile 32 x 32, one
# output per leaf instance.
# ---------------------------------------------------------------------------
def test_literal_small_config(gpu):
    print("case: literal 128^3 seed 0", flush=True)
    A, B, C = inputs.sgemm_operands(128, 128, 128, seed=0)
    ref = oracle.sgemm(A, B, C, 1.0, 0.5)
    got = run(gpu, A, B, C, 1.0, 0.5, tile=LITERAL)
    assert normwise(got, ref) <= 1e-5
    assert np.all(np.abs(got - ref) <= componentwise_bound(A, B, C, 1.0, 0.5, 128))


def test_literal_integers_bit_exact(gpu):
    A, B, C = inputs.sgemm_operands(128, 128, 128, seed=0, dist="int")
    ref = oracle.sgemm(A, B, C, 1.0, 0.5)
    got = run(gpu, A, B, C, 1.0, 0.5, tile=LITERAL)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("m,n,k,tile", [(100, 70, 45, LITERAL), (65, 130, 33, (16, 16, 16, 1, 1, 1)),
                                        (33, 64, 17, (8, 32, 8, 1, 1, 1))])
def test_literal_ragged(gpu, m, n, k, tile):
    A, B, C = inputs.sgemm_operands(m, n, k, seed=1, dist="int")
    ref = oracle.sgemm(A, B, C, 2.0, -1.0)
    got = run(gpu, A, B, C, 2.0, -1.0, tile=tile, pad=3)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("m,n,k,tile", [(128, 128, 128, (32, 32, 0, 1, 1, 0)), (100, 70, 45, (16, 16, 0, 1, 1, 0)),
                                        (33, 64, 17, (8, 32, 0, 1, 1, 0))])
def test_untiled_graph_integers_bit_exact(gpu, m, n, k, tile):
    A, B, C = inputs.sgemm_operands(m, n, k, seed=2, dist="int")
    ref = oracle.sgemm(A, B, C, 2.0, -1.0)
    got = run(gpu, A, B, C, 2.0, -1.0, tile=tile, pad=3)
    assert np.array_equal(got, ref)


def test_untiled_graph_small_config(gpu):
    A, B, C = inputs.sgemm_operands(128, 128, 128, seed=0)
    ref = oracle.sgemm(A, B, C, 1.0, 0.5)
    got = run(gpu, A, B, C, 1.0, 0.5, tile=(32, 32, 0, 1, 1, 0))
    assert normwise(got, ref) <= 1e-5
    assert np.all(np.abs(got - ref) <= componentwise_bound(A, B, C, 1.0, 0.5, 128))


def test_root_launch_packed_args(gpu):
    """The paper's 88-byte root argument block drives the same lowering."""
    import torch

    A, B, C = inputs.sgemm_operands(128, 128, 128, seed=0)
    ref = oracle.sgemm(A, B, C, 1.0, 0.5)
    dA, dB, dC = (to_dev(x) for x in (A, B, C))
    gpu.launch_root(dA, dB, dC, 128, 1.0, 0.5, block=(32, 32), grid=(4, 4))
    gpu.wait()
    got = to_host(dC)
    assert normwise(got, ref) <= 1e-5
    # the same call with too small a byte extent for C is refused, C untouched
    before = dC.clone()
    with pytest.raises(gpu.HpvmError):
        gpu.launch_root(dA, dB, dC, 128, 1.0, 0.5, block=(32, 32), grid=(4, 4),
                        bytes_override=(128 * 128 * 4, 128 * 128 * 4, 100))
    torch.cuda.synchronize()
    assert torch.equal(before, dC)


# ---------------------------------------------------------------------------
# MFMA lowerings, every compiled tile
# ---------------------------------------------------------------------------
def _menu(prec):
    import paper_1611_00860_amd as hp

    return hp.tile_menu(prec)


SHAPES = [(300, 260, 200), (128, 128, 16), (1, 1, 1), (257, 129, 77), (64, 520, 36)]
# Whole tiles of every DMA-fed tile (m, n multiples of 256, k of 32): one
# K-slab, a few, and more slabs than LDS stages.
WHOLE_TILE_SHAPES = [(256, 256, 32), (512, 768, 96), (256, 512, 320)]


@pytest.mark.parametrize("m,n,k", SHAPES + WHOLE_TILE_SHAPES)
def test_f32_mfma_integers_bit_exact_all_tiles(gpu, m, n, k):
    A, B, C = inputs.sgemm_operands(m, n, k, seed=m + n + k, dist="int")
    ref = oracle.sgemm(A, B, C, 1.0, 1.0)
    for tile in _menu("fp32"):
        print(f"case: fp32 int {m}x{n}x{k} tile {tile}", flush=True)
        got = run(gpu, A, B, C, 1.0, 1.0, tile=tile, pad=4)
        assert np.array_equal(got, ref), tile


@pytest.mark.parametrize("m,n,k", SHAPES[:2] + WHOLE_TILE_SHAPES[1:2])
def test_f32_mfma_uniform_within_bound_all_tiles(gpu, m, n, k):
    A, B, C = inputs.sgemm_operands(m, n, k, seed=5)
    alpha, beta = 1.0, 0.5
    ref = oracle.sgemm(A, B, C, alpha, beta)
    bound = componentwise_bound(A, B, C, alpha, beta, k)
    for tile in _menu("fp32"):
        got = run(gpu, A, B, C, alpha, beta, tile=tile)
        assert normwise(got, ref) <= 1e-5, tile
        assert np.all(np.abs(got - ref) <= bound), tile


def test_f32_mfma_unaligned_operands(gpu):
    """Pointers off 16-byte alignment and odd leading dimensions take scalar loads."""
    A, B, C = inputs.sgemm_operands(190, 150, 130, seed=9, dist="int")
    ref = oracle.sgemm(A, B, C, 1.0, -2.0)
    got = run(gpu, A, B, C, 1.0, -2.0, pad=1, misalign=True)
    assert np.array_equal(got, ref)


def test_edge_cases(gpu):
    import torch

    A, B, C = inputs.sgemm_operands(70, 90, 50, seed=2)
    # alpha = 0: C <- beta C, A and B never read (NaN there must not leak)
    An = A.copy()
    An[0, 0] = np.nan
    got = run(gpu, An, B, C, 0.0, 0.25)
    assert np.array_equal(got, (np.float32(0.25) * C).astype(np.float64))
    # beta = 0: C never read (NaN in C is overwritten)
    Cn = np.full_like(C, np.nan)
    got = run(gpu, A, B, Cn, 1.0, 0.0)
    ref = oracle.sgemm(A, B, None, 1.0, 0.0)
    assert np.all(np.isfinite(got)) and normwise(got, ref) <= 1e-5
    # beta = 0 and alpha = 0: zeros
    got = run(gpu, A, B, Cn, 0.0, 0.0)
    assert np.array_equal(got, np.zeros_like(got))
    # k = 0: C <- beta C
    dA = torch.zeros((70, 0), device="cuda")
    dB = torch.zeros((0, 90), device="cuda")
    dC = to_dev(C)
    gpu.sgemm(dA, dB, dC, 1.0, 3.0)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(dC), (np.float32(3.0) * C).astype(np.float64))
    # m = 0 / n = 0: nothing happens
    e = torch.zeros((0, 5), device="cuda")
    gpu.sgemm(e, torch.zeros((5, 7), device="cuda"), torch.zeros((0, 7), device="cuda"), 1.0, 1.0)
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# Full sizes of the FP32 workload, in the launch configuration the benchmark
# times: sampled entries against the oracle's element-wise definition.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,n,k", [(4096, 4096, 4096), (8192, 4096, 2048)])
@pytest.mark.parametrize("beta", [0.0, 1.0])
def test_f32_full_size_sampled(gpu, m, n, k, beta):
    import torch

    print(f"case: fp32 full {m}x{n}x{k} beta {beta}", flush=True)
    A, B, C = inputs.sgemm_operands(m, n, k, seed=1)
    dA, dB, dC = (to_dev(x) for x in (A, B, C))
    gpu.sgemm(dA, dB, dC, 1.0, beta)
    torch.cuda.synchronize()
    got = dC.cpu().numpy()
    rng = np.random.default_rng(123)
    rows = np.concatenate([rng.integers(0, m, 1500), [0, m - 1, m - 1, 0]])
    cols = np.concatenate([rng.integers(0, n, 1500), [0, n - 1, 0, n - 1]])
    ref = oracle.sgemm_entries(A, B, C, 1.0, beta, rows, cols)
    g = got[rows, cols].astype(np.float64)
    assert normwise(g, ref) <= 1e-5
    ab = np.abs(A[rows].astype(np.float64)) * np.abs(B[:, cols].T.astype(np.float64))
    bound = 2 * (k + 2) * 2.0 ** -24 * ab.sum(axis=1) + 4 * 2.0 ** -24 * abs(beta) * np.abs(C[rows, cols])
    assert np.all(np.abs(g - ref) <= bound)


# ---------------------------------------------------------------------------
# DMA-fed FP32 tiles on problems that are not whole tiles: a tile that would
# cross the edge is moved inward and stores only the rows and columns it
# owns, so overlapped outputs are neither computed from outside the
# matrices nor given beta * C twice.
# ---------------------------------------------------------------------------
EDGE_SHAPES = [(300, 520, 96), (257, 260, 64), (511, 1000, 32), (256, 300, 2048), (1000, 256, 160)]


@pytest.mark.parametrize("m,n,k", EDGE_SHAPES)
def test_f32_dma_edge_tiles_integers(gpu, m, n, k):
    """Integer inputs, beta = 2: exact, with NaN-filled row padding (a read
    outside a matrix would poison the result) and, for beta = 0, a NaN-filled
    C that must be overwritten, never read."""
    dma = [t for t in gpu.tile_menu("fp32") if t[4] == 128]
    A, B, C = inputs.sgemm_operands(m, n, k, seed=41, dist="int")
    ref = oracle.sgemm(A, B, C, 1.0, 2.0)
    for tile in dma:
        print(f"case: fp32 dma edge {m}x{n}x{k} tile {tile}", flush=True)
        got = run(gpu, A, B, C, 1.0, 2.0, tile=tile, pad=4)
        assert np.array_equal(got, ref), tile
    nan_c = np.full_like(C, np.nan)
    got0 = run(gpu, A, B, nan_c, 1.0, 0.0, tile=dma[0], pad=4)
    assert np.array_equal(got0, oracle.sgemm(A, B, None, 1.0, 0.0))


def test_f32_dma_edge_tiles_match_whole_tile_bits(gpu):
    """Uniform inputs: every output of a ragged problem equals, bit for bit,
    the same output computed inside a whole-tile problem that holds it (an
    edge tile moved inward computes each of its outputs in the same order as
    any tile)."""
    import torch

    m, n, k = 300, 520, 96
    A, B, C = inputs.sgemm_operands(512, 768, k, seed=43)
    tile = gpu.tile_menu("fp32")[0]
    big = run(gpu, A, B, C, 1.0, 0.5, tile=tile)
    small = run(gpu, np.ascontiguousarray(A[:m]), B[:, :n].copy(), C[:m, :n].copy(), 1.0, 0.5, tile=tile)
    assert np.array_equal(small, big[:m, :n])
    ref = oracle.sgemm(np.ascontiguousarray(A[:m]), B[:, :n].copy(), C[:m, :n].copy(), 1.0, 0.5)
    assert normwise(small, ref) <= 1e-5


# ---------------------------------------------------------------------------
# Split contraction (hpvm_sgemm_ws): FP32 DMA-fed tiles on whole-tile
# problems whose tiles would not cover the CUs run as contraction slices
# whose partial sums are added, in slice order, by a second launch.
# ---------------------------------------------------------------------------
T256 = (256, 256, 32, 64, 128, 2)
T128X256 = (128, 256, 32, 32, 128, 2)
T128 = (128, 128, 32, 32, 128, 2)
SPLIT_CASES = [(1024, 1024, 4096, T256), (1024, 1024, 4096, T128X256), (1024, 1024, 4096, T128),
               (512, 2048, 2048, T128X256), (2048, 2048, 2048, T256), (1024, 1024, 1024, None)]


def sample_entries(m, n, count, seed):
    rng = np.random.default_rng(seed)
    rows = np.concatenate([rng.integers(0, m, count), [0, m - 1, m - 1, 0]])
    cols = np.concatenate([rng.integers(0, n, count), [0, n - 1, 0, n - 1]])
    return rows, cols


@pytest.mark.parametrize("m,n,k,tile", SPLIT_CASES)
def test_split_contraction_integers(gpu, m, n, k, tile):
    """Integer inputs: every partial sum is an integer below 2^24, so the
    result is exact whatever the slicing -- checked against the integer
    product on all outputs and the oracle on sampled ones, with NaN-filled
    row padding, and with beta = 0 on a NaN-filled C that is never read."""
    assert gpu.workspace_bytes(m, n, k, "fp32", tile) > 0
    print(f"case: fp32 split {m}x{n}x{k} tile {tile}", flush=True)
    A, B, C = inputs.sgemm_operands(m, n, k, seed=51, dist="int")
    # integers of at most 8 * 8 * k < 2^53: exact in float64 in any order
    product = A.astype(np.float64) @ B.astype(np.float64)
    assert np.abs(product).max() < 2 ** 24
    got = run(gpu, A, B, C, 1.0, 2.0, tile=tile, pad=4)
    assert np.array_equal(got, product + 2.0 * C.astype(np.float64))
    rows, cols = sample_entries(m, n, 300, 52)
    assert np.array_equal(got[rows, cols], oracle.sgemm_entries(A, B, C, 1.0, 2.0, rows, cols))
    got0 = run(gpu, A, B, np.full_like(C, np.nan), 1.0, 0.0, tile=tile)
    assert np.array_equal(got0, product)


@pytest.mark.parametrize("m,n,k,tile", SPLIT_CASES)
def test_split_contraction_uniform_within_bound(gpu, m, n, k, tile):
    print(f"case: fp32 split uniform {m}x{n}x{k} tile {tile}", flush=True)
    A, B, C = inputs.sgemm_operands(m, n, k, seed=53)
    got = run(gpu, A, B, C, 0.75, -0.5, tile=tile)
    rows, cols = sample_entries(m, n, 600, 54)
    ref = oracle.sgemm_entries(A, B, C, 0.75, -0.5, rows, cols)
    g = got[rows, cols].astype(np.float64)
    assert normwise(g, ref) <= 1e-5
    # each output: slices of k / s terms, then s partials, alpha and beta
    ab = np.abs(A[rows].astype(np.float64)) * np.abs(B[:, cols].T.astype(np.float64))
    bound = 0.75 * (k + 20) * 2.0 ** -24 * ab.sum(axis=1) + 4 * 2.0 ** -24 * 0.5 * np.abs(C[rows, cols])
    assert np.all(np.abs(g - ref) <= bound)


def test_split_contraction_without_workspace_runs_unsplit(gpu):
    """hpvm_sgemm (no workspace) with a DMA-fed tile on a problem the split
    would cover runs the single launch: the same result as the oracle."""
    import ctypes

    import torch

    m, n, k = 1024, 1024, 4096
    A, B, C = inputs.sgemm_operands(m, n, k, seed=55, dist="int")
    dA, dB, dC = (to_dev(x) for x in (A, B, C))
    lib = gpu.load()
    rc = lib.hpvm_sgemm(m, n, k, 1.0, ctypes.c_void_p(dA.data_ptr()), k, ctypes.c_void_p(dB.data_ptr()), n, 1.0,
                        ctypes.c_void_p(dC.data_ptr()), n, gpu.PREC["fp32"], gpu._tile(T128X256),
                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    torch.cuda.synchronize()
    product = A.astype(np.float64) @ B.astype(np.float64)  # exact: integers below 2^53
    assert np.array_equal(to_host(dC), product + C.astype(np.float64))


# ---------------------------------------------------------------------------
# 4096^3, beta = 1, in the launch configuration the benchmark times: every
# output against the oracle (normwise and componentwise).
# ---------------------------------------------------------------------------
def test_f32_4096_beta1_all_outputs(gpu):
    import torch

    n = 4096
    print("case: fp32 4096^3 beta 1, all outputs", flush=True)
    A, B, C = inputs.sgemm_operands(n, n, n, seed=1)
    dA, dB, dC = (to_dev(x) for x in (A, B, C))
    gpu.sgemm(dA, dB, dC, 1.0, 1.0)
    torch.cuda.synchronize()
    got = to_host(dC)
    del dA, dB, dC
    ref = oracle.sgemm(A, B, C, 1.0, 1.0)
    assert normwise(got, ref) <= 1e-5
    assert np.all(np.abs(got - ref) <= componentwise_bound(A, B, C, 1.0, 1.0, n))


# ---------------------------------------------------------------------------
# A stream that is not torch's current one: the scratch memory a call
# allocates for itself (here the split contraction's partial sums) must not
# be handed to other work on the current stream while that stream still
# uses it.
# ---------------------------------------------------------------------------
def test_split_on_a_side_stream_keeps_its_workspace(gpu):
    import torch

    m, n, k = 1024, 1024, 4096
    need = gpu.workspace_bytes(m, n, k, "fp32")
    assert need > 0  # the default tile splits this problem
    A, B, C = inputs.sgemm_operands(m, n, k, seed=57, dist="int")
    dA, dB, dC = (to_dev(x) for x in (A, B, C))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # keep the side stream busy so the split runs late
        x = torch.ones((4096, 4096), device="cuda")
        for _ in range(4):
            x = x @ x
    gpu.sgemm(dA, dB, dC, 1.0, 2.0, stream=side)  # the side stream is not made current
    # the current stream now allocates and fills memory of the workspace's size
    junk = torch.full((need // 4,), float("nan"), device="cuda")
    junk.add_(1.0)
    side.synchronize()
    torch.cuda.synchronize()
    product = A.astype(np.float64) @ B.astype(np.float64)  # integers: exact
    assert np.array_equal(to_host(dC), product + 2.0 * C.astype(np.float64))
    del x, junk


# ---------------------------------------------------------------------------
# The single-launch autotuner: it reads A and B only, records a tile of the
# menu, and a call with no tile then runs exactly that tile (with a
# workspace) or the recorded tile that needs none (without).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,n,k", [(1024, 1024, 4096), (2048, 2048, 1024)])
def test_autotune_records_a_menu_tile_and_uses_it(gpu, m, n, k):
    import torch

    print(f"case: autotune fp32 {m}x{n}x{k}", flush=True)
    gpu.autotune_clear()
    A, B, C = inputs.sgemm_operands(m, n, k, seed=59)
    dA, dB, dC = (to_dev(x) for x in (A, B, C))
    a0, b0, c0 = dA.clone(), dB.clone(), dC.clone()
    best, ms = gpu.autotune(dA, dB, "fp32", reps=2)
    torch.cuda.synchronize()
    assert torch.equal(dA, a0) and torch.equal(dB, b0) and torch.equal(dC, c0)
    menu = gpu.tile_menu("fp32")
    assert best in menu and ms > 0
    assert gpu.autotune_lookup(m, n, k, "fp32") == (best, 2)
    ws = gpu.workspace_bytes(m, n, k, "fp32")
    assert ws == gpu.workspace_bytes(m, n, k, "fp32", best)
    # the choice without a workspace never splits the contraction
    plain = gpu.describe(m, n, k, "fp32")
    assert plain["splits"] == 1 and plain["tile"] in menu
    if gpu.workspace_bytes(m, n, k, "fp32", plain["tile"]) > 0:
        assert plain["tile"] != best  # a split winner is not the no-workspace choice
    with_ws = gpu.describe(m, n, k, "fp32", workspace_bytes=ws)
    assert with_ws["tile"] == best
    ref = oracle.sgemm(A, B, C, 1.0, 0.5)
    for tile, wsarg in ((best, None), (plain["tile"], False)):
        c1, c2 = to_dev(C), to_dev(C)
        gpu.sgemm(dA, dB, c1, 1.0, 0.5, workspace=wsarg)
        gpu.sgemm(dA, dB, c2, 1.0, 0.5, tile=tile, workspace=wsarg)
        torch.cuda.synchronize()
        assert torch.equal(c1, c2), (tile, wsarg)
        assert normwise(to_host(c1), ref) <= 1e-5
    gpu.autotune_clear()


# ---------------------------------------------------------------------------
# A C of more than 2^31 elements (8.6 GB): every lowering addresses it with
# 64-bit offsets.  Integer inputs keep every product and sum exact, so the
# rows around element 2^31 and the last rows must match the oracle bit for
# bit; beta = 0 leaves C unread (it is never filled).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec,tile,workspace", [
    ("fp32", None, None),                       # DMA-fed 256 x 256, ragged n
    ("fp32", (128, 128, 16, 64, 64, 2), None),  # register-staged
    ("bf16", None, None),                       # staged planes (workspace)
    ("bf16", None, False),                      # DMA-fed, converting in the fragment reads
])
def test_offsets_past_2_31_elements(gpu, prec, tile, workspace):
    import torch

    m, n, k = (1 << 21) + 64, 1032, 32
    assert m * n > 2 ** 31
    rng = np.random.default_rng(41)
    A = inputs.draw(rng, (m, k), "int")
    B = inputs.draw(rng, (k, n), "int")
    dA, dB = to_dev(A), to_dev(B)
    dC = torch.empty((m, n), device="cuda")
    print(f"case: {prec} {m}x{n}x{k} tile {tile} workspace {workspace}", flush=True)
    gpu.sgemm(dA, dB, dC, 2.0, 0.0, prec=prec, tile=tile, workspace=workspace)
    torch.cuda.synchronize()
    rows = np.array([0, 1, 2 ** 31 // n - 1, 2 ** 31 // n, 2 ** 31 // n + 1, m - 65, m - 1])
    got = dC[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
    ref = oracle.sgemm(A[rows], B, None, 2.0, 0.0)
    assert np.array_equal(got, ref)
    del dC
    torch.cuda.empty_cache()
