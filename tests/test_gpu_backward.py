"""GPU parity of the hand-written backward pass (needs an MI355X).

The oracle's closed-form gradient is pinned by exact FP64 central differences
(tests/test_oracle_pins.py); here the GPU backward is compared with it.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1611_00860_amd import inputs
from gpu_util import normwise, to_dev, to_host

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
BAR = {"fp32": 1e-5, "bf16": 1e-2, "bf16x3": 1e-5}


def dev_all(*xs):
    return [to_dev(x) for x in xs]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x3"])
def test_backward_16_against_oracle_gradient(gpu, prec):
    import torch

    A, B, C, G = inputs.backward_operands(16, 16, 16, seed=4, dist="dyadic")
    alpha, beta = 0.7, 0.3
    ref = oracle.sgemm_grad(A, B, C, G, alpha, beta)
    dA_, dB_, dC_, dG_ = dev_all(A, B, C, G)
    g = gpu.sgemm_backward(dA_, dB_, dC_, dG_, alpha, beta, prec=prec)
    torch.cuda.synchronize()
    tol = BAR[prec]
    for key in ("dA", "dB", "dC_in"):
        assert normwise(to_host(g[key]), ref[key]) <= tol, key
    assert abs(float(g["dalpha"]) - ref["dalpha"]) <= tol * abs(ref["dalpha"])
    assert abs(float(g["dbeta"]) - ref["dbeta"]) <= tol * abs(ref["dbeta"])
    if prec != "bf16":
        # dyadic inputs: the products are exact, only FP32 accumulation rounds
        bound = 2 * 18 * U32 * (np.abs(G.astype(np.float64)) @ np.abs(B.astype(np.float64)).T) * alpha
        assert np.all(np.abs(to_host(g["dA"]) - ref["dA"]) <= bound + 1e-30)


def test_backward_integers_exact_scalars(gpu):
    """Integer inputs: dA, dB, dC_in exact; the scalars' long FP32 sums to 1e-6."""
    import torch

    A, B, C, G = inputs.backward_operands(100, 90, 70, seed=8, dist="int")
    ref = oracle.sgemm_grad(A, B, C, G, 1.0, 2.0)
    g = gpu.sgemm_backward(*dev_all(A, B, C, G), 1.0, 2.0)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(g["dA"]), ref["dA"])
    assert np.array_equal(to_host(g["dB"]), ref["dB"])
    assert np.array_equal(to_host(g["dC_in"]), ref["dC_in"])
    assert math.isclose(float(g["dalpha"]), ref["dalpha"], rel_tol=1e-6)
    assert math.isclose(float(g["dbeta"]), ref["dbeta"], rel_tol=1e-6)


def test_backward_deterministic_and_partial_outputs(gpu):
    import torch

    A, B, C, G = inputs.backward_operands(300, 260, 200, seed=5)
    d = dev_all(A, B, C, G)
    g1 = gpu.sgemm_backward(*d, 0.7, 0.3)
    g2 = gpu.sgemm_backward(*d, 0.7, 0.3)
    only = gpu.sgemm_backward(*d, 0.7, 0.3, need=("dalpha",))
    only_b = gpu.sgemm_backward(*d, 0.7, 0.3, need=("dB", "dbeta"))
    torch.cuda.synchronize()
    for key in ("dA", "dB", "dC_in", "dalpha", "dbeta"):
        assert torch.equal(g1[key], g2[key]), key
    assert torch.equal(only["dalpha"], g1["dalpha"])
    assert torch.equal(only_b["dB"], g1["dB"]) and torch.equal(only_b["dbeta"], g1["dbeta"])


def test_backward_edge_cases(gpu):
    import torch

    A, B, C, G = inputs.backward_operands(40, 30, 20, seed=6)
    # beta = 0: dC_in is exactly zero, dbeta still <G, C_in>
    g = gpu.sgemm_backward(*dev_all(A, B, C, G), 1.5, 0.0)
    torch.cuda.synchronize()
    assert torch.count_nonzero(g["dC_in"]) == 0
    ref = oracle.sgemm_grad(A, B, C, G, 1.5, 0.0)
    assert math.isclose(float(g["dbeta"]), ref["dbeta"], rel_tol=1e-5)
    # alpha = 0: dA = dB = 0 but dalpha = <G, A B>
    g = gpu.sgemm_backward(*dev_all(A, B, C, G), 0.0, 1.0)
    torch.cuda.synchronize()
    assert torch.count_nonzero(g["dA"]) == 0 and torch.count_nonzero(g["dB"]) == 0
    assert math.isclose(float(g["dalpha"]), ref["dalpha"], rel_tol=1e-5)
    # k = 0: no products; dalpha = 0
    A0 = np.zeros((40, 0), dtype=np.float32)
    B0 = np.zeros((0, 30), dtype=np.float32)
    dA0 = torch.zeros((40, 0), device="cuda")
    dB0 = torch.zeros((0, 30), device="cuda")
    g = gpu.sgemm_backward(dA0, dB0, to_dev(C), to_dev(G), 1.0, 1.0)
    torch.cuda.synchronize()
    assert float(g["dalpha"]) == 0.0
    assert math.isclose(float(g["dbeta"]), ref["dbeta"], rel_tol=1e-5)
    del A0, B0


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("m,n,k", [(512, 512, 256), (256, 1024, 512)])
def test_backward_dma_split_integers(gpu, prec, m, n, k):
    """Whole tiles take the DMA-fed loop with the contraction split into
    slices (dA over n, dB over m) and one ordered pass summing the slices --
    BF16 converting the FP32 slabs in the fragment reads, with no conversion
    pass: integer inputs stay exact, and the DMA tile named explicitly or
    chosen by default gives the same bits."""
    import torch

    print(f"case: backward dma split {prec} {m}x{n}x{k}", flush=True)
    A, B, C, G = inputs.backward_operands(m, n, k, seed=m + n + k, dist="int")
    ref = oracle.sgemm_grad(A, B, C, G, 1.0, 2.0)
    d = dev_all(A, B, C, G)
    dma_tile = gpu.backward_menu(prec)[0]
    assert dma_tile[4] == 128
    g = gpu.sgemm_backward(*d, 1.0, 2.0, prec=prec, tile=dma_tile)
    g0 = gpu.sgemm_backward(*d, 1.0, 2.0, prec=prec)
    torch.cuda.synchronize()
    for key in ("dA", "dB", "dC_in"):
        assert np.array_equal(to_host(g[key]), ref[key]), key
        assert torch.equal(g[key], g0[key]), key
    # dalpha: a long FP32 sum of exact products, within its rounding bound
    terms = np.abs(A.astype(np.float64) * (G.astype(np.float64) @ B.astype(np.float64).T))
    assert abs(float(g["dalpha"]) - ref["dalpha"]) <= 4 * U32 * np.log2(terms.size) * terms.sum()
    assert float(g["dalpha"]) == float(g0["dalpha"])
    assert math.isclose(float(g["dbeta"]), ref["dbeta"], rel_tol=1e-6)


def test_backward_dma_output_subsets(gpu):
    """The DMA-fed FP32 backward runs both gradients in one launch when both
    are wanted (dalpha counts as wanting dA's pass) and each alone otherwise:
    every subset of outputs is exact on integer inputs, including dalpha
    without dA and dB without dC_in."""
    import torch

    m, n, k = 512, 512, 256
    A, B, C, G = inputs.backward_operands(m, n, k, seed=23, dist="int")
    ref = oracle.sgemm_grad(A, B, C, G, 1.0, 2.0)
    d = dev_all(A, B, C, G)
    tile = gpu.backward_menu("fp32")[0]
    for need in [("dA",), ("dB",), ("dalpha",), ("dB", "dalpha"), ("dA", "dB"), ("dA", "dbeta"),
                 ("dB", "dC_in", "dalpha", "dbeta")]:
        print(f"case: backward dma subset {need}", flush=True)
        g = gpu.sgemm_backward(*d, 1.0, 2.0, prec="fp32", tile=tile, need=need)
        torch.cuda.synchronize()
        for key in need:
            if key in ("dalpha", "dbeta"):
                assert math.isclose(float(g[key]), ref[key], rel_tol=1e-6), (need, key)
            else:
                assert np.array_equal(to_host(g[key]), ref[key]), (need, key)


def test_backward_threads_bitwise(gpu):
    """Two host threads on two streams, each calling the DMA-fed FP32
    backward repeatedly with its own workspace, get the single-threaded bits
    every time; each caller's stream alone orders its results."""
    import threading

    import torch

    m, n, k = 512, 512, 256
    A, B, C, G = inputs.backward_operands(m, n, k, seed=19)
    d = dev_all(A, B, C, G)
    ref = gpu.sgemm_backward(*d, 0.7, 0.3, prec="fp32")
    torch.cuda.synchronize()
    errors = []

    def worker(seed):
        try:
            st = torch.cuda.Stream()
            for i in range(4):
                with torch.cuda.stream(st):
                    g = gpu.sgemm_backward(*d, 0.7, 0.3, prec="fp32", stream=st)
                st.synchronize()
                for key in ("dA", "dB", "dC_in", "dalpha", "dbeta"):
                    if not torch.equal(g[key], ref[key]):
                        errors.append((seed, i, key))
        except Exception as exc:  # reported below
            errors.append((seed, repr(exc)))

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors


def test_backward_dma_misaligned_falls_back(gpu):
    """An operand off 16-byte alignment sends that gradient to the fallback tile."""
    import torch

    m, n, k = 256, 512, 256
    A, B, C, G = inputs.backward_operands(m, n, k, seed=77, dist="int")
    ref = oracle.sgemm_grad(A, B, C, G, 1.0, 0.5)
    dA_, dB_, dC_ = dev_all(A, B, C)
    dG_ = to_dev(G, 0, True)
    g = gpu.sgemm_backward(dA_, dB_, dC_, dG_, 1.0, 0.5, prec="fp32", tile=gpu.backward_menu("fp32")[0])
    torch.cuda.synchronize()
    assert np.array_equal(to_host(g["dA"]), ref["dA"])
    assert np.array_equal(to_host(g["dB"]), ref["dB"])


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x3"])
def test_backward_full_size_sampled(gpu, prec):
    """M = N = 4096, K = 1024, alpha = 0.7, beta = 0.3, G uniform, seed 4."""
    import torch

    m, n, k = 4096, 4096, 1024
    print(f"case: backward {prec} {m}x{n}x{k}", flush=True)
    A, B, C, G = inputs.backward_operands(m, n, k, seed=4)
    g = gpu.sgemm_backward(*dev_all(A, B, C, G), 0.7, 0.3, prec=prec)
    torch.cuda.synchronize()
    rng = np.random.default_rng(31)
    ra, ca = rng.integers(0, m, 400), rng.integers(0, k, 400)
    rb, cb = rng.integers(0, k, 400), rng.integers(0, n, 400)
    ref_a = oracle.grad_entries("dA", A, B, G, 0.7, ra, ca)
    ref_b = oracle.grad_entries("dB", A, B, G, 0.7, rb, cb)
    got_a = g["dA"][torch.from_numpy(ra).cuda(), torch.from_numpy(ca).cuda()].cpu().numpy()
    got_b = g["dB"][torch.from_numpy(rb).cuda(), torch.from_numpy(cb).cuda()].cpu().numpy()
    assert normwise(got_a, ref_a) <= BAR[prec]
    assert normwise(got_b, ref_b) <= BAR[prec]
    AB = oracle.sgemm(A, B, None, 1.0, 0.0)
    dalpha = float(np.sum(G.astype(np.float64) * AB))
    dbeta = float(np.sum(G.astype(np.float64) * C.astype(np.float64)))
    assert abs(float(g["dalpha"]) - dalpha) <= BAR[prec] * abs(dalpha)
    assert abs(float(g["dbeta"]) - dbeta) <= 1e-5 * abs(dbeta)
    assert torch.equal(g["dC_in"], 0.3 * to_dev(G)) or normwise(to_host(g["dC_in"]), 0.3 * G.astype(np.float64)) <= 1e-7


def test_autograd_function(gpu):
    import torch

    from paper_1611_00860_amd.autograd import SgemmFn

    A, B, C, G = inputs.backward_operands(70, 50, 40, seed=12)
    tA, tB, tC = (to_dev(x).contiguous().requires_grad_(True) for x in (A, B, C))
    alpha = torch.tensor(0.7, device="cuda", requires_grad=True)
    beta = torch.tensor(0.3, device="cuda", requires_grad=True)
    out = SgemmFn.apply(tA, tB, tC, alpha, beta, "fp32")
    fwd = oracle.sgemm(A, B, C, float(np.float32(0.7)), float(np.float32(0.3)))
    assert normwise(to_host(out), fwd) <= 1e-5
    out.backward(to_dev(G).contiguous())
    ref = oracle.sgemm_grad(A, B, C, G, float(np.float32(0.7)), float(np.float32(0.3)))
    assert normwise(to_host(tA.grad), ref["dA"]) <= 1e-5
    assert normwise(to_host(tB.grad), ref["dB"]) <= 1e-5
    assert normwise(to_host(tC.grad), ref["dC_in"]) <= 1e-6
    assert math.isclose(float(alpha.grad), ref["dalpha"], rel_tol=1e-5)
    assert math.isclose(float(beta.grad), ref["dbeta"], rel_tol=1e-5)
    # input C_in is left untouched by the forward (out of place)
    assert torch.equal(tC.detach(), to_dev(C))


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x3"])
def test_backward_every_tile_integers(gpu, prec):
    """Every backward tile, fused and staged: integer inputs are exact in all precisions."""
    import torch

    A, B, C, G = inputs.backward_operands(300, 260, 200, seed=13, dist="int")
    ref = oracle.sgemm_grad(A, B, C, G, 1.0, 2.0)
    d = dev_all(A, B, C, G)
    for tile in gpu.backward_menu(prec):
        print(f"case: backward {prec} tile {tile}", flush=True)
        g = gpu.sgemm_backward(*d, 1.0, 2.0, prec=prec, tile=tile)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(g["dA"]), ref["dA"]), tile
        assert np.array_equal(to_host(g["dB"]), ref["dB"]), tile
        assert np.array_equal(to_host(g["dC_in"]), ref["dC_in"]), tile
        assert math.isclose(float(g["dalpha"]), ref["dalpha"], rel_tol=1e-6), tile
        assert math.isclose(float(g["dbeta"]), ref["dbeta"], rel_tol=1e-6), tile


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
def test_backward_staged_outputs_and_layouts(gpu, prec):
    """Staged tiles convert G once for both products and take dC_in and the
    dbeta partials from that pass.  Integer inputs keep every output exact,
    for each subset of outputs (including the ones that skip the products)
    and for leading dimensions that rule out 16-byte units (ragged 301 x 259
    x 203, one padded and one misaligned operand)."""
    import torch

    m, n, k = 301, 259, 203
    A, B, C, G = inputs.backward_operands(m, n, k, seed=17, dist="int")
    ref = oracle.sgemm_grad(A, B, C, G, 1.0, 2.0)
    staged = [t for t in gpu.backward_menu(prec) if t[5] == 3]
    layouts = {
        "dense": dev_all(A, B, C, G),
        "padded": [to_dev(A, pad=3), to_dev(B, misalign=True), to_dev(C, pad=1), to_dev(G, pad=5)],
    }
    subsets = [("dA",), ("dB",), ("dC_in",), ("dbeta",), ("dalpha",), ("dA", "dbeta"), ("dB", "dC_in", "dalpha")]
    for tile in staged[:2]:
        for name, d in layouts.items():
            for need in subsets:
                print(f"case: backward staged {prec} tile {tile} {name} {need}", flush=True)
                g = gpu.sgemm_backward(*d, 1.0, 2.0, prec=prec, tile=tile, need=need)
                torch.cuda.synchronize()
                for key in need:
                    got = to_host(g[key]) if g[key].dim() else float(g[key])
                    if key in ("dalpha", "dbeta"):
                        assert math.isclose(got, ref[key], rel_tol=1e-6), (tile, name, need, key)
                    else:
                        assert np.array_equal(got, ref[key]), (tile, name, need, key)


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (7, 300, 65), (300, 7, 1), (63, 65, 257), (257, 64, 3)])
def test_backward_staged_small_and_ragged(gpu, prec, m, n, k):
    """Staged tiles pad every plane to 256-row, 64-deep blocks: sizes below
    one block, one past a block, and contractions of 1 keep every output exact
    on integer inputs (the padding must hold zeros)."""
    import torch

    A, B, C, G = inputs.backward_operands(m, n, k, seed=29, dist="int")
    ref = oracle.sgemm_grad(A, B, C, G, 1.0, 2.0)
    d = dev_all(A, B, C, G)
    tile = [t for t in gpu.backward_menu(prec) if t[5] == 3][0]
    print(f"case: backward staged {prec} {m}x{n}x{k} tile {tile}", flush=True)
    g = gpu.sgemm_backward(*d, 1.0, 2.0, prec=prec, tile=tile)
    torch.cuda.synchronize()
    for key in ("dA", "dB", "dC_in"):
        assert np.array_equal(to_host(g[key]), ref[key]), key
    assert math.isclose(float(g["dalpha"]), ref["dalpha"], rel_tol=1e-6, abs_tol=1e-6)
    assert math.isclose(float(g["dbeta"]), ref["dbeta"], rel_tol=1e-6, abs_tol=1e-6)


def test_backward_autotune_records_a_menu_tile(gpu):
    import torch

    A, B, C, G = inputs.backward_operands(512, 384, 256, seed=14)
    d = dev_all(A, B, C, G)
    tile, ms = gpu.autotune_backward(d[0], d[1], d[3], prec="bf16", reps=1)
    assert tuple(tile) in [tuple(t) for t in gpu.backward_menu("bf16")] and ms > 0
    g = gpu.sgemm_backward(*d, 0.7, 0.3, prec="bf16")  # takes the tuned tile
    torch.cuda.synchronize()
    ref = oracle.sgemm_grad(A, B, C, G, 0.7, 0.3)
    assert normwise(to_host(g["dA"]), ref["dA"]) <= 1e-2
    assert normwise(to_host(g["dB"]), ref["dB"]) <= 1e-2
