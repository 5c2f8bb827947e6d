"""GPU parity of the grouped persistent launch and its HIP graph (needs an MI355X)."""
import numpy as np
import pytest

import oracle
from paper_1611_00860_amd import inputs
from gpu_util import componentwise_bound, normwise, to_dev, to_host

pytestmark = pytest.mark.gpu


def small_batch(seed, dist="int", count=40):
    """Ragged shapes (not multiples of 16), mixed scalars and degenerate cases."""
    rng = np.random.default_rng(seed)
    shapes, alphas, betas = [], [], []
    for i in range(count):
        m, n, k = (int(v) for v in rng.integers(1, 300, size=3))
        shapes.append((m, n, k))
        alphas.append(float(rng.choice([1.0, -2.0, 0.5])))
        betas.append(float(rng.choice([0.0, 1.0, -0.5])))
    shapes[3] = (0, 17, 5)      # empty
    shapes[4] = (33, 65, 0)     # k = 0: C <- beta C
    alphas[5] = 0.0             # alpha = 0: C <- beta C, A and B unread
    shapes[6] = (1, 1, 1)
    ops = [inputs.sgemm_operands(m, n, k, seed=seed * 1000 + i, dist=dist) for i, (m, n, k) in enumerate(shapes)]
    return shapes, alphas, betas, ops


def device_batch(ops, betas):
    As, Bs, Cs = [], [], []
    for (A, B, C), b in zip(ops, betas):
        Cd = C.copy()
        if b == 0.0 and Cd.size:
            Cd[:] = np.nan  # beta = 0 must not read C
        As.append(to_dev(A, pad=2))
        Bs.append(to_dev(B, pad=1))
        Cs.append(to_dev(Cd, pad=3))
    return As, Bs, Cs


def reference(ops, alphas, betas):
    return [oracle.sgemm(A, B, C if b != 0 else None, a, b) for (A, B, C), a, b in zip(ops, alphas, betas)]


def test_grouped_integers_bit_exact(gpu):
    import torch

    shapes, alphas, betas, ops = small_batch(1)
    As, Bs, Cs = device_batch(ops, betas)
    plan = gpu.GroupedPlan(As, Bs, Cs, alphas, betas)
    print("case: grouped int batch", plan.info(), flush=True)
    plan.run()
    torch.cuda.synchronize()
    for i, (got, ref) in enumerate(zip(Cs, reference(ops, alphas, betas))):
        assert np.array_equal(to_host(got), ref), i
    plan.destroy()


def test_grouped_uniform_within_bound(gpu):
    import torch

    shapes, alphas, betas, ops = small_batch(2, dist="uniform")
    As, Bs, Cs = device_batch(ops, betas)
    plan = gpu.GroupedPlan(As, Bs, Cs, alphas, betas)
    plan.run()
    torch.cuda.synchronize()
    for i, ((A, B, C), a, b, got, ref) in enumerate(zip(ops, alphas, betas, Cs, reference(ops, alphas, betas))):
        g = to_host(got)
        if g.size:
            assert np.all(np.abs(g - ref) <= componentwise_bound(A, B, C, a, b, A.shape[1])), i
    plan.destroy()


@pytest.mark.parametrize("shape_idx", [0, 1, 2, 3])
def test_grouped_matches_single_launch_bitwise(gpu, shape_idx):
    import torch

    tile = gpu.grouped_menu()[shape_idx]
    shapes, alphas, betas, ops = small_batch(3, dist="uniform", count=12)
    As, Bs, Cs = device_batch(ops, betas)
    Cs_single = [c.clone() for c in Cs]
    plan = gpu.GroupedPlan(As, Bs, Cs, alphas, betas, tile=tile)
    plan.run()
    for A, B, C, a, b in zip(As, Bs, Cs_single, alphas, betas):
        if C.numel():
            gpu.sgemm(A, B, C, a, b, tile=tile)
    torch.cuda.synchronize()
    for i, (g, s) in enumerate(zip(Cs, Cs_single)):
        assert torch.equal(torch.nan_to_num(g, nan=7.0), torch.nan_to_num(s, nan=7.0)), i
    plan.destroy()


def test_grouped_dma_interior_tiles_bit_exact(gpu):
    """Aligned instances whose k is a multiple of 16 run their interior
    128 x 128 tiles on the DMA-fed loop and their edge tiles on the masked
    one (k = 40: every tile masked): integer inputs stay exact, and the bits
    equal single launches of the same tile shape, whose loop accumulates
    every output in the same k order."""
    import torch

    shapes = [(256, 256, 64), (300, 260, 48), (384, 128, 160), (130, 520, 32), (128, 128, 16), (512, 256, 40)]
    alphas = [1.0, -2.0, 0.5, 1.0, 2.0, 1.0]
    betas = [0.0, 1.0, -0.5, 1.0, 0.0, 0.5]
    ops = [inputs.sgemm_operands(m, n, k, seed=500 + i, dist="int") for i, (m, n, k) in enumerate(shapes)]
    As = [to_dev(A) for A, _, _ in ops]
    Bs = [to_dev(B) for _, B, _ in ops]
    Cs = [to_dev(C) for _, _, C in ops]
    Cs_single = [to_dev(C) for _, _, C in ops]
    tile = gpu.grouped_menu()[0]
    print(f"case: grouped dma interior tiles, tile {tile}", flush=True)
    plan = gpu.GroupedPlan(As, Bs, Cs, alphas, betas, tile=tile)
    plan.run()
    for A, B, C, a, b in zip(As, Bs, Cs_single, alphas, betas):
        gpu.sgemm(A, B, C, a, b, tile=tile)
    torch.cuda.synchronize()
    for i, ((A, B, C), a, b) in enumerate(zip(ops, alphas, betas)):
        assert np.array_equal(to_host(Cs[i]), oracle.sgemm(A, B, C, a, b)), shapes[i]
        assert torch.equal(Cs[i], Cs_single[i]), shapes[i]
    plan.destroy()


def test_grouped_permutation_invariant(gpu):
    import torch

    shapes, alphas, betas, ops = small_batch(4, dist="uniform", count=24)
    As, Bs, Cs = device_batch(ops, betas)
    perm = np.random.default_rng(0).permutation(len(As))
    Cp = [Cs[i].clone() for i in perm]
    plan = gpu.GroupedPlan(As, Bs, Cs, alphas, betas)
    plan_p = gpu.GroupedPlan([As[i] for i in perm], [Bs[i] for i in perm], Cp,
                             [alphas[i] for i in perm], [betas[i] for i in perm])
    plan.run()
    plan_p.run()
    torch.cuda.synchronize()
    for j, i in enumerate(perm):
        assert torch.equal(Cs[i], Cp[j]), i
    plan.destroy()
    plan_p.destroy()


def test_graph_replays_match_eager(gpu):
    """Replays with eager work and synchronisations between them."""
    import torch

    shapes, alphas, betas, ops = small_batch(5, dist="uniform", count=30)
    betas = [0.5 if b == 0 else b for b in betas]  # C is read: replays must restart from C0
    As, Bs, Cs = device_batch(ops, betas)
    C0 = [c.clone() for c in Cs]
    plan = gpu.GroupedPlan(As, Bs, Cs, alphas, betas)
    plan.run()
    torch.cuda.synchronize()
    eager = [c.clone() for c in Cs]
    stream = torch.cuda.Stream()
    graph = plan.capture(stream=stream)
    for rep in range(4):
        for c, c0 in zip(Cs, C0):
            c.copy_(c0)
        torch.cuda.synchronize()
        graph.launch(stream=stream)
        stream.synchronize()
        junk = torch.ones(1000, device="cuda").sum()  # unrelated eager work in between
        torch.cuda.synchronize()
        assert float(junk) == 1000.0
        for i, (c, e) in enumerate(zip(Cs, eager)):
            assert torch.equal(c, e), (rep, i)
    graph.destroy()
    plan.destroy()


def test_autotune_writes_only_scratch(gpu):
    import torch

    shapes, alphas, betas, ops = small_batch(6, dist="uniform", count=20)
    As, Bs, Cs = device_batch(ops, betas)
    before = [c.clone() for c in Cs]
    plan = gpu.GroupedPlan(As, Bs, Cs, alphas, betas)
    ms = plan.autotune(reps=2)
    torch.cuda.synchronize()
    assert ms > 0
    for i, (c, b) in enumerate(zip(Cs, before)):
        assert torch.equal(torch.nan_to_num(c, nan=7.0), torch.nan_to_num(b, nan=7.0)), i
    plan.run()
    torch.cuda.synchronize()
    for i, ((A, B, C), a, b, got, ref) in enumerate(zip(ops, alphas, betas, Cs, reference(ops, alphas, betas))):
        g = to_host(got)
        if g.size:
            assert np.all(np.abs(g - ref) <= componentwise_bound(A, B, C, a, b, A.shape[1])), i
    plan.destroy()


def test_grouped_512_config_autotuned_graph(gpu):
    """512 instances, dims log-uniform in [32, 2048] (multiples of 16), seed 3."""
    import torch

    dims, alphas, betas, rng = inputs.grouped_problem(512, seed=3)
    As_h, Bs_h, Cs_h = inputs.grouped_operands(dims, rng)
    As = [to_dev(x) for x in As_h]
    Bs = [to_dev(x) for x in Bs_h]
    Cs = [to_dev(x) for x in Cs_h]
    plan = gpu.GroupedPlan(As, Bs, Cs, alphas.tolist(), betas.tolist())
    ms = plan.autotune(reps=3)
    info = plan.info()
    print(f"case: grouped 512 autotuned {ms:.3f} ms/launch, {info}", flush=True)
    stream = torch.cuda.Stream()
    graph = plan.capture(stream=stream)
    graph.launch(stream=stream)
    stream.synchronize()
    rs = np.random.default_rng(9)
    for i in range(512):
        m, n, k = (int(v) for v in dims[i])
        rows = rs.integers(0, m, 24)
        cols = rs.integers(0, n, 24)
        got = Cs[i][torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()].cpu().numpy()
        ref = oracle.sgemm_entries(As_h[i], Bs_h[i], Cs_h[i], float(alphas[i]), float(betas[i]), rows, cols)
        assert normwise(got, ref) <= 1e-5, i
    graph.destroy()
    plan.destroy()
