"""GPU checks of hpvm_sgemm_noalloc, the entry point that allocates nothing.

It must give exactly what hpvm_sgemm_ws gives with a caller workspace of
HPVM_NOALLOC_SCRATCH_BYTES: the same lowering (split contraction,
staged BF16 / bf16x3 planes) with the library's fixed per-device array as
the workspace.  Each case runs twice in a row, the second call smaller, so
that what the first call left in the array cannot leak into the second.
Every call goes through the C ABI with ctypes.
"""
import ctypes

import numpy as np
import pytest

import oracle
import paper_1611_00860_amd as hp
from paper_1611_00860_amd import _lib, inputs
from gpu_util import componentwise_bound, normwise, to_dev, to_host

pytestmark = pytest.mark.gpu

CAP = hp.NOALLOC_SCRATCH_BYTES


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def call_noalloc(lib, dA, dB, dC, alpha, beta, prec, tile=None):
    m, k = dA.shape
    n = dB.shape[1]
    t = ctypes.byref(_lib.Tile(*tile)) if tile else None
    return lib.hpvm_sgemm_noalloc(m, n, k, alpha, _ptr(dA), dA.stride(0), _ptr(dB), dB.stride(0), beta,
                                  _ptr(dC), dC.stride(0), hp.PREC[prec], t, _stream())


def call_ws(lib, dA, dB, dC, alpha, beta, prec, ws, ws_bytes, tile=None):
    m, k = dA.shape
    n = dB.shape[1]
    t = ctypes.byref(_lib.Tile(*tile)) if tile else None
    return lib.hpvm_sgemm_ws(m, n, k, alpha, _ptr(dA), dA.stride(0), _ptr(dB), dB.stride(0), beta,
                             _ptr(dC), dC.stride(0), hp.PREC[prec], t, _ptr(ws) if ws is not None else None,
                             ws_bytes, _stream())


def both(lib, A, B, C, alpha, beta, prec, tile=None):
    """C after hpvm_sgemm_ws (workspace of CAP bytes) and after hpvm_sgemm_noalloc."""
    import torch

    dA, dB = to_dev(A), to_dev(B)
    c_ws, c_na = to_dev(C), to_dev(C)
    ws = torch.full((CAP // 4,), float("nan"), device="cuda")  # garbage in the caller's workspace too
    rc = call_ws(lib, dA, dB, c_ws, alpha, beta, prec, ws, CAP, tile)
    assert rc == 0, hp.last_error()
    rc = call_noalloc(lib, dA, dB, c_na, alpha, beta, prec, tile)
    assert rc == 0, hp.last_error()
    torch.cuda.synchronize()
    return to_host(c_ws), to_host(c_na)


# (prec, first shape, second smaller shape, distribution): the FP32 shapes
# split their contraction; the first BF16 / bf16x3 shape takes the staged
# planes, the second (96 tiles of 128 x 128, k = 2048) the split.
CASES = [
    ("fp32", (1024, 1024, 4096), (512, 1024, 4096), "int"),
    ("fp32", (1024, 1024, 4096), (512, 1024, 4096), "uniform"),
    ("bf16", (2048, 2048, 2048), (1536, 1024, 2048), "uniform"),
    ("bf16x3", (2048, 2048, 2048), (1536, 1024, 2048), "uniform"),
]


@pytest.mark.parametrize("prec,first,second,dist", CASES)
def test_noalloc_matches_workspace_entry_twice(gpu, prec, first, second, dist):
    lib = gpu.load()
    for i, (m, n, k) in enumerate((first, second)):
        print(f"case: noalloc {prec} {dist} {m}x{n}x{k} call {i + 1}", flush=True)
        d = gpu.describe(m, n, k, prec, workspace_bytes=CAP)
        # the call really uses the array
        if prec == "fp32" or i == 1:
            assert d["splits"] > 1, d
        else:
            assert d["lowering_name"] == f"staged_{prec}", d
        A, B, C = inputs.sgemm_operands(m, n, k, seed=70 + i, dist=dist)
        alpha, beta = (2.0, -1.0) if dist == "int" else (1.0, 0.5)
        got_ws, got_na = both(lib, A, B, C, alpha, beta, prec)
        # same kernels, same order: the same bits
        assert np.array_equal(got_ws, got_na)
        ref = oracle.sgemm(A, B, C, alpha, beta)
        if dist == "int":
            assert np.array_equal(got_na, ref)
        else:
            bar = {"fp32": 1e-5, "bf16": 1e-2, "bf16x3": 1e-5}[prec]
            assert normwise(got_na, ref) <= bar
            if prec == "fp32":
                assert np.all(np.abs(got_na - ref) <= componentwise_bound(A, B, C, alpha, beta, k))


def test_noalloc_falls_back_when_planes_do_not_fit(gpu):
    """BF16 at 4096^3 would stage 64 MiB of planes: with no tile the call
    takes the choice a 32 MiB workspace allows, the same as hpvm_sgemm_ws's."""
    lib = gpu.load()
    m = n = k = 4096
    assert gpu.workspace_bytes(m, n, k, "bf16", gpu.describe(m, n, k, "bf16", workspace_bytes=1 << 40)["tile"]) > CAP
    d = gpu.describe(m, n, k, "bf16", workspace_bytes=CAP)
    assert d["lowering_name"] != "staged_bf16"
    print("case: noalloc bf16 4096^3 fallback", flush=True)
    A, B, C = inputs.sgemm_operands(m, n, k, seed=75)
    got_ws, got_na = both(lib, A, B, C, 1.0, 0.0, "bf16")
    assert np.array_equal(got_ws, got_na)
    rows = np.arange(0, m, 97)
    ref = oracle.sgemm(A[rows], B, C[rows], 1.0, 0.0)
    assert normwise(got_na[rows], ref) <= 1e-2


def test_noalloc_refuses_staged_tile_beyond_the_array(gpu):
    import torch

    lib = gpu.load()
    m = n = k = 4096
    staged = [t for t in gpu.tile_menu("bf16") if t[5] == 3][0]
    assert gpu.workspace_bytes(m, n, k, "bf16", staged) > CAP
    dA = torch.zeros((m, k), device="cuda")
    dB = torch.zeros((k, n), device="cuda")
    dC = torch.full((m, n), 7.0, device="cuda")
    rc = call_noalloc(lib, dA, dB, dC, 1.0, 0.0, "bf16", staged)
    assert rc == -4 and "scratch" in hp.last_error()
    torch.cuda.synchronize()
    assert bool((dC == 7.0).all())  # nothing ran
