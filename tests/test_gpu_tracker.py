"""GPU checks of the memory tracker for host-resident arrays (Sec. 2.3).

Results are compared with the oracle bit for bit (integer inputs); the copy
counters show which copies the tracker made, so the tests also pin that it
copies only stale data that a launch reads, and copies back only on request.
"""
import numpy as np
import pytest

import oracle
from paper_1611_00860_amd import inputs

pytestmark = pytest.mark.gpu


def delta(before, after):
    return {k: after[k] - before[k] for k in before}


def test_tracked_sgemm_copies_only_what_is_stale(gpu):
    import torch

    m, n, k = 300, 260, 200
    A, B, C = inputs.sgemm_operands(m, n, k, seed=41, dist="int")
    C0 = C.copy()
    for x in (A, B, C):
        gpu.track(x)
    try:
        c0 = gpu.tracker_counters()
        gpu.sgemm_tracked(A, B, C, 1.0, 1.0)
        d = delta(c0, gpu.tracker_counters())
        assert d["h2d_copies"] == 3 and d["d2h_copies"] == 0  # A, B in; C in out with beta != 0
        assert np.array_equal(C, C0)  # host C untouched until requested
        st = gpu.tracked_state(C)
        assert st["on_device"] and not st["on_host"]
        # a second launch on the same arrays copies nothing
        gpu.sgemm_tracked(A, B, C, 1.0, 1.0)
        d = delta(c0, gpu.tracker_counters())
        assert d["h2d_copies"] == 3 and d["launches"] == 2
        gpu.request(C)
        d = delta(c0, gpu.tracker_counters())
        assert d["d2h_copies"] == 1 and d["d2h_bytes"] == C.nbytes
        once = oracle.sgemm(A, B, C0, 1.0, 1.0)
        assert np.array_equal(C, oracle.sgemm(A, B, once.astype(np.float32), 1.0, 1.0))
        gpu.request(C)  # current on the host already: no copy
        assert delta(c0, gpu.tracker_counters())["d2h_copies"] == 1
    finally:
        for x in (A, B, C):
            gpu.untrack(x)
        torch.cuda.synchronize()


def test_tracked_chain_keeps_intermediate_on_device(gpu):
    """C1 = A B1 then C2 = C1 B2: C1 is never copied in or out unless requested."""
    import torch

    m, k, n1, n2 = 128, 96, 80, 72
    A, B1, _ = inputs.sgemm_operands(m, n1, k, seed=42, dist="int")
    _, B2, _ = inputs.sgemm_operands(1, n2, n1, seed=43, dist="int")  # B2: n1 x n2
    # |C1| <= 96 * 64 and |C2| <= 80 * 96 * 64 * 8 < 2^24: both exact in FP32
    C1 = np.full((m, n1), np.nan, dtype=np.float32)
    C2 = np.full((m, n2), np.nan, dtype=np.float32)
    for x in (A, B1, B2, C1, C2):
        gpu.track(x)
    try:
        c0 = gpu.tracker_counters()
        gpu.sgemm_tracked(A, B1, C1, 1.0, 0.0)   # C1 overwritten whole: its NaNs are not copied in
        gpu.sgemm_tracked(C1, B2, C2, 1.0, 0.0)  # C1's latest copy is on the device already
        d = delta(c0, gpu.tracker_counters())
        assert d["h2d_copies"] == 3  # A, B1, B2
        gpu.request(C2)
        assert delta(c0, gpu.tracker_counters())["d2h_copies"] == 1
        ref1 = oracle.sgemm(A, B1, None, 1.0, 0.0)
        assert np.array_equal(C2, oracle.sgemm(ref1.astype(np.float32), B2, None, 1.0, 0.0))
        assert np.all(np.isnan(C1))  # not requested: host copy is stale, untouched
        gpu.request(C1)
        assert np.array_equal(C1, ref1)
    finally:
        for x in (A, B1, B2, C1, C2):
            gpu.untrack(x)
        torch.cuda.synchronize()


def test_tracked_padded_c_keeps_the_gaps(gpu):
    """ldc > n with beta = 0: C's region is copied in, so the gap columns
    come back unchanged after the request."""
    import torch

    m, n, k = 70, 50, 40
    A, B, _ = inputs.sgemm_operands(m, n, k, seed=45, dist="int")
    Cfull = np.full((m, n + 6), 7.0, dtype=np.float32)
    C = Cfull[:, :n]
    for x in (A, B, Cfull):
        gpu.track(x)
    try:
        gpu.sgemm_tracked(A, B, C, 2.0, 0.0)
        gpu.request(Cfull)
        assert np.array_equal(C, oracle.sgemm(A, B, None, 2.0, 0.0))
        assert np.all(Cfull[:, n:] == 7.0)
    finally:
        for x in (A, B, Cfull):
            gpu.untrack(x)
        torch.cuda.synchronize()


def test_tracked_pinned_torch_tensors(gpu):
    import torch

    m, n, k = 256, 192, 128
    A, B, C = inputs.sgemm_operands(m, n, k, seed=46, dist="int")
    tA, tB, tC = (torch.from_numpy(x).pin_memory() for x in (A, B, C))
    for x in (tA, tB, tC):
        gpu.track(x)
    try:
        gpu.sgemm_tracked(tA, tB, tC, 1.0, -1.0)
        gpu.request(tC)
        assert np.array_equal(tC.numpy(), oracle.sgemm(A, B, C, 1.0, -1.0))
    finally:
        for x in (tA, tB, tC):
            gpu.untrack(x)
        torch.cuda.synchronize()


def test_tracked_launch_after_an_injected_allocation_failure(gpu, monkeypatch):
    """HPVM_FAULT_INJECT=alloc fails the first device copy's allocation: the
    launch reports a HIP error and leaves the table as it was; the next launch
    copies and computes as usual."""
    import torch

    A, B, C = inputs.sgemm_operands(70, 90, 50, seed=43, dist="int")
    C0 = C.copy()
    for x in (A, B, C):
        gpu.track(x)
    try:
        c0 = gpu.tracker_counters()
        monkeypatch.setenv("HPVM_FAULT_INJECT", "alloc")
        print("case: tracked launch with an injected allocation failure", flush=True)
        with pytest.raises(gpu.HpvmError) as ei:
            gpu.sgemm_tracked(A, B, C, 2.0, -1.0)
        assert ei.value.status == -3
        monkeypatch.delenv("HPVM_FAULT_INJECT")
        assert delta(c0, gpu.tracker_counters())["h2d_copies"] == 0
        assert all(gpu.tracked_state(x)["on_host"] and not gpu.tracked_state(x)["on_device"] for x in (A, B, C))
        gpu.sgemm_tracked(A, B, C, 2.0, -1.0)
        gpu.request(C)
        assert np.array_equal(C, oracle.sgemm(A, B, C0, 2.0, -1.0))
    finally:
        for x in (A, B, C):
            gpu.untrack(x)
        torch.cuda.synchronize()


def test_tracked_padded_a_region_goes_over_whole(gpu):
    """A is a view of a padded tracked region (lda > k): the region goes over
    once, gaps included, so a later launch that reads the padded rows whole
    sees the gap values; the result matches the oracle bit for bit."""
    import torch

    m, n, k = 1300, 260, 200
    A, B, C = inputs.sgemm_operands(m, n, k, seed=47, dist="int")
    Afull = np.full((m, k + 8), 7.0, dtype=np.float32)
    Afull[:, :k] = A
    Av = Afull[:, :k]
    C0 = C.copy()
    for x in (Afull, B, C):
        gpu.track(x)
    try:
        c0 = gpu.tracker_counters()
        print("case: tracked launch on a padded A", (m, n, k), flush=True)
        gpu.sgemm_tracked(Av, B, C, 1.0, -1.0)
        d = delta(c0, gpu.tracker_counters())
        assert d["h2d_copies"] == 3 and d["h2d_bytes"] == Afull.nbytes + B.nbytes + C.nbytes
        st = gpu.tracked_state(Afull)
        assert st["on_device"] and st["on_host"]
        gpu.sgemm_tracked(Av, B, C, 1.0, -1.0)  # everything resident: no copy
        assert delta(c0, gpu.tracker_counters())["h2d_copies"] == 3
        gpu.request(C)
        once = oracle.sgemm(A, B, C0, 1.0, -1.0)
        assert np.array_equal(C, oracle.sgemm(A, B, once.astype(np.float32), 1.0, -1.0))
        # the gap columns went over with the region: a product that reads the
        # padded rows whole sees them
        Cw = np.zeros((m, 4), dtype=np.float32)
        Bw = np.zeros((k + 8, 4), dtype=np.float32)
        Bw[k:, :] = 1.0
        for x in (Bw, Cw):
            gpu.track(x)
        try:
            gpu.sgemm_tracked(Afull, Bw, Cw, 1.0, 0.0)
            assert delta(c0, gpu.tracker_counters())["h2d_copies"] == 4  # Bw only
            gpu.request(Cw)
            assert np.all(Cw == 56.0)
        finally:
            for x in (Bw, Cw):
                gpu.untrack(x)
    finally:
        for x in (Afull, B, C):
            gpu.untrack(x)
        torch.cuda.synchronize()
