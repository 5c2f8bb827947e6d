"""GPU parity of the streaming sgemm graph (launch with Stream = 1, push, pop).

Every pushed item is compared with the FP64 oracle: bit-exact on integer
inputs, within the FP32 bar on random ones.  The stream's bounded waits are
exercised from the host only (a tiny idle limit); every kernel exits normally.
"""
import ctypes
import time

import numpy as np
import pytest

import oracle
from paper_1611_00860_amd import inputs
from gpu_util import normwise, to_dev, to_host

pytestmark = pytest.mark.gpu


def item(m, n, k, seed, dist="int"):
    A, B, C = inputs.sgemm_operands(m, n, k, seed=seed, dist=dist)
    return A, B, C


def test_stream_items_bit_exact(gpu):
    import torch

    cases = [(300, 260, 200, 1.0, 1.0), (129, 257, 77, 1.0, -2.0), (1, 1, 1, 1.0, 0.5),
             (64, 520, 48, 2.0, 0.0), (256, 256, 64, 1.0, 1.0), (0, 40, 30, 1.0, 1.0),
             (40, 0, 30, 1.0, 1.0)]
    with gpu.SgemmStream(capacity=16, idle_ms=10000) as st:
        pushed = []
        for i, (m, n, k, a, b) in enumerate(cases):
            print(f"case: stream push {m}x{n}x{k} alpha={a} beta={b}", flush=True)
            A, B, C = item(m, n, k, seed=40 + i)
            dA, dB, dC = to_dev(A), to_dev(B), to_dev(C)
            seq = st.push(dA, dB, dC, a, b)
            pushed.append((seq, A, B, C, a, b))
        for seq, A, B, C, a, b in pushed:
            got_seq, dC = st.pop()
            assert got_seq == seq
            ref = oracle.sgemm(A, B, C if b != 0 else None, a, b)
            assert np.array_equal(to_host(dC), ref), (seq, A.shape, B.shape)
        info = st.info()
        assert info["pushed"] == info["popped"] == len(cases) and info["running"] == 1
        # default residency: two workgroups per CU
        assert info["grid"] == 2 * torch.cuda.get_device_properties(0).multi_processor_count


def test_stream_alpha_zero_null_operands_and_k_zero(gpu):
    """alpha == 0 or k == 0: C <- beta C without reading A or B (NULL here),
    on a tile-aligned item that would otherwise take the unmasked main loop."""
    with gpu.SgemmStream(capacity=4, idle_ms=10000) as st:
        _, _, C = item(256, 256, 64, seed=50)
        dC = to_dev(C)
        st.push(None, None, dC, alpha=0.0, beta=0.5, k=64)
        _, _, C2 = item(256, 128, 1, seed=51)
        C2[:] = np.nan
        dC2 = to_dev(C2)
        st.push(None, None, dC2, alpha=1.0, beta=0.0, k=0)
        st.pop()
        st.pop()
        assert np.array_equal(to_host(dC), 0.5 * C.astype(np.float64))
        assert np.count_nonzero(to_host(dC2)) == 0


def test_stream_queue_full_order_and_overlap(gpu):
    with gpu.SgemmStream(capacity=3, idle_ms=10000) as st:
        data = [item(96, 80, 40, seed=60 + i) for i in range(5)]
        dev = [tuple(to_dev(x) for x in d) for d in data]
        for i in range(3):
            assert st.push(*dev[i], 1.0, 1.0) == i
        with pytest.raises(gpu.HpvmError) as ei:
            st.push(*dev[3], 1.0, 1.0)
        assert ei.value.status == -6  # HPVM_QUEUE_FULL
        assert st.pop()[0] == 0
        # an item whose A is (a view of) the C of an item in flight is refused
        with pytest.raises(gpu.HpvmError) as ei:
            st.push(dev[1][2][:, :40], dev[3][1][:40], dev[3][2], 1.0, 1.0)
        assert ei.value.status == -1 and "in-flight" in gpu.last_error()
        assert st.push(*dev[3], 1.0, 1.0) == 3
        assert [st.pop()[0] for _ in range(3)] == [1, 2, 3]
        with pytest.raises(gpu.HpvmError) as ei:
            st.pop(timeout_ms=0)
        assert ei.value.status == -1  # nothing in flight
        for (A, B, C), (_, _, dC) in zip(data[:4], dev[:4]):
            assert np.array_equal(to_host(dC), oracle.sgemm(A, B, C, 1.0, 1.0))


def test_stream_close_drains_unpopped_items(gpu):
    import torch

    st = gpu.SgemmStream(capacity=8, idle_ms=10000)
    data = [item(200, 150, 100, seed=70 + i) for i in range(8)]
    dev = [tuple(to_dev(x) for x in d) for d in data]
    for d in dev:
        st.push(*d, 1.0, 1.0)
    stale = st._h.value
    st.close()
    torch.cuda.synchronize()
    for (A, B, C), (_, _, dC) in zip(data, dev):
        assert np.array_equal(to_host(dC), oracle.sgemm(A, B, C, 1.0, 1.0))
    # the registry refuses the closed handle without dereferencing it
    assert gpu.load().hpvm_stream_close(ctypes.c_void_p(stale), 0) == -5


def test_stream_idle_limit_ends_the_stream(gpu):
    st = gpu.SgemmStream(capacity=4, idle_ms=20)
    _, _, C = item(64, 64, 16, seed=80)
    A, B, _ = item(64, 64, 16, seed=81)
    deadline = time.time() + 10
    while st.info()["running"] and time.time() < deadline:
        time.sleep(0.02)
    info = st.info()
    assert info["running"] == 0 and info["idle_ended"] == 1
    with pytest.raises(gpu.HpvmError) as ei:
        st.push(to_dev(A), to_dev(B), to_dev(C), 1.0, 0.0)
    assert ei.value.status == -8  # HPVM_STREAM_ENDED
    st.close()


def test_stream_equals_single_launch_bitwise(gpu):
    """The persistent kernel runs the same tile code as a single launch of the
    same tile shape, so the bits agree."""
    import torch

    shapes = [(512, 384, 256), (200, 100, 300), (64, 700, 64)]
    with gpu.SgemmStream(capacity=8, idle_ms=10000) as st:
        for i, (m, n, k) in enumerate(shapes):
            A, B, C = item(m, n, k, seed=90 + i, dist="uniform")
            dA, dB = to_dev(A), to_dev(B)
            c1, c2 = to_dev(C), to_dev(C)
            plan = gpu.GroupedPlan([dA], [dB], [to_dev(C)], [0.75], [0.5])  # same cost model -> same shape
            tile = plan.instance_tile(0)
            plan.destroy()
            st.push(dA, dB, c1, 0.75, 0.5)
            st.pop()
            gpu.sgemm(dA, dB, c2, 0.75, 0.5, tile=tile)
            # a device-wide synchronize would wait for the resident kernel
            torch.cuda.current_stream().synchronize()
            assert torch.equal(c1, c2), (m, n, k, tile)


def test_stream_many_random_items(gpu):
    """300 items of log-uniform sizes, pushed with pops whenever the ring is full."""
    import torch

    rng = np.random.default_rng(5)
    dims = np.clip(np.round(np.exp(rng.uniform(np.log(16), np.log(512), (300, 3))) / 16) * 16, 16, 512).astype(int)
    data, dev, done = [], [], []
    with gpu.SgemmStream(capacity=32, idle_ms=10000) as st:
        for i, (m, n, k) in enumerate(dims):
            A, B, C = inputs.sgemm_operands(int(m), int(n), int(k), seed=1000 + i)
            d = (to_dev(A), to_dev(B), to_dev(C))
            while True:
                try:
                    st.push(*d, 1.25, 0.5)
                    break
                except gpu.HpvmError as e:
                    if e.status != -6:
                        raise
                    done.append(st.pop()[0])
            data.append((A, B, C))
            dev.append(d)
        while st.info()["popped"] < len(dims):
            done.append(st.pop()[0])
    assert done == list(range(len(dims)))
    torch.cuda.synchronize()
    worst = 0.0
    for (A, B, C), (_, _, dC) in zip(data, dev):
        worst = max(worst, normwise(to_host(dC), oracle.sgemm(A, B, C, 1.25, 0.5)))
    assert worst <= 1e-5, worst


def test_stream_full_ring_of_slots_wraps(gpu):
    """The largest ring (4096 slots, whose indices fill the ticket map's slot
    bits) held full, then wrapped: 4296 one-tile items sharing A and B, each
    with its own C, all bit-exact, popped in push order."""
    import torch

    cap, count, m, n, k = 4096, 4296, 32, 32, 16
    A, B, _ = inputs.sgemm_operands(m, n, k, seed=60, dist="int")
    dA, dB = to_dev(A), to_dev(B)
    Cs = torch.arange(count, dtype=torch.float32, device="cuda").view(count, 1, 1).repeat(1, m, n)
    done = []
    print(f"case: stream of {count} items through {cap} slots", flush=True)
    with gpu.SgemmStream(capacity=cap, idle_ms=10000) as st:
        for i in range(count):
            if st.in_flight == cap:
                done.append(st.pop()[0])
            assert st.push(dA, dB, Cs[i], 1.0, 1.0) == i
        while st.in_flight:
            done.append(st.pop()[0])
    assert done == list(range(count))
    ab = oracle.sgemm(A, B, None, 1.0, 0.0)
    got = to_host(Cs)
    for i in range(count):
        assert np.array_equal(got[i], ab + np.float32(i)), i


def test_stream_refuses_an_item_larger_than_the_ticket_window(gpu):
    """An item needing more tiles than the stream can hold in flight is refused
    at push (its pointers are never used: the check comes first)."""
    from paper_1611_00860_amd import _lib

    with gpu.SgemmStream(capacity=4, idle_ms=10000) as st:
        fake = 1 << 44
        n = 70000  # ceil(70000 / 128)^2 > 2^18 tiles of 128 x 128
        d = _lib.SgemmDesc(n, n, 1, 1.0, 0.0, fake, 1, fake + (1 << 40), n, fake + (2 << 40), n)
        rc = gpu.load().hpvm_stream_push(st._h, ctypes.byref(d), None)
        assert rc == -2 and "tiles" in gpu.last_error()
        assert st.info()["pushed"] == 0


def test_open_after_an_injected_allocation_failure(gpu, monkeypatch):
    """HPVM_FAULT_INJECT=alloc fails the stream's device counters after its
    host ring, stream and event exist: the open reports a HIP error, releases
    them, and the next open works."""
    import torch

    monkeypatch.setenv("HPVM_FAULT_INJECT", "alloc")
    print("case: stream open with an injected allocation failure", flush=True)
    with pytest.raises(gpu.HpvmError) as ei:
        gpu.SgemmStream(capacity=8, idle_ms=2000)
    assert ei.value.status == -3 and "stream open" in gpu.last_error()
    monkeypatch.delenv("HPVM_FAULT_INJECT")
    A, B, C = item(64, 96, 32, seed=77)
    with gpu.SgemmStream(capacity=8, idle_ms=10000) as st:
        dA, dB, dC = to_dev(A), to_dev(B), to_dev(C)
        st.push(dA, dB, dC, 1.0, 1.0)
        _, out = st.pop()
    torch.cuda.synchronize()
    assert np.array_equal(to_host(out), oracle.sgemm(A, B, C, 1.0, 1.0))
