"""A CPU emulator of the index math of the sgemm graph's GPU lowerings.

It restates, in numpy, how the kernels decompose C into SgemmInternal
instances (workgroup tiles), where each instance starts and which outputs it
owns, how the contraction is cut into slabs and slices, how the DMA feed
lays slabs out in LDS and which k a lane's MFMA fragment holds -- and checks
the properties the kernels rely on (every output written exactly once, every
k summed exactly once, layouts that are bijections and free of bank
conflicts), then runs the decomposition in FP32 against the FP64 oracle.  It
is test infrastructure, not the oracle: the oracle stays the plain
definition and shares none of this.  Where the library states the same
decisions (the grid of a launch, the slices of a split contraction), the
emulator's restatement is compared with it through the C ABI.  No GPU.
"""
import itertools

import numpy as np
import pytest

import oracle
import paper_1611_00860_amd as hp
from paper_1611_00860_amd import inputs

XCDS, GROUP_M = 8, 8


# --------------------------------------------------------------------------
# Internal instances -> workgroups: the XCD-aware order of the tile grid.
# --------------------------------------------------------------------------
def tile_coords(tiles_m, tiles_n, w):
    """Workgroup w's tile: XCD w mod 8 gets a contiguous run of the row-major
    order of groups of GROUP_M tile rows (column by column inside a group)."""
    total = tiles_m * tiles_n
    q, rem = divmod(total, XCDS)
    x = w % XCDS
    t = x * q + min(x, rem) + w // XCDS
    per_group = GROUP_M * tiles_n
    group = t // per_group
    first_m = group * GROUP_M
    gsize = min(tiles_m - first_m, GROUP_M)
    in_group = t - group * per_group
    return first_m + in_group % gsize, in_group // gsize


@pytest.mark.parametrize("tiles_m,tiles_n", [(1, 1), (3, 5), (16, 16), (32, 16), (9, 33), (17, 1), (1, 23), (64, 64)])
def test_tile_order_is_a_bijection_with_contiguous_xcd_runs(tiles_m, tiles_n):
    total = tiles_m * tiles_n
    got = [tile_coords(tiles_m, tiles_n, w) for w in range(total)]
    assert sorted(got) == [(i, j) for i in range(tiles_m) for j in range(tiles_n)]
    # the tiles of one XCD are a contiguous run of the order, so they share
    # A row panels and B column panels
    order = {}
    for w in range(total):
        tm, tn = got[w]
        g = tm // GROUP_M
        gs = min(tiles_m - g * GROUP_M, GROUP_M)
        order[w] = g * GROUP_M * tiles_n + tn * gs + (tm - g * GROUP_M)
    for x in range(XCDS):
        ts = sorted(order[w] for w in range(x, total, XCDS))
        assert ts == list(range(ts[0], ts[0] + len(ts))) if ts else True


# --------------------------------------------------------------------------
# DMA-fed tiles on ragged sizes: edge tiles computed from a corner moved
# inward, each storing only the outputs of its own place in the tile grid.
# --------------------------------------------------------------------------
def tile_corner(t_own, tile, size):
    return size - tile if t_own + tile > size else t_own


@pytest.mark.parametrize("TM,TN", [(256, 256), (128, 256), (128, 128)])
@pytest.mark.parametrize("m,n", [(256, 256), (300, 260), (1000, 1024), (257, 771), (128 * 3 + 1, 256)])
def test_moved_tiles_cover_every_output_once(TM, TN, m, n):
    if m < TM or n < TN:
        pytest.skip("the DMA-fed tile needs at least one tile each way")
    owner = np.zeros((m, n), dtype=np.int32)
    tiles_m, tiles_n = -(-m // TM), -(-n // TN)
    for tm, tn in itertools.product(range(tiles_m), range(tiles_n)):
        m_own, n_own = tm * TM, tn * TN
        m0, n0 = tile_corner(m_own, TM, m), tile_corner(n_own, TN, n)
        assert 0 <= m0 and m0 + TM <= m and 0 <= n0 and n0 + TN <= n  # every load in bounds
        rows = slice(max(m0, m_own), m0 + TM)
        cols = slice(max(n0, n_own), n0 + TN)
        owner[rows, cols] += 1
    assert np.all(owner == 1)


def test_moved_tiles_reproduce_the_definition_in_fp32():
    """The decomposition run in FP32 (each tile's outputs summed over k in
    order from its own corner, stored only where it owns them) equals the
    oracle exactly on integers and within the FP32 bound otherwise."""
    TM = TN = 128
    m, n, k = 300, 260, 48
    for dist in ("int", "uniform"):
        A, B, C = inputs.sgemm_operands(m, n, k, seed=5, dist=dist)
        out = np.full((m, n), np.nan, dtype=np.float32)
        for tm, tn in itertools.product(range(-(-m // TM)), range(-(-n // TN))):
            m0, n0 = tile_corner(tm * TM, TM, m), tile_corner(tn * TN, TN, n)
            acc = np.zeros((TM, TN), dtype=np.float32)
            for p in range(k):
                acc += np.outer(A[m0:m0 + TM, p], B[p, n0:n0 + TN]).astype(np.float32)
            tile = (np.float32(0.5) * C[m0:m0 + TM, n0:n0 + TN] + np.float32(2.0) * acc).astype(np.float32)
            rs, cs = max(m0, tm * TM) - m0, max(n0, tn * TN) - n0
            out[m0 + rs:m0 + TM, n0 + cs:n0 + TN] = tile[rs:, cs:]
        ref = oracle.sgemm(A, B, C, 2.0, 0.5)
        if dist == "int":
            assert np.array_equal(out.astype(np.float64), ref)
        else:
            u = np.finfo(np.float32).eps / 2
            bound = 1.01 * (k + 2) * u * (2 * np.abs(A).astype(np.float64) @ np.abs(B) + 0.5 * np.abs(C)) / (1 - (k + 2) * u)
            assert np.all(np.abs(out - ref) <= bound)


# --------------------------------------------------------------------------
# Contraction slabs and slices.
# --------------------------------------------------------------------------
def split_count(tiles, k, tk):
    """Slices of a split contraction: doubled while the tiles would not
    cover 256 CUs, each slice a whole number of slabs and >= 256 deep, at
    most 16; 1 unless the slices then cover them."""
    sp = 1
    while sp < 16 and tiles * sp < 256 and k % (2 * sp * tk) == 0 and k // (2 * sp) >= 256:
        sp *= 2
    return sp if tiles * sp >= 256 else 1


def slice_slabs(k, tk, splits, z):
    slabs = k // tk
    per = -(-slabs // splits)
    beg = z * per
    return range(beg, min(slabs, beg + per))


@pytest.mark.parametrize("m,n,k,tile", [
    (1024, 1024, 4096, (128, 128, 32, 32, 128, 2)),
    (1024, 1024, 4096, (256, 256, 32, 64, 128, 2)),
    (1024, 1024, 1024, (128, 128, 32, 32, 128, 2)),
    (512, 512, 8192, (128, 256, 32, 32, 128, 2)),
    (2048, 2048, 2048, (128, 128, 32, 32, 128, 2)),
    (512, 768, 4096, (128, 128, 32, 32, 128, 2)),
])
def test_split_slices_partition_the_slabs_and_match_the_library(m, n, k, tile):
    TM, TN, TK = tile[:3]
    sp = split_count((m // TM) * (n // TN), k, TK)
    covered = [s for z in range(sp) for s in slice_slabs(k, TK, sp, z)]
    assert covered == list(range(k // TK))  # each slab once, in order
    assert hp.describe(m, n, k, "fp32", tile=tile, workspace_bytes=1 << 40)["splits"] == sp
    assert hp.workspace_bytes(m, n, k, "fp32", tile) == (sp * m * n * 4 if sp > 1 else 0)


@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
def test_bf16_split_slices_match_the_library(prec):
    t = (128, 128, 32, 64, 64, 4)
    for m, n, k in [(512, 512, 4096), (1024, 512, 2048), (1024, 1024, 4096), (256, 384, 8192)]:
        sp = split_count((m // 128) * (n // 128), k, 32)
        assert hp.describe(m, n, k, prec, tile=t, workspace_bytes=1 << 40)["splits"] == sp, (m, n, k)


def test_launch_grid_matches_the_tile_grid():
    for prec, tile in [("fp32", (256, 256, 32, 64, 128, 2)), ("fp32", (64, 64, 16, 32, 32, 2)),
                       ("bf16", (256, 256, 32, 64, 128, 2)), ("bf16x3", (128, 128, 32, 64, 64, 4))]:
        for m, n, k in [(4096, 4096, 64), (1000, 3000, 32), (257, 129, 64)]:
            d = hp.describe(m, n, k, prec, tile=tile)
            assert (d["grid_x"], d["grid_y"]) == (-(-n // tile[1]), -(-m // tile[0])), (prec, tile, m, n)


# --------------------------------------------------------------------------
# The Allocation node fed by DMA: slab layouts in LDS and the fragments the
# MFMAs read from them.
# --------------------------------------------------------------------------
def dma_write_pos_128(r, c):
    """LDS byte offset, within a 32-row block of 128-byte rows, where the DMA
    puts chunk c (16 bytes) of row r: one instruction per 8 rows, lane l
    landing at 16 l, fetching row (l >> 3) ^ parity and chunk (l & 7) ^ that
    row."""
    g, par = r >> 3, (r >> 3) & 1
    for lane in range(64):
        x = (lane >> 3) ^ par
        if x == (r & 7) and ((lane & 7) ^ x) == c:
            return g * 1024 + 16 * lane
    raise AssertionError


def frag_pos_128(lane, ks):
    r = lane & 31
    rslot = r ^ ((r >> 3) & 1)
    return rslot * 128 + (((2 * ks + (lane >> 5)) ^ (r & 7)) << 4)


def dma_write_pos_64(r, c):
    """The same for 64-byte rows: two rows per 128-byte line, one instruction
    per 16 rows."""
    L = r >> 1
    inst, y = L >> 3, L & 7
    for lane in range(64):
        yy, p = lane >> 3, lane & 7
        g = (yy & 3) ^ ((yy >> 2) & 1)
        row = 2 * yy + ((p >> 2) & 1)
        if yy == y and row == (r - 16 * inst) and ((p ^ g) & 3) == c:
            return inst * 1024 + 16 * lane
    raise AssertionError


def frag_pos_64(lane, ks):
    l = lane & 31
    g = ((l >> 1) & 3) ^ ((l >> 3) & 1)
    pos = (((l & 1) << 2) | (2 * ks + (lane >> 5))) ^ g
    return (l >> 1) * 128 + (pos << 4)


@pytest.mark.parametrize("rb", [128, 64])
def test_dma_layout_is_a_bijection_the_fragments_read(rb):
    chunks = rb // 16
    write = dma_write_pos_128 if rb == 128 else dma_write_pos_64
    frag = frag_pos_128 if rb == 128 else frag_pos_64
    pos = {(r, c): write(r, c) for r in range(32) for c in range(chunks)}
    assert sorted(pos.values()) == list(range(0, 32 * rb, 16))  # fills the block exactly once
    for ks in range(chunks // 2):
        for lane in range(64):
            # lane l reads chunk 2 ks + (l >> 5) of row l & 31
            assert frag(lane, ks) == pos[(lane & 31, 2 * ks + (lane >> 5))]


@pytest.mark.parametrize("rb,group", [(128, 8), (64, 16)])
def test_fragment_reads_are_free_of_bank_conflicts(rb, group):
    """A 16-byte read of `group` consecutive lanes touches every 16-byte bank
    group of a 128 (or 256) byte window once."""
    frag = frag_pos_128 if rb == 128 else frag_pos_64
    for ks in range(rb // 32):
        for g0 in range(0, 64, group):
            banks = [(frag(l, ks) >> 4) % group for l in range(g0, g0 + group)]
            assert sorted(banks) == list(range(group)), (rb, ks, g0)


def test_bf16_fragment_slots_hold_k_in_natural_order():
    """For BF16 MFMA step s, lane half h reads FP32 chunks 4 s + 2 h and
    4 s + 2 h + 1 of its row (four k each): slot j holds k = 16 s + 8 h + j,
    and the steps and halves cover every k of a slab once."""
    for tk in (16, 32):
        seen = []
        for s in range(tk // 16):
            for h in range(2):
                chunks = [4 * s + 2 * h, 4 * s + 2 * h + 1]
                ks = [4 * c + e for c in chunks for e in range(4)]
                assert ks == [16 * s + 8 * h + j for j in range(8)]
                seen += ks
        assert sorted(seen) == list(range(tk))


# --------------------------------------------------------------------------
# The literal lowering (the paper's own two-level graph), run in FP32.
# --------------------------------------------------------------------------
def literal_emulation(A, B, C, alpha, beta, bx, by):
    """Root -> 2-D internal grid of (bx x by)-lane tiles -> one leaf instance
    per output; the Allocation holds a by x bx slab of B per k step of by, as
    the listing's leaf reads it; K tail zero-padded."""
    m, k = A.shape
    n = B.shape[1]
    out = C.astype(np.float32).copy()
    for gy, gx in itertools.product(range(-(-m // by)), range(-(-n // bx))):
        rows = np.arange(gy * by, min(m, gy * by + by))
        cols = np.arange(gx * bx, min(n, gx * bx + bx))
        acc = np.zeros((len(rows), len(cols)), dtype=np.float32)
        for k0 in range(0, k, by):
            slab = np.zeros((by, bx), dtype=np.float32)  # the Allocation node
            kk = np.arange(k0, min(k, k0 + by))
            slab[:len(kk), :len(cols)] = B[np.ix_(kk, cols)]
            a = np.zeros((len(rows), by), dtype=np.float32)
            a[:, :len(kk)] = A[np.ix_(rows, kk)]
            for p in range(by):
                acc += np.outer(a[:, p], slab[p, :len(cols)]).astype(np.float32)
        out[np.ix_(rows, cols)] = (np.float32(alpha) * acc + np.float32(beta) * C[np.ix_(rows, cols)]).astype(np.float32)
    return out


def test_literal_decomposition_in_fp32():
    for (m, n, k), dist in [((128, 128, 128), "int"), ((70, 45, 37), "int"), ((64, 96, 33), "uniform")]:
        A, B, C = inputs.sgemm_operands(m, n, k, seed=9, dist=dist)
        got = literal_emulation(A, B, C, 1.0, 0.5, 32, 32)
        ref = oracle.sgemm(A, B, C, 1.0, 0.5)
        if dist == "int":
            assert np.array_equal(got.astype(np.float64), ref)
        else:
            u = np.finfo(np.float32).eps / 2
            bound = 1.01 * (k + 2) * u * (np.abs(A).astype(np.float64) @ np.abs(B) + 0.5 * np.abs(C)) / (1 - (k + 2) * u)
            assert np.all(np.abs(got - ref) <= bound)
    # the Allocation node's size and the launch the library describes
    assert hp.alloc_bytes((32, 32, 32, 1, 1, 1)) == (32 * 32) << 2
    d = hp.describe(128, 128, 128, "fp32", tile=(32, 32, 32, 1, 1, 1))
    assert (d["grid_x"], d["grid_y"], d["block_x"], d["block_y"]) == (4, 4, 32, 32)
