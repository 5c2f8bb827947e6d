"""C-ABI checks that need no GPU: exports, argument validation, graph structure.

No test here launches a kernel: argument checks return before any HIP call,
and the fault-injection switch stops a valid call right after them.
"""
import ctypes
import json
import os
import re
import subprocess

import pytest

import paper_1611_00860_amd as hp
from paper_1611_00860_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hpvm_sgemm.h")
GOLDEN = os.path.join(ROOT, "tests", "golden", "sgemm_dfg_structure.json")
FAKE = 0x10000  # never dereferenced: validation or injection stops first


@pytest.fixture(scope="module")
def lib():
    return hp.load()


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hpvm_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = header_functions()
    assert names, "no declarations found"
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (hpvm_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    # and the binding declares a signature for every one of them
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def test_struct_sizes_match_header():
    assert ctypes.sizeof(_lib.RootIn) == 88
    assert ctypes.sizeof(_lib.Tile) == 24
    assert ctypes.sizeof(_lib.Edge) == 24


def test_root_in_matches_paper_listing():
    g = json.load(open(GOLDEN))
    assert ctypes.sizeof(_lib.RootIn) == g["root_in_bytes"]
    assert [f for f, _ in _lib.RootIn._fields_] == g["root_in_field_names"]
    kinds = {ctypes.c_void_p: "ptr", ctypes.c_int64: "i64", ctypes.c_int32: "i32",
             ctypes.c_float: "float"}
    assert [kinds[t] for _, t in _lib.RootIn._fields_] == g["root_in_field_types"]


def test_allocation_size_formula():
    g = json.load(open(GOLDEN))
    for bx, by, expect in g["allocation_bytes"]:
        tile = (by, bx, by, 1, 1, 1)
        assert hp.alloc_bytes(tile) == expect


def test_edges_match_paper_listing():
    g = json.load(open(GOLDEN))
    ids = g["nodes"]
    edges = hp.dfg_edges()
    flows = [e for e in edges if e["kind"] == 0]
    binds = [e for e in edges if e["kind"] == 1]
    for e in g["edges_printed"]:
        assert {"kind": 0, "src_node": ids[e["src"]], "dst_node": ids[e["dst"]],
                "src_port": e["src_port"], "dst_port": e["dst_port"],
                "all_to_all": int(e["all_to_all"])} in flows
    assert len(flows) == len(g["edges_printed"])
    for b in g["binds_printed"]:
        assert any(x["src_node"] == ids[b["parent"]] and x["dst_node"] == ids[b["child"]] and
                   x["src_port"] == b["parent_port"] and x["dst_port"] == b["child_port"]
                   for x in binds), b
    lo, hi = g["binds_implied"]["SgemmInternal->SgemmLeaf"]
    leaf = sorted(x["src_port"] for x in binds if x["src_node"] == 1 and x["dst_node"] == 3)
    assert leaf == list(range(lo, hi + 1))
    lo, hi = g["binds_implied"]["SgemmRoot->SgemmInternal"]
    root = sorted(x["src_port"] for x in binds if x["src_node"] == 0 and x["dst_node"] == 1)
    assert root == list(range(lo, hi + 1))
    # every leaf input (0..13) is fed exactly once, by a bind or an edge
    fed = sorted([x["dst_port"] for x in binds if x["dst_node"] == 3] +
                 [x["dst_port"] for x in flows if x["dst_node"] == 3])
    assert fed == list(range(14))


def test_describe_literal_config():
    g = json.load(open(GOLDEN))
    d = hp.describe(128, 128, 128, "fp32", (32, 32, 32, 1, 1, 1))
    assert d["root_instances"] == g["root_instances"] == 1
    assert (d["grid_x"], d["grid_y"], d["block_x"], d["block_y"]) == (4, 4, 32, 32)
    assert d["alloc_bytes"] == 4096 and d["lowering_name"] == "literal" and d["k_slabs"] == 4
    assert d["waves"] == 16


def test_describe_untiled_graph():
    """tile_k = 0, stages = 0: the one-level graph with no Allocation node."""
    d = hp.describe(128, 128, 128, "fp32", (32, 32, 0, 1, 1, 0))
    assert (d["grid_x"], d["grid_y"], d["block_x"], d["block_y"]) == (4, 4, 32, 32)
    assert d["alloc_bytes"] == 0 and d["lowering_name"] == "flat" and d["k_slabs"] == 0
    assert hp.alloc_bytes((32, 32, 0, 1, 1, 0)) == 0
    for bad in ((32, 32, 0, 1, 1, 2), (32, 32, 16, 1, 1, 0), (4, 4, 0, 1, 1, 0)):
        with pytest.raises(hp.HpvmError):
            hp.describe(128, 128, 128, "fp32", bad)
    with pytest.raises(hp.HpvmError):
        hp.describe(128, 128, 128, "bf16", (32, 32, 0, 1, 1, 0))


def test_describe_mfma_grids():
    menu = hp.tile_menu("fp32")
    assert menu, "no FP32 MFMA tile compiled"
    for tile in menu:
        tm, tn, tk, lm, ln, st = tile
        d = hp.describe(4096, 4096, 4096, "fp32", tile)
        assert d["grid_x"] == -(-4096 // tn) and d["grid_y"] == -(-4096 // tm)
        assert d["waves"] == (tm // lm) * (tn // ln)
        assert d["k_slabs"] == -(-4096 // tk)
        assert d["alloc_bytes"] == hp.alloc_bytes(tile, "fp32") <= 160 * 1024
        assert d["lowering_name"] == "mfma_f32"
    d = hp.describe(8192, 4096, 2048, "fp32", None)
    assert d["lowering_name"] == "mfma_f32"


def call(lib, m=4, n=4, k=4, alpha=1.0, A=FAKE, lda=4, B=FAKE * 2, ldb=4, beta=0.0, C=FAKE * 4,
         ldc=4, prec=0, tile=None):
    t = ctypes.byref(_lib.Tile(*tile)) if tile else None
    return lib.hpvm_sgemm(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, prec, t, None)


@pytest.mark.parametrize("kw,argno", [
    ({"m": -1}, 1), ({"n": -1}, 2), ({"k": -2}, 3), ({"A": None}, 5), ({"lda": 3}, 6),
    ({"B": None}, 7), ({"ldb": 2}, 8), ({"C": None}, 10), ({"ldc": 1}, 11), ({"prec": 9}, 12),
])
def test_invalid_arguments_name_the_first_bad_one(lib, kw, argno):
    rc = call(lib, **kw)
    assert rc == -1
    assert hp.last_error().startswith(f"argument {argno}:"), hp.last_error()


def test_checks_run_in_argument_order(lib):
    rc = call(lib, m=-1, lda=0, C=None)
    assert rc == -1 and hp.last_error().startswith("argument 1:")


def test_unsupported_tile_and_literal_precision(lib):
    assert call(lib, tile=(48, 48, 16, 16, 16, 2)) == -2
    assert "argument 13" in hp.last_error()
    assert call(lib, tile=(32, 32, 32, 1, 1, 1), prec=1) == -2
    assert call(lib, tile=(32, 32, 16, 1, 1, 1)) == -2  # literal needs tile_k == tile_m
    assert call(lib, tile=(4, 4, 4, 1, 1, 1)) == -2     # fewer lanes than a wavefront


def test_overlap_of_c_with_inputs_is_refused(lib):
    assert call(lib, A=FAKE, C=FAKE + 8) == -1
    assert "overlaps" in hp.last_error()


def test_quick_returns_without_device(lib):
    assert call(lib, m=0, A=None, B=None, C=None) == 0
    assert call(lib, n=0, A=None, B=None, C=None) == 0


def test_fault_injection_reports_hip_error(lib, monkeypatch):
    monkeypatch.setenv("HPVM_FAULT_INJECT", "launch")
    rc = call(lib)
    assert rc == -3 and "injected" in hp.last_error()
    monkeypatch.setenv("HPVM_FAULT_INJECT", "wait")
    assert lib.hpvm_wait(None) == -3
    with pytest.raises(hp.HpvmError) as ei:
        hp._check(-3)
    assert ei.value.status == -3


def test_status_strings(lib):
    for code, name in [(0, "HPVM_OK"), (-1, "HPVM_INVALID_ARG"), (-2, "HPVM_UNSUPPORTED"),
                       (-3, "HPVM_HIP_ERROR"), (-4, "HPVM_WORKSPACE_TOO_SMALL"), (-5, "HPVM_BAD_HANDLE"),
                       (-6, "HPVM_QUEUE_FULL"), (-7, "HPVM_TIMEOUT"), (-8, "HPVM_STREAM_ENDED")]:
        assert hp.status_string(code) == name


def test_root_launch_validation(lib):
    r = _lib.RootIn(FAKE, 16 * 16 * 4, 16, FAKE * 2, 16 * 16 * 4, 16, FAKE * 4, 16 * 16 * 4, 16,
                    16, 1.0, 0.0, 16, 16, 1, 1)
    r.bytesC = 100
    assert lib.hpvm_launch_root(ctypes.byref(r), None) == -1 and "bytesC" in hp.last_error()
    r.bytesC = 16 * 16 * 4
    r.block_x = 3
    assert lib.hpvm_launch_root(ctypes.byref(r), None) == -2
    assert lib.hpvm_launch_root(None, None) == -1


# ---------------------------------------------------------------------------
# Grouped plans: host-side construction, validation and handles
# ---------------------------------------------------------------------------
def _descs(shapes, base=0x100000):
    arr = (_lib.SgemmDesc * len(shapes))()
    addr = base
    for i, (m, n, k) in enumerate(shapes):
        a, b, c = addr, addr + 4 * m * k + 256, addr + 4 * (m * k + k * n) + 512
        addr = c + 4 * m * n + 4096
        arr[i] = _lib.SgemmDesc(m, n, k, 1.0, 0.5, a, max(k, 1), b, max(n, 1), c, max(n, 1))
    return arr


def _plan(lib, shapes, tile=None):
    h = ctypes.c_void_p()
    t = ctypes.byref(_lib.Tile(*tile)) if tile else None
    rc = lib.hpvm_grouped_plan_create(len(shapes), _descs(shapes), 0, t, ctypes.byref(h))
    return rc, h


def test_grouped_plan_host_side(lib):
    shapes = [(48, 48, 64), (2048, 2048, 512), (100, 300, 7), (0, 5, 5), (64, 64, 0)]
    rc, h = _plan(lib, shapes)
    assert rc == 0, hp.last_error()
    info = _lib.GroupedInfo()
    assert lib.hpvm_grouped_plan_info(h, ctypes.byref(info)) == 0
    assert info.count == 5
    assert info.flops == sum(2.0 * m * n * k for m, n, k in shapes)
    tiles = []
    for i, (m, n, k) in enumerate(shapes):
        t = _lib.Tile()
        assert lib.hpvm_grouped_instance_tile(h, i, ctypes.byref(t)) == 0
        tiles.append(t.as_tuple())
        if m and n:
            tiles_i = -(-m // t.tile_m) * -(-n // t.tile_n)
        else:
            tiles_i = 0
        shapes[i] = (m, n, k, tiles_i)
    # every tile of every instance is listed exactly once
    assert info.total_tiles == sum(s[3] for s in shapes)
    # the cost model gives the small instance the small tile, the big one the big tile
    assert tiles[0] == (64, 64, 16, 32, 32, 2)
    assert tiles[1] == (128, 128, 16, 64, 64, 2)
    ws = ctypes.c_int64()
    assert lib.hpvm_grouped_workspace_bytes(h, ctypes.byref(ws)) == 0 and ws.value == info.workspace_bytes
    assert info.scratch_bytes == 4 * sum(m * n for m, n, *_ in shapes)
    # too small a workspace is refused before any device work
    assert lib.hpvm_grouped_run(h, FAKE, ws.value - 1, None) == -4
    assert lib.hpvm_grouped_run(h, FAKE + 4, ws.value, None) == -1  # misaligned
    assert lib.hpvm_grouped_plan_destroy(h) == 0
    # stale handles
    assert lib.hpvm_grouped_plan_destroy(h) == -5
    assert lib.hpvm_grouped_plan_info(h, ctypes.byref(info)) == -5
    assert lib.hpvm_grouped_run(h, FAKE, 1 << 30, None) == -5
    assert lib.hpvm_graph_launch(ctypes.c_void_p(FAKE), None) == -5
    assert lib.hpvm_graph_destroy(None) == -5


def test_grouped_plan_fixed_tile_and_menu(lib):
    menu = hp.grouped_menu()
    assert len(menu) == 4 and all(t[3] * 0 == 0 for t in menu)
    for tile in menu:
        rc, h = _plan(lib, [(300, 200, 50), (17, 33, 9)], tile)
        assert rc == 0
        t = _lib.Tile()
        assert lib.hpvm_grouped_instance_tile(h, 1, ctypes.byref(t)) == 0 and t.as_tuple() == tuple(tile)
        assert lib.hpvm_grouped_plan_destroy(h) == 0
    rc, h = _plan(lib, [(8, 8, 8)], (32, 32, 16, 16, 16, 2))
    assert rc == -2 and "grouped menu" in hp.last_error()
    # every grouped shape can also run as a single launch (bitwise comparisons)
    single = hp.tile_menu("fp32")
    assert all(tuple(t) in single for t in menu)


def test_grouped_plan_validation(lib):
    h = ctypes.c_void_p()
    assert lib.hpvm_grouped_plan_create(-1, None, 0, None, ctypes.byref(h)) == -1
    assert lib.hpvm_grouped_plan_create(2, None, 0, None, ctypes.byref(h)) == -1
    d = _descs([(10, 10, 10), (20, 20, 20)])
    assert lib.hpvm_grouped_plan_create(2, d, 1, None, ctypes.byref(h)) == -2
    d[1].ldb = 3
    assert lib.hpvm_grouped_plan_create(2, d, 0, None, ctypes.byref(h)) == -1
    assert hp.last_error().startswith("instance 1: argument 8"), hp.last_error()
    d = _descs([(10, 10, 10), (20, 20, 20)])
    d[1].C = d[0].C + 16  # two instances writing overlapping memory
    assert lib.hpvm_grouped_plan_create(2, d, 0, None, ctypes.byref(h)) == -1
    assert "overlapping" in hp.last_error()


def test_grouped_fault_injection(lib, monkeypatch):
    rc, h = _plan(lib, [(64, 64, 64)])
    assert rc == 0
    ws = ctypes.c_int64()
    lib.hpvm_grouped_workspace_bytes(h, ctypes.byref(ws))
    monkeypatch.setenv("HPVM_FAULT_INJECT", "capture")
    g = ctypes.c_void_p()
    assert lib.hpvm_grouped_capture(h, FAKE, ws.value, None, ctypes.byref(g)) == -3
    monkeypatch.setenv("HPVM_FAULT_INJECT", "launch")
    assert lib.hpvm_grouped_run(h, FAKE, ws.value, None) == -3
    assert lib.hpvm_grouped_plan_destroy(h) == 0


def test_autotune_cache_host_side(lib, tmp_path):
    hp.autotune_clear()
    menu = hp.tile_menu("fp32")
    tile, found = hp.autotune_lookup(4096, 4096, 4096, "fp32")
    assert found == 0 and tile == menu[0]
    hp.autotune_record(4096, 4096, 4096, menu[2], "fp32", 1.25)
    assert hp.autotune_lookup(4096, 4096, 4096, "fp32") == (menu[2], 2)
    # same shape class (ceil log2 of each size) falls back to the class entry
    assert hp.autotune_lookup(3000, 4000, 2500, "fp32") == (menu[2], 1)
    assert hp.autotune_lookup(5000, 4096, 4096, "fp32")[1] == 0
    assert hp.autotune_lookup(4096, 4096, 4096, "bf16")[1] == 0
    path = tmp_path / "cache.txt"
    hp.autotune_save(path)
    hp.autotune_clear()
    assert hp.autotune_lookup(4096, 4096, 4096, "fp32")[1] == 0
    with open(path, "a") as f:
        f.write("0 10 10 10 48 48 16 16 16 2 1.0\n")  # not compiled: skipped
        f.write("garbage line\n")
    hp.autotune_load(path)
    assert hp.autotune_lookup(4096, 4096, 4096, "fp32") == (menu[2], 2)
    assert hp.autotune_lookup(10, 10, 10, "fp32")[1] == 0
    with pytest.raises(hp.HpvmError):
        hp.autotune_record(8, 8, 8, (48, 48, 16, 16, 16, 2), "fp32")
    hp.autotune_clear()


def test_autotune_cache_keyed_by_arch_and_runtime(lib, tmp_path):
    """Saved entries carry the GPU architecture and HIP runtime they were
    timed on; loading skips entries whose tag differs from this process's."""
    hp.autotune_clear()
    menu = hp.tile_menu("fp32")
    hp.autotune_record(2048, 2048, 2048, menu[1], "fp32", 0.5)
    path = tmp_path / "cache.txt"
    hp.autotune_save(path)
    lines = [l for l in open(path) if not l.startswith("#")]
    assert len(lines) == 1
    arch, runtime = lines[0].split()[:2]
    assert arch.startswith("gfx") and ":" not in arch and runtime.startswith("hip")
    rest = " ".join(lines[0].split()[2:])
    hp.autotune_clear()
    hp.autotune_load(path)
    assert hp.autotune_lookup(2048, 2048, 2048, "fp32") == (menu[1], 2)
    for other in (f"gfx942 {runtime}", f"{arch} hip1", "0"):  # another arch, another runtime, untagged
        hp.autotune_clear()
        with open(path, "w") as f:
            f.write(f"{other} {rest}\n")
        hp.autotune_load(path)
        assert hp.autotune_lookup(2048, 2048, 2048, "fp32")[1] == 0, other
    hp.autotune_clear()


def test_describe_ws_reports_the_split_only_when_the_workspace_holds_it(lib):
    """hpvm_sgemm_ws with no tile splits the contraction of an FP32 problem
    that even 128 x 128 tiles leave CUs idle on, only when the workspace
    holds the partial sums; otherwise it takes hpvm_sgemm's tile."""
    hp.autotune_clear()
    m, n, k = 1024, 1024, 4096
    need = hp.workspace_bytes(m, n, k, "fp32")
    assert need > 0 and need % (4 * m * n) == 0
    full = hp.describe(m, n, k, "fp32", workspace_bytes=need)
    assert full["splits"] == need // (4 * m * n) > 1
    plain = hp.describe(m, n, k, "fp32")
    assert plain["splits"] == 1
    for short in (0, need - 1):
        d = hp.describe(m, n, k, "fp32", workspace_bytes=short)
        assert d == plain, short  # the single launch's own choice, not the split tile unsplit
    assert (full["grid_x"], full["grid_y"]) != (plain["grid_x"], plain["grid_y"])
    # a problem 128 x 128 tiles cover never splits
    assert hp.workspace_bytes(4096, 4096, 4096, "fp32") == 0
    assert hp.describe(4096, 4096, 4096, "fp32", workspace_bytes=1 << 30)["splits"] == 1
    with pytest.raises(hp.HpvmError):
        hp.describe(m, n, k, "fp32", workspace_bytes=-1)


def test_backward_validation(lib):
    ws = ctypes.c_int64()
    assert lib.hpvm_sgemm_backward_workspace_bytes(4096, 4096, 1024, 0, None, ctypes.byref(ws)) == 0
    assert ws.value >= 4 * 256
    for prec in ("fp32", "bf16", "bf16x3"):
        menu = hp.backward_menu(prec)
        assert menu
        for t in menu:
            b = hp.backward_workspace_bytes(4096, 4096, 1024, prec, t)
            if t[5] == 3:  # staged: holds the bfloat16 planes of the larger of dA's and dB's products
                assert b >= hp.workspace_bytes(4096, 1024, 4096, prec, t)
    with pytest.raises(hp.HpvmError):
        hp.backward_workspace_bytes(64, 64, 64, "fp32", (48, 48, 16, 16, 16, 2))
    args = dict(m=16, n=16, k=16, alpha=0.7, beta=0.3, A=FAKE, lda=16, B=FAKE * 2, ldb=16, C_in=FAKE * 3,
                ldci=16, G=FAKE * 4, ldg=16, dA=FAKE * 5, ldda=16, dB=FAKE * 6, lddb=16, dC_in=FAKE * 7,
                lddci=16, dalpha=FAKE * 8, dbeta=FAKE * 8 + 4, prec=0, tile=None, ws=FAKE * 9, wsb=1 << 20)

    def call_bw(**kw):
        a = dict(args)
        a.update(kw)
        t = ctypes.byref(_lib.Tile(*a["tile"])) if a["tile"] else None
        return lib.hpvm_sgemm_backward(a["m"], a["n"], a["k"], a["alpha"], a["beta"], a["A"], a["lda"],
                                       a["B"], a["ldb"], a["C_in"], a["ldci"], a["G"], a["ldg"], a["dA"],
                                       a["ldda"], a["dB"], a["lddb"], a["dC_in"], a["lddci"], a["dalpha"],
                                       a["dbeta"], a["prec"], t, a["ws"], a["wsb"], None)

    assert call_bw(m=-1) == -1 and hp.last_error().startswith("argument 1")
    assert call_bw(A=None) == -1 and hp.last_error().startswith("argument 6")
    assert call_bw(B=None) == -1 and hp.last_error().startswith("argument 8")
    assert call_bw(C_in=None) == -1 and hp.last_error().startswith("argument 10")
    assert call_bw(G=None) == -1 and hp.last_error().startswith("argument 12")
    assert call_bw(lddb=3) == -1 and hp.last_error().startswith("argument 17")
    assert call_bw(prec=7) == -1
    assert call_bw(tile=(48, 48, 16, 16, 16, 2)) == -2
    assert call_bw(wsb=8) == -4
    assert call_bw(ws=FAKE + 4) == -1
    # C_in is not needed without dbeta, B not needed for dB alone: the checks
    # pass and the (injected) launch is reached
    import os
    os.environ["HPVM_FAULT_INJECT"] = "launch"
    try:
        rc = call_bw(C_in=None, dbeta=None, wsb=0, ws=None, dalpha=None, B=None, dA=None, dC_in=None)
        assert rc == -3 and "injected" in hp.last_error()
        # a staged tile needs the workspace even without the scalars
        st = [t for t in hp.backward_menu("bf16") if t[5] == 3][0]
        rc = call_bw(C_in=None, dbeta=None, wsb=0, ws=None, dalpha=None, dC_in=None, prec=1, tile=st)
        assert rc == -1 and "workspace" in hp.last_error()
    finally:
        del os.environ["HPVM_FAULT_INJECT"]


def test_default_tile_with_a_workspace(lib):
    """Without an autotuned entry, a workspace-capable BF16 / bf16x3 call with
    no tile takes the first staged tile once m n k reaches 2^31, else the
    menu's entry 0 (which needs no workspace); FP32 never needs one."""
    hp.autotune_clear()
    for prec in ("bf16", "bf16x3"):
        staged = [t for t in hp.tile_menu(prec) if t[5] == 3]
        big = (2048, 1024, 1024)  # 2^31 multiply-adds
        assert hp.workspace_bytes(*big, prec, None) == hp.workspace_bytes(*big, prec, staged[0]) > 0
        assert hp.workspace_bytes(2048, 1024, 1023, prec, None) == 0
    assert hp.workspace_bytes(8192, 8192, 8192, "fp32", None) == 0


def test_default_fp32_tile_for_small_problems(lib):
    """Without an autotuned entry the FP32 default is the menu's entry 0
    when it gives at least 256 tiles, else the DMA-fed 128 x 128 x 32 tile
    when that does, else the 64 x 64 x 16 tile.  BF16 and bf16x3 keep
    entry 0 from 256 tiles up, else take 64 x 64 x 32."""
    hp.autotune_clear()
    menu = hp.tile_menu("fp32")
    mid_t, small_t = (128, 128, 32, 32, 128, 2), (64, 64, 16, 32, 32, 2)
    assert mid_t in menu and small_t in menu
    big = hp.describe(4096, 4096, 1024, "fp32", None)
    assert (big["grid_x"], big["grid_y"]) == (4096 // menu[0][1], 4096 // menu[0][0])
    for m, n, tile in ((2048, 4096, mid_t), (2048, 2048, mid_t), (1000, 1000, small_t)):
        d = hp.describe(m, n, 1024, "fp32", None)
        assert (d["grid_x"], d["grid_y"]) == (-(-n // tile[1]), -(-m // tile[0])), (m, n)
        assert d["alloc_bytes"] == hp.alloc_bytes(tile, "fp32"), (m, n)
    # BF16 and bf16x3: entry 0 (256 x 256) from 256 tiles up, else 64 x 64 x 32
    for prec in ("bf16", "bf16x3"):
        menu = hp.tile_menu(prec)
        assert menu[0][:2] == (256, 256) and (64, 64, 32, 32, 32, 2) in menu
        big = hp.describe(4096, 4096, 512, prec, None)
        assert (big["grid_x"], big["grid_y"]) == (16, 16)
        small = hp.describe(1024, 1024, 1024, prec, None)
        assert (small["grid_x"], small["grid_y"]) == (16, 16) and small["waves"] == 4


def test_describe_follows_the_autotuned_tile(lib):
    """hpvm_describe reports the launch hpvm_sgemm would make: a recorded
    autotuner entry for the shape takes precedence over the built-in rule."""
    hp.autotune_clear()
    tile = (64, 128, 16, 32, 64, 2)
    hp.autotune_record(4096, 4096, 1024, tile, "fp32")
    d = hp.describe(4096, 4096, 1024, "fp32", None)
    assert (d["grid_x"], d["grid_y"]) == (4096 // 128, 4096 // 64)
    assert d["alloc_bytes"] == hp.alloc_bytes(tile, "fp32")
    hp.autotune_clear()
    d = hp.describe(4096, 4096, 1024, "fp32", None)
    assert (d["grid_x"], d["grid_y"]) == (16, 16)


def test_split_contraction_workspace_rules(lib):
    """FP32 DMA-fed tiles split the contraction of whole-tile problems whose
    tiles would not cover 256 CUs, doubling the slices (each a whole number
    of slabs, at least 256 deep, at most 16) until they do; the workspace
    holds one m x n float plane per slice.  With no tile, hpvm_sgemm_ws
    splits only when even 128 x 128 tiles would not cover the CUs, on the
    entry with the fewest slices."""
    hp.autotune_clear()
    plane = lambda m, n: 4 * m * n
    t256, t128x256, t128 = (256, 256, 32, 64, 128, 2), (128, 256, 32, 32, 128, 2), (128, 128, 32, 32, 128, 2)
    # 16 tiles of 256 x 256 -> 16 slices of 256; 32 of 128 x 256 -> 8 of 512;
    # 64 of 128 x 128 -> 4 of 1024
    assert hp.workspace_bytes(1024, 1024, 4096, "fp32", t256) == 16 * plane(1024, 1024)
    assert hp.workspace_bytes(1024, 1024, 4096, "fp32", t128x256) == 8 * plane(1024, 1024)
    assert hp.workspace_bytes(1024, 1024, 4096, "fp32", t128) == 4 * plane(1024, 1024)
    assert hp.workspace_bytes(1024, 1024, 4096, "fp32", None) == 4 * plane(1024, 1024)
    assert hp.workspace_bytes(1024, 1024, 1024, "fp32", None) == 4 * plane(1024, 1024)
    assert hp.workspace_bytes(2048, 2048, 2048, "fp32", t256) == 4 * plane(2048, 2048)
    for m, n, k, tile in (
            (2048, 2048, 2048, None),         # 256 tiles of 128 x 128: no split
            (1024, 1024, 1024, t256),         # slices would stay under 256 workgroups
            (512, 512, 8192, t128x256),       # 8 tiles: 16 slices are not enough
            (4096, 4096, 4096, None),         # already 256 tiles
            (1000, 1024, 4096, t256),         # not whole tiles
            (1024, 1024, 4000, t256),         # contraction not whole slabs per slice
            (1024, 1024, 4096, (128, 128, 16, 64, 64, 2)),  # not DMA-fed
    ):
        assert hp.workspace_bytes(m, n, k, "fp32", tile) == 0, (m, n, k, tile)


def test_bf16_split_contraction_workspace_rules(lib):
    """The DMA-fed BF16 and bf16x3 tiles split the contraction by the FP32
    rule; with no tile, hpvm_sgemm_ws splits when even 128 x 128 tiles would
    not cover the CUs and k >= 2048, only when the workspace holds the
    partial sums, else it keeps its other choices."""
    hp.autotune_clear()
    plane = lambda m, n: 4 * m * n
    t128 = (128, 128, 32, 64, 64, 4)
    for prec in ("bf16", "bf16x3"):
        big = hp.tile_menu(prec)[0]
        assert big[:2] == (256, 256) and t128 in hp.tile_menu(prec)
        # 16 tiles of 128 x 128 -> 16 slices of 256; 4 of 256 x 256: not enough
        assert hp.workspace_bytes(512, 512, 4096, prec, t128) == 16 * plane(512, 512)
        assert hp.workspace_bytes(512, 512, 4096, prec, big) == 0
        assert hp.workspace_bytes(1024, 1024, 4096, prec, t128) == 4 * plane(1024, 1024)
        need = hp.workspace_bytes(512, 512, 4096, prec)
        assert need == 16 * plane(512, 512)
        d = hp.describe(512, 512, 4096, prec, workspace_bytes=need)
        assert d["tile"] == t128 and d["splits"] == 16
        short = hp.describe(512, 512, 4096, prec, workspace_bytes=need - 1)
        assert short["splits"] == 1 and short == hp.describe(512, 512, 4096, prec)
        assert hp.describe(1024, 1024, 4096, prec, workspace_bytes=1 << 30)["splits"] == 4
        # k < 2048, or 128 x 128 tiles that cover the CUs: no split
        assert hp.describe(1024, 1024, 1024, prec, workspace_bytes=1 << 30)["splits"] == 1
        assert hp.describe(2048, 2048, 4096, prec, workspace_bytes=1 << 30)["splits"] == 1
        # not whole tiles: no split, whatever the tile
        assert hp.workspace_bytes(1000, 1024, 4096, prec, t128) == 0


def test_staged_workspace_rules(lib):
    BIG = 1 << 24  # far enough apart that no two matrices overlap
    for prec, planes in (("bf16", 1), ("bf16x3", 2)):
        menu = hp.tile_menu(prec)
        staged = [t for t in menu if t[5] == 3]
        fused = [t for t in menu if t[5] != 3]
        assert staged and fused and menu[0][5] != 3  # the default needs no workspace
        m, n, k = 300, 520, 100
        need = hp.workspace_bytes(m, n, k, prec, staged[0])
        assert need == planes * 2 * (512 + 768) * 128  # padded to 256 x 256 x 64 blocks
        assert hp.workspace_bytes(m, n, k, prec, fused[0]) == 0
        assert hp.describe(m, n, k, prec, staged[0])["lowering_name"] == f"staged_{prec}"
        t = ctypes.byref(_lib.Tile(*staged[0]))
        rc = lib.hpvm_sgemm(m, n, k, 1.0, BIG, k, BIG * 2, n, 0.0, BIG * 4, n, hp.PREC[prec], t, None)
        assert rc == -2 and "workspace" in hp.last_error()
        rc = lib.hpvm_sgemm_ws(m, n, k, 1.0, BIG, k, BIG * 2, n, 0.0, BIG * 4, n, hp.PREC[prec], t,
                               BIG * 8, need - 16, None)
        assert rc == -4
        rc = lib.hpvm_sgemm_ws(m, n, k, 1.0, BIG, k, BIG * 2, n, 0.0, BIG * 4, n, hp.PREC[prec], t,
                               BIG * 8 + 4, need, None)
        assert rc == -1 and "aligned" in hp.last_error()
        # alpha = 0 needs no workspace: nothing is converted
        import os
        os.environ["HPVM_FAULT_INJECT"] = "launch"
        try:
            rc = lib.hpvm_sgemm_ws(m, n, k, 0.0, None, k, None, n, 1.0, BIG * 4, n, hp.PREC[prec], t, None, 0,
                                   None)
            assert rc == -3
        finally:
            del os.environ["HPVM_FAULT_INJECT"]
    assert all(t[5] != 3 for t in hp.tile_menu("fp32"))


def test_stream_validation(lib, monkeypatch):
    """Config checks run before any HIP call; unknown handles are refused."""
    h = ctypes.c_void_p()

    def open_(cap=8, grid=0, idle=100, handle=True):
        cfg = _lib.StreamConfig(cap, grid, idle, 0)
        return lib.hpvm_stream_open(ctypes.byref(cfg), ctypes.byref(h) if handle else None)

    assert lib.hpvm_stream_open(None, ctypes.byref(h)) == -1
    assert open_(cap=0) == -1 and "capacity" in hp.last_error()
    assert open_(cap=4097) == -1
    assert open_(grid=-1) == -1 and "grid" in hp.last_error()
    # more than two resident workgroups per CU would starve every other
    # kernel while the stream is open: refused before any HIP call
    for grid in (513, 768, 65536):
        monkeypatch.setenv("HPVM_FAULT_INJECT", "launch")  # a grid that passed would stop here with -3
        assert open_(grid=grid) == -1 and "grid" in hp.last_error(), grid
    monkeypatch.setenv("HPVM_FAULT_INJECT", "launch")
    assert open_(grid=512) == -3  # two per CU of 256 CUs passes the host check
    monkeypatch.delenv("HPVM_FAULT_INJECT")
    assert open_(idle=0) == -1 and "idle_ms" in hp.last_error()
    assert open_(idle=60001) == -1
    assert open_(handle=False) == -1 and "argument 2" in hp.last_error()
    monkeypatch.setenv("HPVM_FAULT_INJECT", "launch")
    assert open_() == -3 and "injected" in hp.last_error()
    monkeypatch.delenv("HPVM_FAULT_INJECT")
    bogus = ctypes.c_void_p(FAKE)
    d = _lib.SgemmDesc(4, 4, 4, 1.0, 0.0, FAKE, 4, FAKE + 4096, 4, FAKE + 8192, 4)
    assert lib.hpvm_stream_push(bogus, ctypes.byref(d), None) == -5
    assert lib.hpvm_stream_push(None, ctypes.byref(d), None) == -5
    seq = ctypes.c_int64()
    assert lib.hpvm_stream_pop(bogus, 0, ctypes.byref(seq), None) == -5
    st = _lib.StreamStatus()
    assert lib.hpvm_stream_info(bogus, ctypes.byref(st)) == -5
    assert lib.hpvm_stream_close(bogus, 0) == -5


def test_stream_status_layout():
    assert ctypes.sizeof(_lib.StreamConfig) == 16
    assert ctypes.sizeof(_lib.StreamStatus) == 48


def test_fusion_menus(lib):
    # the consumer kernel takes the FP32 single-launch tiles, in order
    assert hp.fusion_menu("consumer") == hp.tile_menu("fp32")
    pair = hp.fusion_menu("pair")
    assert len(pair) == 4 and all(t[5] == 2 for t in pair) and pair[0][4] == 128
    assert pair[3] == (128, 128, 32, 32, 128, 2)  # the tile that splits the contraction
    cnt = ctypes.c_int32()
    assert lib.hpvm_fusion_menu(2, None, 0, ctypes.byref(cnt)) == -1


def _consumer_call(lib, **kw):
    a = dict(m=64, n=48, k=32, alpha=1.0, A=FAKE, lda=32, B=FAKE + (1 << 24), ldb=48, beta=1.0,
             C=FAKE + (2 << 24), ldc=48, op=1, bias=0, lo=0.0, hi=1.0, D=FAKE + (3 << 24), ldd=48,
             tile=None, cons=True)
    a.update(kw)
    cons = _lib.Consumer(a["op"], 0, a["bias"], a["lo"], a["hi"])
    t = None
    if a["tile"] is not None:
        t = ctypes.byref(_lib.Tile(*a["tile"]))
    return lib.hpvm_sgemm_consumer(a["m"], a["n"], a["k"], a["alpha"], a["A"], a["lda"], a["B"], a["ldb"],
                                   a["beta"], a["C"], a["ldc"], ctypes.byref(cons) if a["cons"] else None,
                                   a["D"], a["ldd"], t, None)


@pytest.mark.parametrize("kw,argno", [
    (dict(m=-1), 1), (dict(n=-1), 2), (dict(k=-1), 3), (dict(A=None), 5), (dict(lda=31), 6),
    (dict(B=None), 7), (dict(ldb=47), 8), (dict(C=None), 10), (dict(ldc=47), 11),
    (dict(cons=False), 12), (dict(op=9), 12), (dict(op=2), 12), (dict(op=4, lo=2.0, hi=1.0), 12),
    (dict(D=None), 13), (dict(ldd=47), 14), (dict(D=FAKE + 64), 13), (dict(D=FAKE + (2 << 24) + 64), 13),
])
def test_consumer_validation(lib, kw, argno):
    assert _consumer_call(lib, **kw) == -1
    assert f"argument {argno}:" in hp.last_error(), hp.last_error()


def test_consumer_accepts_in_place_and_null_c(lib, monkeypatch):
    monkeypatch.setenv("HPVM_FAULT_INJECT", "launch")
    # D == C with the same leading dimension is in place
    assert _consumer_call(lib, D=FAKE + (2 << 24)) == -3
    # beta == 0: C may be NULL and may overlap D
    assert _consumer_call(lib, beta=0.0, C=None) == -3
    # alpha == 0: A and B may be NULL
    assert _consumer_call(lib, alpha=0.0, A=None, B=None) == -3
    assert _consumer_call(lib, tile=(32, 32, 8, 32, 32, 2)) == -2
    assert _consumer_call(lib, m=0) == 0  # empty: quick return


def test_pair_validation(lib, monkeypatch):
    def call(**kw):
        a = dict(m=64, n=48, k=32, A=FAKE, lda=32, a1=1.0, B1=FAKE + (1 << 24), ldb1=48, b1=1.0,
                 C1=FAKE + (2 << 24), ldc1=48, a2=1.0, B2=FAKE + (3 << 24), ldb2=48, b2=0.0,
                 C2=FAKE + (4 << 24), ldc2=48, tile=None)
        a.update(kw)
        t = ctypes.byref(_lib.Tile(*a["tile"])) if a["tile"] is not None else None
        return lib.hpvm_sgemm_pair(a["m"], a["n"], a["k"], a["A"], a["lda"], a["a1"], a["B1"], a["ldb1"],
                                   a["b1"], a["C1"], a["ldc1"], a["a2"], a["B2"], a["ldb2"], a["b2"],
                                   a["C2"], a["ldc2"], t, None)

    assert call(C2=FAKE + (2 << 24) + 128) == -1 and "overlap" in hp.last_error()
    assert call(C1=FAKE + (3 << 24)) == -1 and "C1 overlaps B2" in hp.last_error()
    assert call(B2=None) == -1 and "output 2" in hp.last_error()
    assert call(lda=31) == -1 and "output 1" in hp.last_error()
    assert call(tile=(128, 128, 32, 64, 64, 2)) == -2
    assert call(n=0) == 0
    monkeypatch.setenv("HPVM_FAULT_INJECT", "launch")
    assert call() == -3


def test_tracker_table_host_side(lib, monkeypatch):
    """Track / state / request / untrack on host memory; no copy is needed, so no HIP call."""
    import numpy as np

    base = hp.tracker_counters()
    A = np.zeros((8, 8), np.float32)
    B = np.zeros((8, 8), np.float32)
    hp.track(A)
    hp.track(B)
    with pytest.raises(hp.HpvmError) as ei:
        hp.track(A)  # already tracked: overlap
    assert ei.value.status == -1
    assert lib.hpvm_track_mem(ctypes.c_void_p(A.ctypes.data + 16), 16) == -1  # inside A
    st = hp.tracked_state(A[3:])  # any address inside the region resolves to it
    assert st["start"] == A.ctypes.data and st["bytes"] == A.nbytes
    assert st["on_host"] and not st["on_device"] and st["device"] == 0
    hp.request(A)  # host copy is current: nothing to copy
    assert lib.hpvm_request_mem(ctypes.c_void_p(A.ctypes.data), A.nbytes + 4, None) == -1  # past the region
    assert lib.hpvm_untrack_mem(ctypes.c_void_p(A.ctypes.data + 4), None) == -1  # not a region start
    C = np.zeros((8, 8), np.float32)
    # the launch refuses untracked operands, in argument order
    assert lib.hpvm_sgemm_tracked(8, 8, 8, 1.0, ctypes.c_void_p(C.ctypes.data), 8, ctypes.c_void_p(B.ctypes.data),
                                  8, 0.0, ctypes.c_void_p(A.ctypes.data), 8, 0, None, None) == -1
    assert "argument 5" in hp.last_error()
    assert lib.hpvm_sgemm_tracked(8, 8, 8, 1.0, ctypes.c_void_p(A.ctypes.data), 8, ctypes.c_void_p(B.ctypes.data),
                                  8, 0.0, ctypes.c_void_p(C.ctypes.data), 8, 0, None, None) == -1
    assert "argument 10" in hp.last_error()
    hp.track(C)
    monkeypatch.setenv("HPVM_FAULT_INJECT", "launch")
    assert lib.hpvm_sgemm_tracked(8, 8, 8, 1.0, ctypes.c_void_p(A.ctypes.data), 8, ctypes.c_void_p(B.ctypes.data),
                                  8, 0.0, ctypes.c_void_p(C.ctypes.data), 8, 0, None, None) == -3
    # the first device copy's allocation fails: an error, and the table is as before
    monkeypatch.setenv("HPVM_FAULT_INJECT", "alloc")
    assert lib.hpvm_sgemm_tracked(8, 8, 8, 1.0, ctypes.c_void_p(A.ctypes.data), 8, ctypes.c_void_p(B.ctypes.data),
                                  8, 0.0, ctypes.c_void_p(C.ctypes.data), 8, 0, None, None) == -3
    assert "tracked copy" in hp.last_error()
    for x in (A, B, C):
        st = hp.tracked_state(x)
        assert st["on_host"] and not st["on_device"] and st["device"] == 0
    monkeypatch.delenv("HPVM_FAULT_INJECT")
    assert hp.tracker_counters()["regions"] == base["regions"] + 3
    assert hp.tracker_counters()["h2d_copies"] == base["h2d_copies"]
    for x in (A, B, C):
        hp.untrack(x)
    after = hp.tracker_counters()
    assert after["regions"] == base["regions"] and after["h2d_copies"] == base["h2d_copies"]
    with pytest.raises(hp.HpvmError):
        hp.tracked_state(A)



def test_staged_tiles_refuse_too_deep_a_contraction(lib):
    """Staged loads use 32-bit offsets within a tile's rows of a plane: k must
    stay below 2^32 / (256 rows * 2 bytes) once padded; deeper k is refused."""
    BIG = 1 << 40  # fake, never dereferenced: the check comes first
    staged = [t for t in hp.tile_menu("bf16") if t[5] == 3][0]
    t = ctypes.byref(_lib.Tile(*staged))
    k = 1 << 23
    rc = lib.hpvm_sgemm_ws(4, 4, k, 1.0, BIG, k, BIG * 2, 4, 0.0, BIG * 3, 4, hp.PREC["bf16"], t,
                           BIG * 4, 1 << 40, None)
    assert rc == -2 and "too deep" in hp.last_error()
    # one padded block less is accepted (stopped by the fault injection instead)
    import os
    os.environ["HPVM_FAULT_INJECT"] = "launch"
    try:
        k = (1 << 23) - 64
        rc = lib.hpvm_sgemm_ws(4, 4, k, 1.0, BIG, k, BIG * 2, 4, 0.0, BIG * 3, 4, hp.PREC["bf16"], t,
                               BIG * 4, 1 << 40, None)
        assert rc == -3
    finally:
        del os.environ["HPVM_FAULT_INJECT"]


def test_workspace_choice_fits_the_workspace(lib):
    """With no tile, hpvm_sgemm_ws takes the staged BF16 / bf16x3 planes only
    when the workspace holds them; a smaller one gives the choice without a
    workspace instead of a refusal."""
    hp.autotune_clear()
    for prec, size in (("bf16", 8192), ("bf16x3", 2048)):
        big = hp.describe(size, size, size, prec, workspace_bytes=1 << 40)
        assert big["lowering_name"] == f"staged_{prec}"
        need = hp.workspace_bytes(size, size, size, prec, big["tile"])
        assert hp.describe(size, size, size, prec, workspace_bytes=need)["lowering_name"] == f"staged_{prec}"
        small = hp.describe(size, size, size, prec, workspace_bytes=need - 1)
        assert small["lowering_name"] != f"staged_{prec}"
        assert small["tile"] == hp.describe(size, size, size, prec)["tile"]
    # bf16x3 products that 256 x 256 tiles cover take the DMA-fed tile,
    # which converts in its own load path: no workspace
    d = hp.describe(8192, 8192, 8192, "bf16x3", workspace_bytes=1 << 40)
    assert d["lowering_name"] == "mfma_bf16x3" and d["tile"] == hp.tile_menu("bf16x3")[0]
    assert hp.workspace_bytes(8192, 8192, 8192, "bf16x3") == 0


def test_noalloc_checks_before_device_work(lib, monkeypatch):
    """hpvm_sgemm_noalloc: argument checks, and the refusal of a staged tile
    whose planes exceed the fixed array, happen before any HIP call."""
    text = open(HEADER).read()
    m = re.search(r"#define HPVM_NOALLOC_SCRATCH_BYTES \(\(int64_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == hp.NOALLOC_SCRATCH_BYTES
    BIG = 1 << 28  # far enough apart that no two matrices overlap
    bf16 = hp.PREC["bf16"]
    staged = [t for t in hp.tile_menu("bf16") if t[5] == 3][0]
    t = ctypes.byref(_lib.Tile(*staged))
    assert hp.workspace_bytes(4096, 4096, 4096, "bf16", staged) > hp.NOALLOC_SCRATCH_BYTES
    rc = lib.hpvm_sgemm_noalloc(4096, 4096, 4096, 1.0, BIG, 4096, BIG * 2, 4096, 0.0, BIG * 4, 4096, bf16, t, None)
    assert rc == -4 and "scratch" in hp.last_error()
    rc = lib.hpvm_sgemm_noalloc(-1, 4, 4, 1.0, BIG, 4, BIG * 2, 4, 0.0, BIG * 4, 4, bf16, None, None)
    assert rc == -1 and "argument 1" in hp.last_error()
    rc = lib.hpvm_sgemm_noalloc(4, 4, 4, 1.0, BIG, 4, BIG * 2, 4, 0.0, BIG * 4, 4, 9, None, None)
    assert rc == -1 and "argument 12" in hp.last_error()
    # calls that fit pass every check (the injected failure stops them)
    monkeypatch.setenv("HPVM_FAULT_INJECT", "launch")
    for prec, size in (("bf16", 2048), ("bf16x3", 2048), ("fp32", 1024), ("bf16", 4096)):
        rc = lib.hpvm_sgemm_noalloc(size, size, 4096, 1.0, BIG, 4096, BIG * 2, size, 0.0, BIG * 4, size,
                                    hp.PREC[prec], None, None)
        assert rc == -3, (prec, size, hp.last_error())


def test_pair_split_workspace_rules(lib, monkeypatch):
    """hpvm_sgemm_pair_ws splits the contraction of pairs whose tiles would
    not cover 256 CUs (the single launch's slice rule, on 128 x 128 tiles
    per output); the workspace holds both outputs' partial sums."""
    plane = lambda m, n: 4 * m * n
    split = (128, 128, 32, 32, 128, 2)
    # 64 tiles of 128 x 128 per output -> 4 slices of 1024
    assert hp.pair_workspace_bytes(1024, 1024, 4096) == 2 * 4 * plane(1024, 1024)
    assert hp.pair_workspace_bytes(1024, 1024, 4096, split) == 2 * 4 * plane(1024, 1024)
    assert hp.pair_workspace_bytes(512, 512, 4096) == 2 * 16 * plane(512, 512)
    for m, n, k, tile in ((4096, 4096, 4096, None),    # the first pair tile covers the CUs
                          (1024, 1024, 4096, (128, 128, 16, 64, 64, 2)),  # not a splitting tile
                          (1000, 1024, 4096, split),     # not whole tiles
                          (1024, 1024, 256, split)):     # slices would be under 256 deep
        assert hp.pair_workspace_bytes(m, n, k, tile) == 0, (m, n, k, tile)
    BIG = 1 << 28
    A, B1, C1, B2, C2 = BIG, 2 * BIG, 3 * BIG, 4 * BIG, 5 * BIG
    args = (1024, 1024, 4096, A, 4096, 1.0, B1, 1024, 0.0, C1, 1024, 1.0, B2, 1024, 0.0, C2, 1024, None)
    assert lib.hpvm_sgemm_pair_ws(*args, 6 * BIG, -1, None) == -1 and "argument 20" in hp.last_error()
    assert lib.hpvm_sgemm_pair_ws(*args, 6 * BIG + 4, 1 << 30, None) == -1 and "argument 19" in hp.last_error()
    monkeypatch.setenv("HPVM_FAULT_INJECT", "launch")
    assert lib.hpvm_sgemm_pair_ws(*args, 6 * BIG, 1 << 30, None) == -3
    assert lib.hpvm_sgemm_pair_ws(*args, None, 0, None) == -3  # no workspace: the unsplit pair


def test_autotune_cache_persists_through_the_environment(tmp_path):
    """HPVM_AUTOTUNE_CACHE: a choice recorded in one process is written to the
    file and found by the next process that names it; without it, nothing
    carries over."""
    import sys

    path = tmp_path / "tune.txt"

    def run(code, cache):
        env = dict(os.environ)
        env.pop("HPVM_AUTOTUNE_CACHE", None)
        if cache:
            env["HPVM_AUTOTUNE_CACHE"] = str(path)
        out = subprocess.run([sys.executable, "-c", "import paper_1611_00860_amd as hp\n" + code], cwd=ROOT, env=env,
                             capture_output=True, text=True, timeout=300)
        assert out.returncode == 0, out.stderr[-2000:]
        return out.stdout.strip()

    menu = hp.tile_menu("fp32")
    run(f"hp.autotune_record(4096, 4096, 4096, {tuple(menu[2])}, 'fp32', 1.25)", cache=True)
    assert path.exists() and "4096 4096 4096" in path.read_text()
    assert [p.name for p in tmp_path.iterdir()] == ["tune.txt"]  # written aside, then renamed over
    got = run("t, f = hp.autotune_lookup(4096, 4096, 4096, 'fp32'); print(list(t), f, "
              "list(hp.describe(4096, 4096, 4096, 'fp32')['tile']))", cache=True)
    assert got == f"{list(menu[2])} 2 {list(menu[2])}"
    assert run("print(hp.autotune_lookup(4096, 4096, 4096, 'fp32')[1])", cache=False) == "0"
