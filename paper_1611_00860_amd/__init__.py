"""MI355X (gfx950) lowering of the HPVM sgemm dataflow graph -- Python binding.

Thin marshalling over the C ABI in ``include/hpvm_sgemm.h``: every call here
checks tensor types, takes device pointers and torch's current HIP stream, and
calls the library of the same name.  All arithmetic runs in the library's HIP
kernels; there is no CPU fallback, and a missing library raises ImportError.

HPVM technical report (arXiv:1611.00860): the sgemm graph of Sec. 6.1, its GPU
lowering of Sec. 3.4 and 6.2-6.3.
"""
from __future__ import annotations

import atexit
import ctypes

from . import _lib

PREC = {"fp32": 0, "bf16": 1, "bf16x3": 2}
LOWERINGS = {0: "literal", 1: "mfma_f32", 2: "mfma_bf16", 3: "mfma_bf16x3", 4: "staged_bf16",
             5: "staged_bf16x3", 6: "flat"}


class HpvmError(RuntimeError):
    """A non-zero status from the library, with its detail text."""

    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__(f"{status_string(status)} ({status}): {detail}")


def load():
    """Load the HIP library (binding it to torch's HIP runtime)."""
    return _lib.load()


def status_string(status: int) -> str:
    return load().hpvm_status_string(status).decode()


def last_error() -> str:
    return load().hpvm_last_error().decode()


def _check(rc: int):
    if rc != 0:
        raise HpvmError(rc, last_error())


def _prec(prec) -> int:
    if isinstance(prec, str):
        return PREC[prec]
    return int(prec)


def _tile(tile):
    if tile is None:
        return None
    if isinstance(tile, _lib.Tile):
        return ctypes.byref(tile)
    return ctypes.byref(_lib.Tile(*[int(v) for v in tile]))


def _stream(stream=None):
    import torch

    if stream is None:
        if not torch.cuda.is_available():
            return ctypes.c_void_p(None)  # host-only calls; a HIP call then fails loudly
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _empty(shape, dtype, device, stream=None):
    """torch.empty on the stream the library will use the memory on.

    Scratch memory a call hands to the library is used on ``stream`` (when
    given, else torch's current stream).  Allocating it under that stream
    makes torch's caching allocator order its reuse after the work queued
    there: a block freed when this call returns is not handed to another
    allocation until the stream's kernels have finished with it.
    """
    import torch

    if stream is None:
        return torch.empty(shape, dtype=dtype, device=device)
    with torch.cuda.stream(stream):
        return torch.empty(shape, dtype=dtype, device=device)


def _mat(t, name, rows=None, cols=None):
    """(pointer, leading dimension) of a 2-D row-major float32 device tensor."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float32 or t.dim() != 2:
        raise TypeError(f"{name} must be a 2-D float32 tensor")
    if not t.is_cuda:
        raise TypeError(f"{name} must live on the GPU")
    if t.numel() and t.stride(1) != 1 and t.shape[1] > 1:
        raise ValueError(f"{name} must have unit column stride (row-major)")
    ld = t.stride(0) if t.shape[0] > 1 else max(t.shape[1], 1)
    return ctypes.c_void_p(t.data_ptr() if t.numel() else 0), max(ld, 1)


def workspace_bytes(m: int, n: int, k: int, prec="fp32", tile=None) -> int:
    """Workspace hpvm_sgemm_ws needs: the staged lowering's planes or a split
    FP32 contraction's partial sums, else 0."""
    out = ctypes.c_int64(0)
    _check(load().hpvm_sgemm_workspace_bytes(m, n, k, _prec(prec), _tile(tile), ctypes.byref(out)))
    return out.value


def sgemm(A, B, C, alpha: float = 1.0, beta: float = 0.0, prec="fp32", tile=None, stream=None,
          workspace=None):
    """C <- alpha * A @ B + beta * C in place; returns C.

    A (m x k), B (k x n), C (m x n): float32 CUDA tensors, row-major, any
    leading dimension.  ``prec`` is 'fp32', 'bf16' or 'bf16x3'; ``tile`` is
    None (autotuned or default) or (tile_m, tile_n, tile_k, leaf_m, leaf_n,
    stages).  Tiles of the staged lowering (stages = 3) need a workspace,
    and FP32 problems that a DMA-fed tile splits into contraction slices use
    one: ``workspace`` (a CUDA tensor) is used when given and large enough,
    else one is allocated from torch's caching allocator for the call
    (hpvm_sgemm_ws).  ``workspace=False`` calls hpvm_sgemm, which takes none
    (FP32 then runs as one launch; staged tiles are refused).
    """
    import torch

    lib = load()
    m, k = A.shape
    k2, n = B.shape
    if k2 != k or tuple(C.shape) != (m, n):
        raise ValueError(f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}, C {tuple(C.shape)}")
    pa, lda = _mat(A, "A")
    pb, ldb = _mat(B, "B")
    pc, ldc = _mat(C, "C")
    need = 0 if workspace is False else workspace_bytes(m, n, k, prec, tile)
    if need == 0:
        _check(lib.hpvm_sgemm(m, n, k, float(alpha), pa, lda, pb, ldb, float(beta), pc, ldc,
                              _prec(prec), _tile(tile), _stream(stream)))
        return C
    if workspace is None or workspace.numel() * workspace.element_size() < need:
        workspace = _empty(need, torch.uint8, C.device, stream)
    _check(lib.hpvm_sgemm_ws(m, n, k, float(alpha), pa, lda, pb, ldb, float(beta), pc, ldc,
                             _prec(prec), _tile(tile), ctypes.c_void_p(workspace.data_ptr()),
                             workspace.numel() * workspace.element_size(), _stream(stream)))
    return C


# Bytes of the device array hpvm_sgemm_noalloc uses as its workspace (the
# header's HPVM_NOALLOC_SCRATCH_BYTES).
NOALLOC_SCRATCH_BYTES = 32 << 20


def sgemm_noalloc(A, B, C, alpha: float = 1.0, beta: float = 0.0, prec="fp32", tile=None, stream=None):
    """sgemm through hpvm_sgemm_noalloc: the library allocates nothing and its
    fixed per-device array serves as the workspace (calls that overlap on one
    device race on it).  Same arguments and results as ``sgemm`` with a
    workspace of NOALLOC_SCRATCH_BYTES."""
    lib = load()
    m, k = A.shape
    k2, n = B.shape
    if k2 != k or tuple(C.shape) != (m, n):
        raise ValueError(f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}, C {tuple(C.shape)}")
    pa, lda = _mat(A, "A")
    pb, ldb = _mat(B, "B")
    pc, ldc = _mat(C, "C")
    _check(lib.hpvm_sgemm_noalloc(m, n, k, float(alpha), pa, lda, pb, ldb, float(beta), pc, ldc,
                                  _prec(prec), _tile(tile), _stream(stream)))
    return C


def launch_root(A, B, C, k: int, alpha: float, beta: float, block, grid, stream=None,
                bytes_override=None):
    """The root node's launch with the paper's packed 88-byte argument block.

    ``block`` = (block_x, block_y) leaf instances per internal instance and
    ``grid`` = (grid_x, grid_y) internal instances; m = grid_y * block_y and
    n = grid_x * block_x.  Byte extents are those of the tensors' storage
    unless ``bytes_override`` = (bytesA, bytesB, bytesC) is given.
    """
    lib = load()
    pa, lda = _mat(A, "A")
    pb, ldb = _mat(B, "B")
    pc, ldc = _mat(C, "C")

    def nbytes(t):
        return (t.untyped_storage().nbytes() - t.storage_offset() * 4) if t.numel() else 0

    bA, bB, bC = bytes_override or (nbytes(A), nbytes(B), nbytes(C))
    r = _lib.RootIn(pa.value, bA, lda, pb.value, bB, ldb, pc.value, bC, ldc, int(k),
                    float(alpha), float(beta), int(block[0]), int(block[1]), int(grid[0]),
                    int(grid[1]))
    _check(lib.hpvm_launch_root(ctypes.byref(r), _stream(stream)))
    return C


def wait(stream=None):
    """Complete all work on the stream (hpvm_wait)."""
    _check(load().hpvm_wait(_stream(stream)))


def alloc_bytes(tile, prec="fp32") -> int:
    """The Allocation node: LDS bytes per SgemmInternal instance."""
    out = ctypes.c_int64(0)
    _check(load().hpvm_alloc_bytes(_tile(tile), _prec(prec), ctypes.byref(out)))
    return out.value


def describe(m: int, n: int, k: int, prec="fp32", tile=None, workspace_bytes=None) -> dict:
    """Grid / block / LDS / lowering / contraction slices of one launch:
    hpvm_sgemm's (hpvm_describe), or with ``workspace_bytes`` hpvm_sgemm_ws's
    given a workspace of that size (hpvm_describe_ws)."""
    d = _lib.Dfg()
    if workspace_bytes is None:
        _check(load().hpvm_describe(m, n, k, _prec(prec), _tile(tile), ctypes.byref(d)))
    else:
        _check(load().hpvm_describe_ws(m, n, k, _prec(prec), _tile(tile), int(workspace_bytes), ctypes.byref(d)))
    out = {f: getattr(d, f) for f, _ in _lib.Dfg._fields_ if f not in ("reserved", "tile")}
    out["tile"] = d.tile.as_tuple()
    out["lowering_name"] = LOWERINGS.get(d.lowering, "?")
    return out


def dfg_edges() -> list:
    """The static edge / binding table of the sgemm graph."""
    lib = load()
    count = ctypes.c_int32(0)
    _check(lib.hpvm_dfg_edges(None, 0, ctypes.byref(count)))
    arr = (_lib.Edge * count.value)()
    _check(lib.hpvm_dfg_edges(arr, count.value, ctypes.byref(count)))
    return [{f: getattr(e, f) for f, _ in _lib.Edge._fields_} for e in arr]


def tile_menu(prec="fp32") -> list:
    """Compiled tiles for a precision; entry 0 is the default."""
    lib = load()
    count = ctypes.c_int32(0)
    _check(lib.hpvm_tile_menu(_prec(prec), None, 0, ctypes.byref(count)))
    arr = (_lib.Tile * count.value)()
    _check(lib.hpvm_tile_menu(_prec(prec), arr, count.value, ctypes.byref(count)))
    return [t.as_tuple() for t in arr]


# ---------------------------------------------------------------------------
# Backward pass
# ---------------------------------------------------------------------------
def backward_workspace_bytes(m: int, n: int, k: int, prec="fp32", tile=None) -> int:
    out = ctypes.c_int64(0)
    _check(load().hpvm_sgemm_backward_workspace_bytes(m, n, k, _prec(prec), _tile(tile), ctypes.byref(out)))
    return out.value


def backward_menu(prec="fp32") -> list:
    """Tiles the backward can use at `prec`."""
    lib = load()
    count = ctypes.c_int32(0)
    _check(lib.hpvm_sgemm_backward_menu(_prec(prec), None, 0, ctypes.byref(count)))
    arr = (_lib.Tile * count.value)()
    _check(lib.hpvm_sgemm_backward_menu(_prec(prec), arr, count.value, ctypes.byref(count)))
    return [t.as_tuple() for t in arr]


def sgemm_backward(A, B, C_in, G, alpha: float, beta: float, prec="fp32", need=("dA", "dB", "dC_in",
                   "dalpha", "dbeta"), tile=None, stream=None) -> dict:
    """Gradients of <G, alpha A B + beta C_in> (hpvm_sgemm_backward).

    Returns a dict with the requested entries of dA, dB, dC_in (tensors) and
    dalpha, dbeta (0-dim device tensors).
    """
    import torch

    lib = load()
    m, k = A.shape
    n = B.shape[1]
    dev = G.device
    out = {}
    if "dA" in need:
        out["dA"] = _empty((m, k), torch.float32, dev, stream)
    if "dB" in need:
        out["dB"] = _empty((k, n), torch.float32, dev, stream)
    if "dC_in" in need:
        out["dC_in"] = _empty((m, n), torch.float32, dev, stream)
    scal = _empty(2, torch.float32, dev, stream)  # the call writes each requested scalar
    nbytes = backward_workspace_bytes(m, n, k, prec, tile)
    ws = _empty(max(nbytes, 16), torch.uint8, dev, stream)

    def mat(name, t, rows, cols):
        if t is None:
            return ctypes.c_void_p(0), max(cols, 1)
        return _mat(t, name)

    pa, lda = mat("A", A, m, k)
    pb, ldb = mat("B", B, k, n)
    pci, ldci = mat("C_in", C_in if "dbeta" in need else None, m, n)
    pg, ldg = mat("G", G, m, n)
    pda, ldda = mat("dA", out.get("dA"), m, k)
    pdb, lddb = mat("dB", out.get("dB"), k, n)
    pdc, lddc = mat("dC_in", out.get("dC_in"), m, n)
    base = scal.data_ptr()
    da = ctypes.c_void_p(base) if "dalpha" in need else ctypes.c_void_p(0)
    db = ctypes.c_void_p(base + 4) if "dbeta" in need else ctypes.c_void_p(0)
    _check(lib.hpvm_sgemm_backward(m, n, k, float(alpha), float(beta), pa, lda, pb, ldb, pci, ldci,
                                   pg, ldg, pda, ldda, pdb, lddb, pdc, lddc, da, db, _prec(prec),
                                   _tile(tile), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                   _stream(stream)))
    if "dalpha" in need:
        out["dalpha"] = scal[0]
    if "dbeta" in need:
        out["dbeta"] = scal[1]
    out["_keep"] = ws
    return out


def autotune_backward(A, B, G, prec="fp32", reps: int = 3, stream=None):
    """Times every backward tile for these operands; caches and returns (tile, ms)."""
    import torch

    lib = load()
    m, k = A.shape
    n = B.shape[1]
    dev = G.device
    need = max(backward_workspace_bytes(m, n, k, prec, t) for t in backward_menu(prec)) + 256
    ws = _empty(need, torch.uint8, dev, stream)
    dA = _empty((m, k), torch.float32, dev, stream)
    dB = _empty((k, n), torch.float32, dev, stream)
    pa, lda = _mat(A, "A")
    pb, ldb = _mat(B, "B")
    pg, ldg = _mat(G, "G")
    best = _lib.Tile()
    ms = ctypes.c_float(0.0)
    _check(lib.hpvm_autotune_backward(m, n, k, _prec(prec), pa, lda, pb, ldb, pg, ldg,
                                      ctypes.c_void_p(dA.data_ptr()), k, ctypes.c_void_p(dB.data_ptr()), n,
                                      ctypes.c_void_p(ws.data_ptr()), need, int(reps), _stream(stream),
                                      ctypes.byref(best), ctypes.byref(ms)))
    return best.as_tuple(), ms.value


# ---------------------------------------------------------------------------
# Autotuner of single launches
# ---------------------------------------------------------------------------
def autotune(A, B, prec="fp32", reps: int = 5, scratch=None, stream=None, allow_workspace=True):
    """Times every compiled tile for A @ B at `prec`; caches and returns (tile, ms).

    ``scratch`` (m x n float32, overwritten) is allocated when not given;
    with ``allow_workspace`` the staged tiles are timed too, and FP32 tiles
    that split the contraction run split, on a workspace allocated for the
    call.
    """
    import torch

    m, k = A.shape
    n = B.shape[1]
    if scratch is None:
        scratch = _empty((m, n), torch.float32, A.device, stream)
    need = 0
    if allow_workspace:
        need = max([workspace_bytes(m, n, k, prec, t) for t in tile_menu(prec)] + [0])
    ws = _empty(max(need, 1), torch.uint8, A.device, stream)
    pa, lda = _mat(A, "A")
    pb, ldb = _mat(B, "B")
    pc, ldc = _mat(scratch, "scratch")
    best = _lib.Tile()
    ms = ctypes.c_float(0.0)
    _check(load().hpvm_autotune(m, n, k, _prec(prec), pa, lda, pb, ldb, pc, ldc,
                                ctypes.c_void_p(ws.data_ptr()), need, int(reps), _stream(stream),
                                ctypes.byref(best), ctypes.byref(ms)))
    return best.as_tuple(), ms.value


def autotune_lookup(m: int, n: int, k: int, prec="fp32"):
    """(tile, found): found = 2 exact, 1 shape class, 0 default."""
    t = _lib.Tile()
    found = ctypes.c_int32(0)
    _check(load().hpvm_autotune_lookup(m, n, k, _prec(prec), ctypes.byref(t), ctypes.byref(found)))
    return t.as_tuple(), found.value


def autotune_record(m: int, n: int, k: int, tile, prec="fp32", ms: float = 0.0):
    _check(load().hpvm_autotune_record(m, n, k, _prec(prec), _tile(tile), float(ms)))


def autotune_clear():
    _check(load().hpvm_autotune_clear())


def autotune_save(path: str):
    _check(load().hpvm_autotune_save(str(path).encode()))


def autotune_load(path: str):
    _check(load().hpvm_autotune_load(str(path).encode()))


# ---------------------------------------------------------------------------
# Grouped launch
# ---------------------------------------------------------------------------
def grouped_menu() -> list:
    """Tile shapes the grouped persistent kernel supports."""
    lib = load()
    count = ctypes.c_int32(0)
    _check(lib.hpvm_grouped_menu(None, 0, ctypes.byref(count)))
    arr = (_lib.Tile * count.value)()
    _check(lib.hpvm_grouped_menu(arr, count.value, ctypes.byref(count)))
    return [t.as_tuple() for t in arr]


class Graph:
    """An instantiated HIP graph of a grouped launch (hpvm_graph_*)."""

    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep  # tensors the graph reads or writes

    def launch(self, stream=None):
        _check(load().hpvm_graph_launch(self._h, _stream(stream)))

    def destroy(self):
        if self._h is not None:
            _check(load().hpvm_graph_destroy(self._h))
            self._h = None


class GroupedPlan:
    """Many independent sgemms C_i <- alpha_i A_i B_i + beta_i C_i in one launch.

    Holds references to every tensor so they outlive the plan; the device
    workspace is a torch allocation of the size the library asks for.
    """

    def __init__(self, As, Bs, Cs, alphas, betas, prec="fp32", tile=None):
        import torch

        lib = load()
        n = len(As)
        if not (len(Bs) == len(Cs) == len(alphas) == len(betas) == n):
            raise ValueError("As, Bs, Cs, alphas, betas must have the same length")
        descs = (_lib.SgemmDesc * max(n, 1))()
        for i, (A, B, C) in enumerate(zip(As, Bs, Cs)):
            m, k = A.shape
            k2, nn = B.shape
            if k2 != k or tuple(C.shape) != (m, nn):
                raise ValueError(f"instance {i}: shape mismatch")
            pa, lda = _mat(A, f"A[{i}]")
            pb, ldb = _mat(B, f"B[{i}]")
            pc, ldc = _mat(C, f"C[{i}]")
            descs[i] = _lib.SgemmDesc(m, nn, k, float(alphas[i]), float(betas[i]), pa.value, lda,
                                      pb.value, ldb, pc.value, ldc)
        h = ctypes.c_void_p()
        _check(lib.hpvm_grouped_plan_create(n, descs, _prec(prec), _tile(tile), ctypes.byref(h)))
        self._h = h
        self._keep = (list(As), list(Bs), list(Cs))
        self.workspace = torch.empty(max(self.info()["workspace_bytes"], 16), dtype=torch.uint8,
                                     device=Cs[0].device if n else "cuda")

    def info(self) -> dict:
        inf = _lib.GroupedInfo()
        _check(load().hpvm_grouped_plan_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in _lib.GroupedInfo._fields_}

    def instance_tile(self, i: int):
        t = _lib.Tile()
        _check(load().hpvm_grouped_instance_tile(self._h, int(i), ctypes.byref(t)))
        return t.as_tuple()

    def _ws(self, stream=None):
        if stream is not None:  # freed with the plan: not before that stream's work is done
            self.workspace.record_stream(stream)
        return ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel()

    def run(self, stream=None):
        ws, nb = self._ws(stream)
        _check(load().hpvm_grouped_run(self._h, ws, nb, _stream(stream)))

    def autotune(self, reps: int = 3, stream=None) -> float:
        """Times candidate shape assignments on scratch outputs; keeps the fastest."""
        import torch

        scratch = _empty(max(self.info()["scratch_bytes"] // 4, 1), torch.float32, self.workspace.device, stream)
        ws, nb = self._ws(stream)
        best = ctypes.c_float(0.0)
        _check(load().hpvm_grouped_autotune(self._h, ws, nb, ctypes.c_void_p(scratch.data_ptr()),
                                            scratch.numel() * 4, int(reps), _stream(stream),
                                            ctypes.byref(best)))
        return best.value

    def capture(self, stream=None) -> Graph:
        ws, nb = self._ws(stream)
        g = ctypes.c_void_p()
        _check(load().hpvm_grouped_capture(self._h, ws, nb, _stream(stream), ctypes.byref(g)))
        return Graph(g, (self._keep, self.workspace))

    def destroy(self):
        if self._h is not None:
            _check(load().hpvm_grouped_plan_destroy(self._h))
            self._h = None


# ---------------------------------------------------------------------------
# Node fusion: sgemm + one-to-one consumer, two sgemms sharing A
# ---------------------------------------------------------------------------
CONSUMER_OPS = {"none": 0, "relu": 1, "bias": 2, "bias_relu": 3, "clamp": 4}
FUSIONS = {"consumer": 0, "pair": 1}


def fusion_menu(which="consumer") -> list:
    """Tiles compiled for a fusion ('consumer' or 'pair'); entry 0 is the default."""
    lib = load()
    w = FUSIONS[which] if isinstance(which, str) else int(which)
    count = ctypes.c_int32(0)
    _check(lib.hpvm_fusion_menu(w, None, 0, ctypes.byref(count)))
    arr = (_lib.Tile * count.value)()
    _check(lib.hpvm_fusion_menu(w, arr, count.value, ctypes.byref(count)))
    return [t.as_tuple() for t in arr]


def sgemm_consumer(A, B, C, alpha: float = 1.0, beta: float = 0.0, op="none", bias=None,
                   lo: float = float("-inf"), hi: float = float("inf"), D=None, tile=None, stream=None):
    """D <- op(alpha A B + beta C) in one launch (hpvm_sgemm_consumer); returns D.

    ``C`` may be None when beta == 0; ``D`` defaults to C (in place) when C
    is given, else to a new tensor.  ``bias``: float32 device vector of n.
    """
    import torch

    lib = load()
    m, k = A.shape
    k2, n = B.shape
    if k2 != k:
        raise ValueError(f"shape mismatch: A {tuple(A.shape)}, B {tuple(B.shape)}")
    if D is None:
        D = C if C is not None else _empty((m, n), torch.float32, A.device, stream)
    if tuple(D.shape) != (m, n) or (C is not None and tuple(C.shape) != (m, n)):
        raise ValueError("C and D must be m x n")
    pa, lda = _mat(A, "A")
    pb, ldb = _mat(B, "B")
    pc, ldc = _mat(C, "C") if C is not None else (ctypes.c_void_p(0), max(n, 1))
    pd, ldd = _mat(D, "D")
    code = CONSUMER_OPS[op] if isinstance(op, str) else int(op)
    pbias = 0
    if bias is not None:
        if bias.dtype != torch.float32 or not bias.is_cuda or tuple(bias.shape) != (n,) or \
                (n > 1 and bias.stride(0) != 1):
            raise TypeError("bias must be a contiguous float32 CUDA vector of length n")
        pbias = bias.data_ptr()
    cons = _lib.Consumer(code, 0, pbias, float(lo), float(hi))
    _check(lib.hpvm_sgemm_consumer(m, n, k, float(alpha), pa, lda, pb, ldb, float(beta), pc, ldc,
                                   ctypes.byref(cons), pd, ldd, _tile(tile), _stream(stream)))
    return D


def pair_workspace_bytes(m: int, n: int, k: int, tile=None) -> int:
    """Workspace hpvm_sgemm_pair_ws needs: the split pair's partial sums, else 0."""
    out = ctypes.c_int64(0)
    _check(load().hpvm_sgemm_pair_workspace_bytes(m, n, k, _tile(tile), ctypes.byref(out)))
    return out.value


def sgemm_pair(A, B1, C1, B2, C2, alpha1: float = 1.0, beta1: float = 0.0, alpha2: float = 1.0,
               beta2: float = 0.0, tile=None, stream=None, workspace=None):
    """C1 <- alpha1 A B1 + beta1 C1 and C2 <- alpha2 A B2 + beta2 C2 in one launch.

    Pairs whose tiles would not cover the CUs split the contraction into
    slices when a workspace holds the partial sums (hpvm_sgemm_pair_ws):
    ``workspace`` (a CUDA tensor) is used when given and large enough, else
    one is allocated on the call's stream; ``workspace=False`` calls
    hpvm_sgemm_pair, which takes none.
    """
    import torch

    lib = load()
    m, k = A.shape
    n = B1.shape[1]
    for name, X, shape in (("B1", B1, (k, n)), ("B2", B2, (k, n)), ("C1", C1, (m, n)), ("C2", C2, (m, n))):
        if tuple(X.shape) != shape:
            raise ValueError(f"{name} must be {shape[0]} x {shape[1]}")
    pa, lda = _mat(A, "A")
    p1, l1 = _mat(B1, "B1")
    q1, m1 = _mat(C1, "C1")
    p2, l2 = _mat(B2, "B2")
    q2, m2 = _mat(C2, "C2")
    need = 0 if workspace is False else pair_workspace_bytes(m, n, k, tile)
    if need == 0:
        _check(lib.hpvm_sgemm_pair(m, n, k, pa, lda, float(alpha1), p1, l1, float(beta1), q1, m1,
                                   float(alpha2), p2, l2, float(beta2), q2, m2, _tile(tile), _stream(stream)))
        return C1, C2
    if workspace is None or workspace.numel() * workspace.element_size() < need:
        workspace = _empty(need, torch.uint8, C1.device, stream)
    _check(lib.hpvm_sgemm_pair_ws(m, n, k, pa, lda, float(alpha1), p1, l1, float(beta1), q1, m1,
                                  float(alpha2), p2, l2, float(beta2), q2, m2, _tile(tile),
                                  ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size(),
                                  _stream(stream)))
    return C1, C2


# ---------------------------------------------------------------------------
# Memory tracker for host-resident arrays
# ---------------------------------------------------------------------------
def _host(x, name):
    """(address, bytes, row stride in elements) of a host float32 array or CPU tensor."""
    import numpy as np
    import torch

    if isinstance(x, np.ndarray):
        if x.dtype != np.float32 and name != "region":
            raise TypeError(f"{name} must be float32")
        if x.size == 0:  # numpy gives empty arrays zero strides
            return x.ctypes.data, 0, max(x.shape[-1] if x.ndim else 1, 1)
        ld = x.strides[0] // x.itemsize if x.ndim == 2 and x.shape[0] > 1 else (x.shape[-1] if x.ndim else 1)
        if x.ndim == 2 and x.shape[1] > 1 and x.strides[1] != x.itemsize:
            raise ValueError(f"{name} must have unit column stride (row-major)")
        return x.ctypes.data, x.nbytes, max(int(ld), 1)
    if isinstance(x, torch.Tensor):
        if x.is_cuda:
            raise TypeError(f"{name} must be host memory (the tracker manages the device copy)")
        if x.dtype != torch.float32 and name != "region":
            raise TypeError(f"{name} must be float32")
        ld = x.stride(0) if x.dim() == 2 and x.shape[0] > 1 else (x.shape[-1] if x.dim() else 1)
        if x.dim() == 2 and x.shape[1] > 1 and x.stride(1) != 1:
            raise ValueError(f"{name} must have unit column stride (row-major)")
        return x.data_ptr(), x.numel() * x.element_size(), max(int(ld), 1)
    raise TypeError(f"{name} must be a numpy array or a CPU torch tensor")


def track(x):
    """llvm_hpvm_track_mem on a host array (numpy or CPU tensor)."""
    addr, nbytes, _ = _host(x, "region")
    _check(load().hpvm_track_mem(ctypes.c_void_p(addr), nbytes))
    return x


def request(x, stream=None):
    """llvm_hpvm_request_mem: make the host copy of x current (copies back only if needed)."""
    addr, nbytes, _ = _host(x, "region")
    _check(load().hpvm_request_mem(ctypes.c_void_p(addr), nbytes, _stream(stream)))
    return x


def untrack(x, stream=None):
    """llvm_hpvm_untrack_mem: forget x and free its device copy."""
    addr, _, _ = _host(x, "region")
    _check(load().hpvm_untrack_mem(ctypes.c_void_p(addr), _stream(stream)))


def tracked_state(x) -> dict:
    addr, _, _ = _host(x, "region")
    st = _lib.Tracked()
    _check(load().hpvm_tracked_state(ctypes.c_void_p(addr), ctypes.byref(st)))
    return {"start": st.start or 0, "bytes": st.bytes, "device": st.device or 0,
            "on_host": bool(st.on_host), "on_device": bool(st.on_device)}


def tracker_counters() -> dict:
    st = _lib.TrackerStats()
    _check(load().hpvm_tracker_counters(ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in _lib.TrackerStats._fields_}


def sgemm_tracked(A, B, C, alpha: float = 1.0, beta: float = 0.0, prec="fp32", tile=None, stream=None):
    """C <- alpha A B + beta C on tracked host arrays (the latest C stays on the device until request(C))."""
    m, k = A.shape
    k2, n = B.shape
    if k2 != k or tuple(C.shape) != (m, n):
        raise ValueError("shape mismatch")
    pa, _, lda = _host(A, "A")
    pb, _, ldb = _host(B, "B")
    pc, _, ldc = _host(C, "C")
    _check(load().hpvm_sgemm_tracked(m, n, k, float(alpha), ctypes.c_void_p(pa), lda, ctypes.c_void_p(pb),
                                     ldb, float(beta), ctypes.c_void_p(pc), ldc, _prec(prec), _tile(tile),
                                     _stream(stream)))
    return C


# ---------------------------------------------------------------------------
# CPU (vector) lowering of the same graph: a separate target on host memory
# ---------------------------------------------------------------------------
def cpu_menu() -> list:
    lib = load()
    count = ctypes.c_int32(0)
    _check(lib.hpvm_cpu_menu(None, 0, ctypes.byref(count)))
    arr = (_lib.Tile * count.value)()
    _check(lib.hpvm_cpu_menu(arr, count.value, ctypes.byref(count)))
    return [t.as_tuple() for t in arr]


def cpu_isa() -> str:
    return load().hpvm_cpu_isa().decode()


def sgemm_cpu(A, B, C, alpha: float = 1.0, beta: float = 0.0, tile=None, threads: int = 0, k: int | None = None):
    """C <- alpha A B + beta C on host arrays with the CPU lowering (synchronous); returns C.

    A or B may be None when alpha == 0 or k == 0 (pass k then).
    """
    m, n = C.shape
    if A is not None:
        k = A.shape[1]
    elif k is None:
        raise ValueError("k is needed when A is None")
    pa, _, lda = _host(A, "A") if A is not None else (0, 0, max(k, 1))
    pb, _, ldb = _host(B, "B") if B is not None else (0, 0, max(n, 1))
    pc, _, ldc = _host(C, "C")
    if A is not None and tuple(A.shape) != (m, k):
        raise ValueError("A must be m x k")
    if B is not None and tuple(B.shape) != (k, n):
        raise ValueError("B must be k x n")
    _check(load().hpvm_sgemm_cpu(m, n, k, float(alpha), ctypes.c_void_p(pa), lda, ctypes.c_void_p(pb), ldb,
                                 float(beta), ctypes.c_void_p(pc), ldc, _tile(tile), int(threads)))
    return C


# ---------------------------------------------------------------------------
# Streaming graph: launch with Stream = 1, push, pop
# ---------------------------------------------------------------------------
_open_streams = set()


def _close_open_streams():
    for st in list(_open_streams):
        try:
            st.close()
        except HpvmError:
            pass


atexit.register(_close_open_streams)


class SgemmStream:
    """A streaming sgemm graph: a resident kernel that runs every pushed sgemm.

    push() hands it C <- alpha A B + beta C (FP32, in place) and returns the
    item's sequence number; pop() returns (seq, C) of the oldest item once it
    is complete.  Items in flight run concurrently and must be independent.
    The tensors of an item are kept alive until it is popped.  While the
    stream is open, synchronize streams (torch.cuda.current_stream()
    .synchronize()), not the device: torch.cuda.synchronize() waits for the
    resident kernel until the stream is closed or reaches its idle limit.
    """

    def __init__(self, capacity: int = 64, grid: int = 0, idle_ms: int = 2000):
        cfg = _lib.StreamConfig(int(capacity), int(grid), int(idle_ms), 0)
        h = ctypes.c_void_p()
        _check(load().hpvm_stream_open(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._items = {}
        self._seq = ctypes.c_int64(-1)
        lib = load()
        self._push, self._pop = lib.hpvm_stream_push, lib.hpvm_stream_pop
        _open_streams.add(self)

    @staticmethod
    def pack(A, B, C, alpha: float = 1.0, beta: float = 0.0, k: int | None = None):
        """The packed argument struct of one item (validated once; reusable).

        A or B may be None when alpha == 0 or k == 0 (pass k then).  Returns
        (desc, tensors) for push_packed.
        """
        m, n = C.shape
        if A is not None:
            k = A.shape[1]
        elif k is None:
            raise ValueError("k is needed when A is None")
        pa, lda = _mat(A, "A") if A is not None else (ctypes.c_void_p(0), max(k, 1))
        pb, ldb = _mat(B, "B") if B is not None else (ctypes.c_void_p(0), max(n, 1))
        pc, ldc = _mat(C, "C")
        if A is not None and tuple(A.shape) != (m, k):
            raise ValueError("A must be m x k")
        if B is not None and tuple(B.shape) != (k, n):
            raise ValueError("B must be k x n")
        d = _lib.SgemmDesc(m, n, k, float(alpha), float(beta), pa.value, lda, pb.value, ldb, pc.value, ldc)
        return d, (A, B, C)

    def push_packed(self, packed) -> int:
        """llvm.hpvm.push of a struct from pack(); returns the sequence number."""
        desc, tensors = packed
        rc = self._push(self._h, ctypes.byref(desc), ctypes.byref(self._seq))
        if rc != 0:
            raise HpvmError(rc, last_error())
        self._items[self._seq.value] = tensors
        return self._seq.value

    def push(self, A, B, C, alpha: float = 1.0, beta: float = 0.0, k: int | None = None) -> int:
        """Packs and pushes one item: C <- alpha A B + beta C."""
        return self.push_packed(self.pack(A, B, C, alpha, beta, k))

    @property
    def in_flight(self) -> int:
        """Items pushed and not yet popped."""
        return len(self._items)

    def pop(self, timeout_ms: int = 10000):
        """llvm.hpvm.pop: (seq, C) of the oldest item, once it is complete."""
        rc = self._pop(self._h, int(timeout_ms), ctypes.byref(self._seq), None)
        if rc != 0:
            raise HpvmError(rc, last_error())
        _, _, C = self._items.pop(self._seq.value)
        return self._seq.value, C

    def info(self) -> dict:
        st = _lib.StreamStatus()
        _check(load().hpvm_stream_info(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in _lib.StreamStatus._fields_ if f != "reserved"}

    def close(self, timeout_ms: int = 30000):
        if self._h is not None:
            _check(load().hpvm_stream_close(self._h, int(timeout_ms)))
            self._h = None
            self._items.clear()
            _open_streams.discard(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

