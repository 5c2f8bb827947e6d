"""FP64 CPU oracle for the hierarchical-dataflow sgemm -- TEST INFRASTRUCTURE.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU product path never imports it; the two share no
code.  The arithmetic lives in ``sgemm_oracle.c`` (plain C, FP64); this module
only marshals numpy arrays into it.

Functions (each follows the definition stated in ``sgemm_oracle.c``):

* ``sgemm``          -- C_out = alpha * A @ B + beta * C, FP64, row-major.
* ``sgemm_entries``  -- selected elements of the same definition.
* ``sgemm_grad``     -- closed-form gradient of <G, C_out>.
* ``grad_entries``   -- selected elements of dA or dB.
* ``bf16_round`` / ``bf16_split`` -- the oracle's own RNE bfloat16 rounder.
* ``consumer``       -- a one-to-one element-wise node after the sgemm node
  (the dependent pair that node fusion merges): relu, bias, bias+relu, clamp.
* ``sgemm_consumed`` -- consumer(sgemm(...)): what the fused node computes.

Mode names: ``"fp32"`` (inputs as given), ``"bf16"`` (A, B rounded to
bfloat16 first), ``"bf16x3"`` (hi*hi + hi*lo + lo*hi of the bfloat16 split).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_MODES = {"fp32": 0, "bf16": 1, "bf16x3": 2}
_lib = None

_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_ptr = ctypes.c_void_p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # HPVM_ORACLE_LIB names another build of the oracle (the tests'
    # sanitizer build); otherwise the default one, rebuilt when stale.
    path = os.environ.get("HPVM_ORACLE_LIB")
    if not path:
        src_m = os.path.getmtime(_build.SRC)
        if not os.path.exists(_build.LIB) or os.path.getmtime(_build.LIB) < src_m:
            _build.build()
        path = _build.LIB
    lib = ctypes.CDLL(path)
    lib.oracle_bf16_round.restype = ctypes.c_float
    lib.oracle_bf16_round.argtypes = [ctypes.c_float]
    lib.oracle_bf16_round_array.argtypes = [_ptr, _ptr, _i64]
    lib.oracle_bf16_split_array.argtypes = [_ptr, _ptr, _ptr, _i64]
    lib.oracle_sgemm.restype = ctypes.c_int
    lib.oracle_sgemm.argtypes = [_i64, _i64, _i64, _dbl, _ptr, _i64, _ptr, _i64,
                                 _dbl, _ptr, _i64, _ptr, _i64, ctypes.c_int,
                                 ctypes.c_int]
    lib.oracle_sgemm_entries.restype = ctypes.c_int
    lib.oracle_sgemm_entries.argtypes = [_i64, _i64, _i64, _dbl, _ptr, _i64, _ptr,
                                         _i64, _dbl, _ptr, _i64, _i64, _ptr, _ptr,
                                         _ptr, ctypes.c_int]
    lib.oracle_sgemm_grad.restype = ctypes.c_int
    lib.oracle_sgemm_grad.argtypes = [_i64, _i64, _i64, _dbl, _dbl, _ptr, _i64,
                                      _ptr, _i64, _ptr, _i64, _ptr, _i64, _ptr,
                                      _ptr, _ptr, _ptr, _ptr, ctypes.c_int]
    lib.oracle_grad_entries.restype = ctypes.c_int
    lib.oracle_grad_entries.argtypes = [ctypes.c_int, _i64, _i64, _i64, _dbl, _ptr,
                                        _i64, _ptr, _i64, _ptr, _i64, _i64, _ptr,
                                        _ptr, _ptr]
    lib.oracle_consumer.restype = ctypes.c_int
    lib.oracle_consumer.argtypes = [_i64, _i64, _ptr, ctypes.c_int, _ptr, _dbl, _dbl, _ptr]
    _lib = lib
    return lib


def _f32_2d(x, name):
    x = np.asarray(x)
    if x.dtype != np.float32 or x.ndim != 2:
        raise TypeError(f"{name} must be a 2-D float32 array")
    if x.size == 0:
        return x, max(x.shape[1], 1)
    if x.strides[1] != 4 or (x.shape[0] > 1 and x.strides[0] % 4):
        raise ValueError(f"{name} must be row-major with unit column stride")
    return x, (x.strides[0] // 4 if x.shape[0] > 1 else max(x.shape[1], 1))


def _p(x):
    return x.ctypes.data_as(_ptr) if x is not None else None


def default_threads():
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()


def sgemm(A, B, C, alpha, beta, mode="fp32", threads=None):
    """FP64 result of alpha * A @ B + beta * C for float32 A (m x k), B (k x n), C (m x n).

    ``C`` may be None when ``beta == 0`` (it is then never read).
    """
    lib = _load()
    A, lda = _f32_2d(A, "A")
    B, ldb = _f32_2d(B, "B")
    m, k = A.shape
    k2, n = B.shape
    if k2 != k:
        raise ValueError("inner dimensions differ")
    if C is not None:
        C, ldc = _f32_2d(C, "C")
        if C.shape != (m, n):
            raise ValueError("C shape mismatch")
    else:
        if beta != 0:
            raise ValueError("C is needed when beta != 0")
        ldc = max(n, 1)
    out = np.empty((m, n), dtype=np.float64)
    rc = lib.oracle_sgemm(m, n, k, float(alpha), _p(A), lda, _p(B), ldb, float(beta),
                          _p(C), ldc, _p(out), max(n, 1), _MODES[mode],
                          int(threads or default_threads()))
    if rc != 0:
        raise RuntimeError("oracle_sgemm rejected its arguments")
    return out


def sgemm_entries(A, B, C, alpha, beta, rows, cols, mode="fp32"):
    """FP64 elements (rows[t], cols[t]) of alpha * A @ B + beta * C."""
    lib = _load()
    A, lda = _f32_2d(A, "A")
    B, ldb = _f32_2d(B, "B")
    m, k = A.shape
    n = B.shape[1]
    if C is not None:
        C, ldc = _f32_2d(C, "C")
    else:
        if beta != 0:
            raise ValueError("C is needed when beta != 0")
        ldc = max(n, 1)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.empty(rows.shape[0], dtype=np.float64)
    rc = lib.oracle_sgemm_entries(m, n, k, float(alpha), _p(A), lda, _p(B), ldb,
                                  float(beta), _p(C), ldc, rows.shape[0], _p(rows),
                                  _p(cols), _p(out), _MODES[mode])
    if rc != 0:
        raise RuntimeError("oracle_sgemm_entries rejected its arguments")
    return out


def sgemm_grad(A, B, C_in, G, alpha, beta, threads=None):
    """Closed-form FP64 gradient of <G, alpha*A@B + beta*C_in>.

    Returns dict with dA, dB, dC_in (float64 arrays) and dalpha, dbeta (floats).
    """
    lib = _load()
    A, lda = _f32_2d(A, "A")
    B, ldb = _f32_2d(B, "B")
    C_in, ldci = _f32_2d(C_in, "C_in")
    G, ldg = _f32_2d(G, "G")
    m, k = A.shape
    n = B.shape[1]
    dA = np.empty((m, k), dtype=np.float64)
    dB = np.empty((k, n), dtype=np.float64)
    dC = np.empty((m, n), dtype=np.float64)
    da = _dbl(0.0)
    db = _dbl(0.0)
    rc = lib.oracle_sgemm_grad(m, n, k, float(alpha), float(beta), _p(A), lda, _p(B),
                               ldb, _p(C_in), ldci, _p(G), ldg, _p(dA), _p(dB), _p(dC),
                               ctypes.byref(da), ctypes.byref(db),
                               int(threads or default_threads()))
    if rc != 0:
        raise RuntimeError("oracle_sgemm_grad rejected its arguments")
    return {"dA": dA, "dB": dB, "dC_in": dC, "dalpha": da.value, "dbeta": db.value}


def grad_entries(which, A, B, G, alpha, rows, cols):
    """Selected FP64 entries of dA (which='dA') or dB (which='dB')."""
    lib = _load()
    A, lda = _f32_2d(A, "A")
    B, ldb = _f32_2d(B, "B")
    G, ldg = _f32_2d(G, "G")
    m, k = A.shape
    n = B.shape[1]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.empty(rows.shape[0], dtype=np.float64)
    rc = lib.oracle_grad_entries({"dA": 0, "dB": 1}[which], m, n, k, float(alpha),
                                 _p(A), lda, _p(B), ldb, _p(G), ldg, rows.shape[0],
                                 _p(rows), _p(cols), _p(out))
    if rc != 0:
        raise RuntimeError("oracle_grad_entries rejected its arguments")
    return out


def bf16_round(x):
    """The oracle's RNE rounding of float32 values to bfloat16 (returned as float32)."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty_like(x)
    lib.oracle_bf16_round_array(_p(x), _p(y), x.size)
    return y


def bf16_split(x):
    """(hi, lo) with hi = bf16(x), lo = bf16(x - hi), both float32 arrays."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float32)
    hi = np.empty_like(x)
    lo = np.empty_like(x)
    lib.oracle_bf16_split_array(_p(x), _p(hi), _p(lo), x.size)
    return hi, lo


CONSUMER_OPS = {"none": 0, "relu": 1, "bias": 2, "bias_relu": 3, "clamp": 4}


def consumer(X, op, bias=None, lo=-np.inf, hi=np.inf):
    """The consumer node's function applied to an m x n FP64 array (FP64 out).

    ``bias`` (one float32 per column) is used by "bias" and "bias_relu";
    ``lo`` and ``hi`` by "clamp".
    """
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    m, n = X.shape
    code = CONSUMER_OPS[op] if isinstance(op, str) else int(op)
    b = np.ascontiguousarray(bias if bias is not None else np.zeros(n), dtype=np.float32)
    if b.shape != (n,):
        raise ValueError("bias must hold one value per column")
    D = np.empty_like(X)
    if X.size == 0:
        return D
    rc = lib.oracle_consumer(m, n, _p(X), code, _p(b), float(lo), float(hi), _p(D))
    if rc != 0:
        raise ValueError(f"unknown consumer op {op!r}")
    return D


def sgemm_consumed(A, B, C, alpha, beta, op, bias=None, lo=-np.inf, hi=np.inf):
    """consumer(alpha A B + beta C): the dependent pair, evaluated one node after the other."""
    return consumer(sgemm(A, B, C, alpha, beta), op, bias, lo, hi)

