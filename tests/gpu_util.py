"""Helpers shared by the GPU tests: device copies and error measures."""
import numpy as np

U32 = 2.0 ** -24


def to_dev(x, pad=0, misalign=False):
    """float32 numpy matrix -> CUDA tensor view with leading dimension cols + pad.

    ``misalign`` shifts the data by one float so 16-byte vector loads are off.
    """
    import torch

    r, c = x.shape
    ld = c + pad
    off = 1 if misalign else 0
    flat = torch.full((r * ld + off + 4,), float("nan"), dtype=torch.float32)
    view = flat[off:off + r * ld].view(r, ld)
    view[:, :c] = torch.from_numpy(np.ascontiguousarray(x))
    flat = flat.cuda()
    return flat[off:off + r * ld].view(r, ld)[:, :c]


def to_host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def normwise(got, ref):
    """||got - ref||_F / ||ref||_F in float64."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (den if den else 1.0))


def componentwise_bound(A, B, C, alpha, beta, k, extra=0.0):
    """Order-independent FP32 bound: gamma_k |alpha| |A||B| + 2u |beta C| (+ extra |A||B|)."""
    ab = np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64))
    g = (k + 2) * U32 / (1 - (k + 2) * U32)
    b = (2 * g + extra) * abs(alpha) * ab
    if beta != 0:
        b = b + 4 * U32 * abs(beta) * np.abs(C.astype(np.float64))
    return b + 1e-30
