"""torch.autograd.Function over the sgemm node: forward and hand-written backward.

``SgemmFn.apply(A, B, C_in, alpha, beta, prec)`` returns
C_out = alpha * A @ B + beta * C_in (out of place: C_in is not modified).
alpha and beta are Python floats or 0-dim tensors; gradients flow to every
tensor argument that requires them.  Both passes run in the library's HIP
kernels (hpvm_sgemm, hpvm_sgemm_backward); nothing falls back to torch math.
"""
from __future__ import annotations

import torch

from . import sgemm, sgemm_backward


def _scalar(x) -> float:
    return float(x.detach().item()) if isinstance(x, torch.Tensor) else float(x)


class SgemmFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, C_in, alpha, beta, prec="fp32"):
        a, b = _scalar(alpha), _scalar(beta)
        out = C_in.detach().clone() if b != 0.0 else torch.empty_like(C_in)
        sgemm(A.detach(), B.detach(), out, a, b, prec=prec)
        ctx.save_for_backward(A, B, C_in)
        ctx.alpha, ctx.beta, ctx.prec = a, b, prec
        ctx.alpha_is_tensor = isinstance(alpha, torch.Tensor)
        ctx.beta_is_tensor = isinstance(beta, torch.Tensor)
        return out

    @staticmethod
    def backward(ctx, G):
        A, B, C_in = ctx.saved_tensors
        need = []
        if ctx.needs_input_grad[0]:
            need.append("dA")
        if ctx.needs_input_grad[1]:
            need.append("dB")
        if ctx.needs_input_grad[2]:
            need.append("dC_in")
        if ctx.alpha_is_tensor and ctx.needs_input_grad[3]:
            need.append("dalpha")
        if ctx.beta_is_tensor and ctx.needs_input_grad[4]:
            need.append("dbeta")
        g = sgemm_backward(A.detach(), B.detach(), C_in.detach(), G.contiguous(), ctx.alpha, ctx.beta,
                           prec=ctx.prec, need=tuple(need))
        return g.get("dA"), g.get("dB"), g.get("dC_in"), g.get("dalpha"), g.get("dbeta"), None


def sgemm_fn(A, B, C_in, alpha=1.0, beta=0.0, prec="fp32"):
    """Differentiable C_out = alpha * A @ B + beta * C_in."""
    return SgemmFn.apply(A, B, C_in, alpha, beta, prec)
