"""torch.autograd binding of the quaternion GEMM and a quaternion linear layer.

Tensors use the library's storage layout: a rows x cols quaternion matrix is a
contiguous tensor of shape (cols, rows, 4) (column-major, leading dimension =
rows, four interleaved components).  float64 tensors run the FP64 path,
float32 tensors the split-BF16 path.  The gradient is the hand-written one of
the C ABI (qgemm_backward_d / qgemm_backward_s); alpha and beta are constants.
"""
import math

import torch

from . import _lib


def _dims(op, t):
    """(rows, cols) of op(X) for a stored tensor t of shape (cols, rows, 4)."""
    cols, rows = t.shape[0], t.shape[1]
    return (rows, cols) if op in ("N", "R") else (cols, rows)


def _gemm(opA, opB, M, N, K, alpha, A, B, beta, C, split_terms):
    if A.dtype == torch.float64:
        _lib.qgemm_d(opA, opB, M, N, K, alpha, A, A.shape[1], B, B.shape[1], beta, C, C.shape[1])
    else:
        _lib.qgemm_s(opA, opB, M, N, K, alpha, A, A.shape[1], B, B.shape[1], beta, C, C.shape[1],
                     split_terms=split_terms)


class QGemmFn(torch.autograd.Function):
    """C = alpha op(A) op(B) + beta C0 (C0 optional)."""

    @staticmethod
    def forward(ctx, A, B, C0=None, alpha=(1.0, 0.0, 0.0, 0.0), beta=(0.0, 0.0, 0.0, 0.0),
                opA="N", opB="N", split_terms=6):
        A = A.contiguous()
        B = B.contiguous()
        M, K = _dims(opA, A)
        K2, N = _dims(opB, B)
        if K != K2:
            raise ValueError(f"inner dimensions differ: op(A) is {M}x{K}, op(B) is {K2}x{N}")
        if C0 is not None:
            C = C0.detach().clone().contiguous()
            if tuple(C.shape) != (N, M, 4):
                raise ValueError(f"C0 must have shape {(N, M, 4)}")
        else:
            C = torch.empty((N, max(M, 1), 4), dtype=A.dtype, device=A.device)
            beta = (0.0, 0.0, 0.0, 0.0)
        _gemm(opA, opB, M, N, K, alpha, A, B, beta, C, split_terms)
        ctx.save_for_backward(A, B)
        ctx.cfg = (opA, opB, M, N, K, tuple(alpha), tuple(beta), split_terms, C0 is not None)
        return C

    @staticmethod
    def backward(ctx, G):
        A, B = ctx.saved_tensors
        opA, opB, M, N, K, alpha, beta, split_terms, has_c0 = ctx.cfg
        G = G.contiguous()
        dA = torch.empty_like(A) if ctx.needs_input_grad[0] else None
        dB = torch.empty_like(B) if ctx.needs_input_grad[1] else None
        dC0 = torch.empty_like(G) if (has_c0 and ctx.needs_input_grad[2]) else None
        _lib.qgemm_backward(opA, opB, M, N, K, alpha, A, A.shape[1], B, B.shape[1], G, G.shape[1], beta,
                            dA, A.shape[1], dB, B.shape[1], dC0, G.shape[1], split_terms=split_terms)
        return dA, dB, dC0, None, None, None, None, None


def qgemm(A, B, C0=None, alpha=(1.0, 0.0, 0.0, 0.0), beta=(0.0, 0.0, 0.0, 0.0), opA="N", opB="N",
          split_terms=6):
    return QGemmFn.apply(A, B, C0, alpha, beta, opA, opB, split_terms)


class QLinear(torch.nn.Module):
    """Y = X W with X (rows x fan_in) and W (fan_in x fan_out) quaternion
    matrices.  W is Glorot-initialised with sigma^2 = 2 / (4 fan_in + 4 fan_out)
    per component (the fans of the real 4x4 embedding)."""

    def __init__(self, fan_in, fan_out, dtype=torch.float32, device="cuda", split_terms=6):
        super().__init__()
        sigma = math.sqrt(2.0 / (4 * fan_in + 4 * fan_out))
        w = torch.randn((fan_out, fan_in, 4), dtype=dtype, device=device) * sigma
        self.weight = torch.nn.Parameter(w)
        self.split_terms = split_terms

    def forward(self, X):
        return QGemmFn.apply(X, self.weight, None, (1.0, 0.0, 0.0, 0.0), (0.0, 0.0, 0.0, 0.0), "N", "N",
                             self.split_terms)
