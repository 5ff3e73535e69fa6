"""Helpers shared by the GPU parity tests (marshalling and error measures)."""
import numpy as np
import torch

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def logical(X, rows, cols):
    return np.asarray(X)[:cols, :rows, :].transpose(1, 0, 2)


def relfro(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    den = np.linalg.norm(want)
    return np.linalg.norm(got - want) / (den if den > 0 else 1.0)


def norm1(X):
    """Per-element 1-norm of a logical (r, c, 4) quaternion matrix."""
    return np.abs(np.asarray(X, dtype=np.float64)).sum(-1)


def op_logical(op, X, rows, cols):
    """Logical op(X) from a stored operand, magnitudes only matter here."""
    if op in ("N", "R"):
        return logical(X, rows, cols)
    return logical(X, cols, rows).transpose(1, 0, 2)


def error_bound(p, u=U64, extra=8):
    """Componentwise rounding bound (4K + extra) u (|alpha|_1 S + |beta|_1 |C|_1)
    with S = sum_k |op(A)_{mu k}|_1 |op(B)_{k nu}|_1, an upper bound of the
    absolute values feeding each real output."""
    M, N, K = p["M"], p["N"], p["K"]
    a1 = norm1(op_logical(p["opA"], p["A"], M, K)) if K else np.zeros((M, 0))
    b1 = norm1(op_logical(p["opB"], p["B"], K, N)) if K else np.zeros((0, N))
    S = a1 @ b1
    c1 = norm1(logical(p["C"], M, N))
    beta = np.abs(np.asarray(p["beta"])).sum()
    cterm = beta * np.nan_to_num(c1) if beta != 0 else 0.0
    return (4 * K + extra) * u * (np.abs(np.asarray(p["alpha"])).sum() * S + cterm)
