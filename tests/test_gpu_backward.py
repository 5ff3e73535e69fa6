"""GPU checks of the hand-written gradient (C-ABI qgemm_backward_d/_s and the
torch.autograd binding) against the oracle's gradient, central finite
differences, and torch autograd through the real 4x4 embedding.

Parity bars: relative Frobenius 1e-13 (FP64) / 1e-6 (FP32 split) over each
gradient and each of its 32 x 32 blocks, and every real within the
componentwise bounds of tests/gpu_util.grad_bounds."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_1903_05575_amd as q
from tests.gpu_util import (assert_parity, bound_f64, bound_split, dev, error_bound, grad_bounds, host, logical,
                            norm1, relfro, split_pipeline)

pytestmark = pytest.mark.gpu


def run_backward(p, G, dtype, terms=6):
    A, B, Gd = dev(p["A"], dtype), dev(p["B"], dtype), dev(G, dtype)
    dA = torch.full_like(A, float("nan"))
    dB = torch.full_like(B, float("nan"))
    dC0 = torch.full_like(Gd, float("nan"))
    q.qgemm_backward(p["opA"], p["opB"], p["M"], p["N"], p["K"], p["alpha"], A, p["lda"], B, p["ldb"],
                     Gd, p["M"], p["beta"], dA, p["lda"], dB, p["ldb"], dC0, p["M"], split_terms=terms)
    return host(dA), host(dB), host(dC0)


def stored_rows(op, r, c):
    return r if op in "NR" else c


def check_grads(p, G, got, want, f64, terms=6, label=""):
    """got, want: (dA, dB, dC0) in stored layout; any pair may be None."""
    M, N, K = p["M"], p["N"], p["K"]
    ra, ca = (M, K) if p["opA"] in "NR" else (K, M)
    rb, cb = (K, N) if p["opB"] in "NR" else (N, K)
    bars = 1e-13 if f64 else 1e-6
    bounds = grad_bounds(p, G, f64, terms)
    for name, g, o, (r, c), b in zip(("dA", "dB", "dC0"), got, want, ((ra, ca), (rb, cb), (M, N)), bounds):
        if g is None or o is None:
            continue
        assert_parity(logical(g, r, c), logical(o, r, c), b, bars, label=f"{label} {name}")


def widen32(x):
    return np.asarray(x).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("opA", "NTCR")
@pytest.mark.parametrize("opB", "NTCR")
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_backward_all_ops(gpu, opA, opB, dtype):
    M, N, K = 70, 45, 53
    p = W.gemm_problem(3000 + "NTCR".index(opA) * 4 + "NTCR".index(opB), M, N, K, opA, opB, dist="normal")
    G = W.qmatrix(W.rng(77), M, N)
    if dtype == "f32":
        for k in ("A", "B", "C"):
            p[k] = widen32(p[k])
        G = widen32(G)
    oA, oB, oC = oracle.qgemm_backward(opA, opB, M, N, K, p["alpha"], p["A"], p["lda"], p["B"], p["ldb"],
                                       G, M, p["beta"])
    tdt = torch.float64 if dtype == "f64" else torch.float32
    check_grads(p, G, run_backward(p, G, tdt), (oA, oB, oC), dtype == "f64", label=f"backward {dtype} {opA}{opB}")


@pytest.mark.parametrize("opA", "NTCR")
@pytest.mark.parametrize("opB", "NT")
def test_backward_s_tl2_dA(gpu, opA, opB):
    """FP32 gradient whose dA product (2047 x 1000 outputs, contraction over
    N = 96) runs on the TL2 pipeline: G is its A operand (op N), op(B)^H its B
    operand; the store maps d op(A) back through op(A)."""
    M, N, K = 2047, 96, 1000
    assert split_pipeline(M, K) == "TL2"
    p = W.gemm_problem(3100 + "NTCR".index(opA) * 4 + "NT".index(opB), M, N, K, opA, opB, dist="normal")
    for k in ("A", "B", "C"):
        p[k] = widen32(p[k])
    G = widen32(W.qmatrix(W.rng(78), M, N))
    oA, _, _ = oracle.qgemm_backward(opA, opB, M, N, K, p["alpha"], p["A"], p["lda"], p["B"], p["ldb"], G, M,
                                     p["beta"], want_dB=False, want_dC0=False)
    gA, _, _ = run_backward(p, G, torch.float32)
    check_grads(p, G, (gA, None, None), (oA, None, None), False, label=f"TL2 dA {opA}{opB}")


@pytest.mark.parametrize("opA", "NTCR")
@pytest.mark.parametrize("opB", "NC")
def test_backward_s_tl2_dB(gpu, opA, opB):
    """FP32 gradient whose dB product (1000 x 2047 outputs, contraction over
    M = 96) runs on the TL2 pipeline with op(A)^H as its A operand: a
    transposed A for op(A) in {N, R} (stored A read through op C / T), a
    plain one for {T, C}; conj(alpha) scales G as it is staged."""
    M, N, K = 96, 2047, 1000
    assert split_pipeline(K, N) == "TL2"
    p = W.gemm_problem(3200 + "NTCR".index(opA) * 4 + "NC".index(opB), M, N, K, opA, opB, dist="normal")
    for k in ("A", "B", "C"):
        p[k] = widen32(p[k])
    G = widen32(W.qmatrix(W.rng(79), M, N))
    _, oB, _ = oracle.qgemm_backward(opA, opB, M, N, K, p["alpha"], p["A"], p["lda"], p["B"], p["ldb"], G, M,
                                     p["beta"], want_dA=False, want_dC0=False)
    _, gB, _ = run_backward(p, G, torch.float32)
    check_grads(p, G, (None, gB, None), (None, oB, None), False, label=f"TL2 dB {opA}{opB}")


def _loss(X, Wt, G, fwd):
    Y = fwd(X, Wt)
    return float((Y * G).sum())


def test_finite_differences_16(gpu):
    """Linear layer slice 16x16x16: central differences with h = 1 of the GPU
    FP64 forward (exact for this bilinear loss) against the GPU gradient."""
    p = W.linear_layer(rows=16, fan_in=16, fan_out=16, dtype=np.float64)
    X, Wm, dY = p["X"], p["W"], p["dY"]
    one, zero = [1, 0, 0, 0], [0, 0, 0, 0]

    def fwd(Xn, Wn):
        Xd, Wd = dev(Xn), dev(Wn)
        Yd = torch.zeros((16, 16, 4), dtype=torch.float64, device="cuda")
        q.qgemm_d("N", "N", 16, 16, 16, one, Xd, 16, Wd, 16, zero, Yd, 16)
        return host(Yd)

    prob = dict(opA="N", opB="N", M=16, N=16, K=16, alpha=np.array(one, float), beta=np.zeros(4),
                A=X, lda=16, B=Wm, ldb=16)
    gX, gW, _ = run_backward(prob, dY, torch.float64)
    for name, T, gT in (("X", X, gX), ("W", Wm, gW)):
        fd = np.zeros_like(T)
        for idx in np.ndindex(T.shape):
            Tp, Tm = T.copy(), T.copy()
            Tp[idx] += 1.0
            Tm[idx] -= 1.0
            if name == "X":
                lp, lm = _loss(Tp, Wm, dY, fwd), _loss(Tm, Wm, dY, fwd)
            else:
                lp, lm = _loss(X, Tp, dY, fwd), _loss(X, Tm, dY, fwd)
            fd[idx] = (lp - lm) / 2.0
        assert np.abs(fd - gT).max() <= 1e-11 * max(1.0, np.abs(fd).max()), name


def test_finite_differences_16_fp32(gpu):
    """Same slice on the FP32 split path with h = 0.1, tolerance 1e-3 relative."""
    p = W.linear_layer(rows=16, fan_in=16, fan_out=16, dtype=np.float32)
    X, Wm, dY = p["X"], p["W"], p["dY"]
    one, zero = [1, 0, 0, 0], [0, 0, 0, 0]
    h = 0.1

    def fwd(Xn, Wn):
        Xd, Wd = dev(Xn.astype(np.float32)), dev(Wn.astype(np.float32))
        Yd = torch.zeros((16, 16, 4), dtype=torch.float32, device="cuda")
        q.qgemm_s("N", "N", 16, 16, 16, one, Xd, 16, Wd, 16, zero, Yd, 16)
        return host(Yd).astype(np.float64)

    prob = dict(opA="N", opB="N", M=16, N=16, K=16, alpha=np.array(one, float), beta=np.zeros(4),
                A=X, lda=16, B=Wm, ldb=16)
    gX, gW, _ = run_backward(prob, dY, torch.float32)
    for name, T, gT in (("X", X, gX), ("W", Wm, gW)):
        fd = np.zeros(T.shape)
        for idx in list(np.ndindex(T.shape))[::7]:
            Tp, Tm = T.astype(np.float64), T.astype(np.float64)
            Tp = Tp.copy(); Tm = Tm.copy()
            Tp[idx] += h
            Tm[idx] -= h
            args = (Tp, Wm) if name == "X" else (X, Tp)
            argm = (Tm, Wm) if name == "X" else (X, Tm)
            fd[idx] = (_loss(*args, dY.astype(np.float64), fwd) - _loss(*argm, dY.astype(np.float64), fwd)) / (2 * h)
            assert abs(fd[idx] - gT[idx]) <= 1e-3 * max(1.0, abs(fd[idx])), (name, idx, fd[idx], gT[idx])


def real_embedding_grad(X, Wm, dY):
    """Reference gradient: torch autograd (CPU, fp64) of <dY, Y> with
    Y_real (4M x N) = L(X) (4M x 4K) W_real (4K x N), where L(X) is built from
    X by index selection and signs only (row r, column c of the block of x is
    sign(r, c) x[r ^ c], the left-multiplication matrix of Eq. quaternion_prod)."""
    M, K = X.shape[1], X.shape[0]
    N = Wm.shape[0]
    sign = torch.tensor([[1, -1, -1, -1], [1, 1, -1, 1], [1, 1, 1, -1], [1, -1, 1, 1]], dtype=torch.float64)
    perm = torch.tensor([[r ^ c for c in range(4)] for r in range(4)])
    x = torch.tensor(X[:, :M].transpose(1, 0, 2).copy(), requires_grad=True)       # (M, K, 4)
    w = torch.tensor(Wm[:, :K].transpose(1, 0, 2).copy(), requires_grad=True)      # (K, N, 4)
    blocks = x[:, :, perm] * sign                                                  # (M, K, 4, 4) [mu, k, r, c]
    Lx = blocks.permute(0, 2, 1, 3).reshape(4 * M, 4 * K)
    wr = w.permute(0, 2, 1).reshape(4 * K, N)
    Y = (Lx @ wr).reshape(M, 4, N).permute(0, 2, 1)                                # (M, N, 4)
    g = torch.tensor(dY[:, :M].transpose(1, 0, 2).copy())
    (Y * g).sum().backward()
    return x.grad.numpy().transpose(1, 0, 2), w.grad.numpy().transpose(1, 0, 2)


def test_real_embedding_gradient(gpu):
    p = W.linear_layer(rows=48, fan_in=40, fan_out=24, dtype=np.float64)
    X, Wm, dY = p["X"], p["W"], p["dY"]
    ref_x, ref_w = real_embedding_grad(X, Wm, dY)
    prob = dict(opA="N", opB="N", M=48, N=24, K=40, alpha=np.array([1.0, 0, 0, 0]), beta=np.zeros(4),
                A=X, lda=48, B=Wm, ldb=40)
    gX, gW, _ = run_backward(prob, dY, torch.float64)
    # the reference's own FP64 rounding is bounded like the library's: twice the bound
    bX, bW, _ = grad_bounds(prob, dY, True)
    assert_parity(logical(gX, 48, 40), logical(ref_x, 48, 40), 2 * bX, 1e-13, label="real-embedding dX")
    assert_parity(logical(gW, 40, 24), logical(ref_w, 40, 24), 2 * bW, 1e-13, label="real-embedding dW")


def test_autograd_function(gpu):
    """QGemmFn through torch.autograd with C0 and quaternion alpha/beta."""
    M, N, K = 33, 29, 41
    p = W.gemm_problem(9, M, N, K, "C", "T", dist="normal")
    G = W.qmatrix(W.rng(10), M, N)
    A = dev(p["A"]).requires_grad_(True)
    B = dev(p["B"]).requires_grad_(True)
    C0 = dev(p["C"]).requires_grad_(True)
    C = q.qgemm(A, B, C0, alpha=tuple(p["alpha"]), beta=tuple(p["beta"]), opA="C", opB="T")
    want = oracle.qgemm("C", "T", M, N, K, p["alpha"], p["A"], p["lda"], p["B"], p["ldb"], p["beta"], p["C"], p["ldc"])
    assert_parity(logical(host(C), M, N), logical(want, M, N), error_bound(p), 1e-13, label="QGemmFn forward")
    (C * dev(G)).sum().backward()
    oA, oB, oC = oracle.qgemm_backward("C", "T", M, N, K, p["alpha"], p["A"], p["lda"], p["B"], p["ldb"],
                                       G, M, p["beta"])
    check_grads(p, G, (host(A.grad), host(B.grad), host(C0.grad)), (oA, oB, oC), True, label="QGemmFn")


@pytest.mark.slow
def test_linear_layer_full_sampled(gpu):
    """X 8192 x 1024, W 1024 x 1024 (FP32, Glorot), dY N(0,1): forward and
    backward on the GPU; error against the oracle on sampled rows of Y and dX
    and sampled columns of dW."""
    p = W.linear_layer()
    M, K, N = p["M"], p["K"], p["N"]
    X = dev(p["X"]).requires_grad_(True)
    layer = q.QLinear(K, N)
    with torch.no_grad():
        layer.weight.copy_(dev(p["W"]))
    Y = layer(X)
    Y.backward(dev(p["dY"]))
    Yh, dXh, dWh = host(Y), host(X.grad), host(layer.weight.grad)
    g = np.random.default_rng(5)
    rows = np.sort(g.choice(M, 64, replace=False))
    cols = np.sort(g.choice(N, 16, replace=False))
    one, zero = np.array([1.0, 0, 0, 0]), np.zeros(4)
    Xs = p["X"][:, rows, :].astype(np.float64)                                   # rows of X (stored K x 64)
    Ys = oracle.qgemm("N", "N", 64, N, K, one, Xs, 64, p["W"].astype(np.float64), K, zero,
                      np.zeros((N, 64, 4)), 64)
    dYs = p["dY"][:, rows, :].astype(np.float64)
    dXs, _, _ = oracle.qgemm_backward("N", "N", 64, N, K, one, Xs, 64, p["W"].astype(np.float64), K,
                                      dYs, 64, zero, want_dB=False, want_dC0=False)
    dYc = p["dY"][cols].astype(np.float64)                                       # columns of dY (N' = 16)
    Wc = p["W"][cols].astype(np.float64)
    _, dWc, _ = oracle.qgemm_backward("N", "N", M, 16, K, one, p["X"].astype(np.float64), M, Wc, K,
                                      dYc, M, zero, want_dA=False, want_dC0=False)
    x1 = norm1(logical(p["X"], M, K))
    w1 = norm1(logical(p["W"], K, N))
    dy1 = norm1(logical(p["dY"], M, N))
    assert_parity(logical(Yh[:, rows], 64, N), logical(Ys, 64, N), bound_split(x1[rows] @ w1, K, 6, 1.0), 1e-6,
                  label="linear Y rows")
    assert_parity(logical(dXh[:, rows], 64, K), logical(dXs, 64, K), bound_split(dy1[rows] @ w1.T, N, 6, 1.0),
                  1e-6, label="linear dX rows")
    assert_parity(logical(dWh[cols], K, 16), logical(dWc, K, 16), bound_split(x1.T @ dy1[:, cols], M, 6, 1.0),
                  1e-6, label="linear dW columns")
