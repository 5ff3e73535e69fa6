"""GPU checks of the level-1/2 operations (C-ABI qaxpy_*, qdot_*, qgemv_*)
against the oracle: strided vectors whose gaps hold NaN (never read or
written), several blocks with ragged ends, the BLAS scalar rules and
run-to-run reproducibility of the reductions.  Bars: relative Frobenius 1e-13
(double storage) / 1e-6 (float storage), globally and over runs of 256
outputs, and every real within a componentwise bound: n u64 (plus a few
roundings of the scalar products) times the sum of the magnitudes feeding it,
plus one FP32 rounding of the result for float storage."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_1903_05575_amd as q
from tests.gpu_util import U32, U64, assert_parity, dev, gamma, host, logical, norm1, qnorm1, relfro

pytestmark = pytest.mark.gpu

NP = {"d": np.float64, "s": np.float32}
TOL = {"d": 1e-13, "s": 1e-6}


def vec_parity(got, want, mag, n_terms, p, label):
    """got, want: (n, 4) results; mag: (n,) sum of the magnitudes feeding
    each output (products and the scaled old value)."""
    bound = gamma(n_terms + 8, U64) * mag + (1.01 * U32 * mag if p == "s" else 0.0)
    assert_parity(np.asarray(got)[None], np.asarray(want)[None], np.asarray(bound)[None], TOL[p], block=256,
                  label=label)


def vnorm1(v, n, inc):
    return np.abs(np.asarray(v, dtype=np.float64)[::inc][:n]).sum(-1)


@pytest.mark.parametrize("p", "ds")
@pytest.mark.parametrize("incx,incy", [(1, 1), (3, 2)])
def test_qaxpy(gpu, p, incx, incy):
    g = W.rng(1300 + incx + 10 * (p == "s"))
    n = 100_003
    x, y = W.qvector(g, n, incx, dtype=NP[p]), W.qvector(g, n, incy, dtype=NP[p])
    al = W.quaternion(g)
    yd = dev(y)
    q.qaxpy(n, al, dev(x), incx, yd, incy)
    got = host(yd)
    want = oracle.qaxpy(n, al, x, incx, y, incy)
    mag = qnorm1(al) * vnorm1(x, n, incx) + vnorm1(y, n, incy)
    vec_parity(got[::incy][:n], want[::incy][:n], mag, 1, p, f"qaxpy_{p} inc {incx},{incy}")
    if incy > 1:
        assert np.isnan(got[1::incy]).all()


def test_qaxpy_rules(gpu):
    g = W.rng(1310)
    n = 1000
    x, y = W.qvector(g, n), W.qvector(g, n)
    yd = dev(y)
    q.qaxpy(n, [0.0] * 4, dev(np.full_like(x, np.nan)), 1, yd, 1)     # alpha = 0: untouched
    np.testing.assert_array_equal(host(yd), y)
    al = W.quaternion(g)
    q.qaxpy(n, al, yd, 1, yd, 1)                                       # x is y: y <- alpha y + y
    np.testing.assert_allclose(host(yd), oracle.qaxpy(n, al, y, 1, y, 1), rtol=0, atol=1e-15)


@pytest.mark.parametrize("p", "ds")
@pytest.mark.parametrize("conj", [False, True])
@pytest.mark.parametrize("n,incx,incy", [(1, 1, 1), (255, 2, 1), (100_003, 1, 3), (3_000_000, 1, 1)])
def test_qdot(gpu, p, conj, n, incx, incy):
    g = W.rng(1320 + n % 97 + conj + 2 * (p == "s"))
    x, y = W.qvector(g, n, incx, dtype=NP[p]), W.qvector(g, n, incy, dtype=NP[p])
    r = q.qdot(n, dev(x), incx, dev(y), incy, conj=conj)
    got = host(r).astype(np.float64)
    want = oracle.qdot(conj, n, x, incx, y, incy)
    # both sides sum in binary64 in different orders: bound by n u sum |x_i|_1 |y_i|_1
    mag = (np.abs(x[::incx][:n].astype(np.float64)).sum(1) * np.abs(y[::incy][:n].astype(np.float64)).sum(1)).sum()
    bound = n * 2.0 ** -53 * 4 * mag + (2.0 ** -24 * np.abs(want).max() if p == "s" else 0.0)
    assert np.abs(got - want).max() <= bound


def test_qdot_reproducible_and_empty(gpu):
    g = W.rng(1330)
    n = 1_000_003
    x, y = dev(W.qvector(g, n)), dev(W.qvector(g, n))
    work = torch.zeros(q._lib.DOT_WORK_DOUBLES, dtype=torch.float64, device="cuda")
    a = host(q.qdot(n, x, 1, y, 1, conj=True, work=work)).copy()
    b = host(q.qdot(n, x, 1, y, 1, conj=True, work=work)).copy()
    np.testing.assert_array_equal(a, b)
    r = dev(np.full(4, np.nan))
    q.qdot(0, None, 1, None, 1, result=r)
    np.testing.assert_array_equal(host(r), np.zeros(4))


def gemv_mag(trans, M, N, al, A, x, incx, be, y, incy):
    """|alpha|_1 sum_k |op(A)_{i k}|_1 |x_k|_1 + |beta|_1 |y_i|_1 per output."""
    a1 = norm1(logical(A, M, N))
    nx, ny = (M, N) if trans in "TC" else (N, M)
    x1, y1 = vnorm1(x, nx, incx), vnorm1(y, ny, incy)
    s = a1.T @ x1 if trans in "TC" else a1 @ x1
    return qnorm1(al) * s + (qnorm1(be) * np.nan_to_num(y1) if qnorm1(be) else 0.0)


@pytest.mark.parametrize("p", "ds")
@pytest.mark.parametrize("trans", "NTCR")
def test_qgemv(gpu, p, trans):
    g = W.rng(1340 + "NTCR".index(trans) + 4 * (p == "s"))
    M, N = 300, 217
    A = W.qmatrix(g, M, N, ld=M + 3, dtype=NP[p])
    nx, ny = (M, N) if trans in "TC" else (N, M)
    x, y = W.qvector(g, nx, 2, dtype=NP[p]), W.qvector(g, ny, 3, dtype=NP[p])
    al, be = W.quaternion(g), W.quaternion(g)
    yd = dev(y)
    q.qgemv(trans, M, N, al, dev(A), M + 3, dev(x), 2, be, yd, 3)
    got = host(yd)
    want = oracle.qgemv(trans, M, N, al, A, M + 3, x, 2, be, y, 3)
    vec_parity(got[::3][:ny], want[::3][:ny], gemv_mag(trans, M, N, al, A, x, 2, be, y, 3), nx, p,
               f"qgemv_{p} {trans}")
    assert np.isnan(got[1::3]).all()


@pytest.mark.parametrize("p", "ds")
@pytest.mark.parametrize("trans", "NTC")
def test_qgemv_edge_shapes(gpu, p, trans):
    """Shapes at the edges of the block layouts: op T/C splits the rows of a
    block over four waves in runs of 64 (fewer rows than one run leaves waves
    with nothing), op N takes 16 (FP64) or 8 (FP32) rows per block; output
    counts below, at and above the four outputs of an op T/C block."""
    for i, (M, N) in enumerate(((1, 1), (5, 3), (63, 4), (64, 5), (65, 8), (257, 9), (8, 1), (17, 2))):
        g = W.rng(1360 + 10 * i + "NTC".index(trans) + 5 * (p == "s"))
        A = W.qmatrix(g, M, N, ld=M + 1, dtype=NP[p])
        nx, ny = (M, N) if trans in "TC" else (N, M)
        x, y = W.qvector(g, nx, dtype=NP[p]), W.qvector(g, ny, dtype=NP[p])
        al, be = W.quaternion(g), W.quaternion(g)
        yd = dev(y)
        q.qgemv(trans, M, N, al, dev(A), M + 1, dev(x), 1, be, yd, 1)
        want = oracle.qgemv(trans, M, N, al, A, M + 1, x, 1, be, y, 1)
        vec_parity(host(yd), want, gemv_mag(trans, M, N, al, A, x, 1, be, y, 1), nx, p,
                   f"qgemv_{p} {trans} {M}x{N}")


@pytest.mark.parametrize("trans", "NC")
def test_qgemv_large_and_rules(gpu, trans):
    g = W.rng(1350 + (trans == "C"))
    M, N = 2051, 1999
    A = W.qmatrix(g, M, N)
    nx, ny = (M, N) if trans == "C" else (N, M)
    x, y = W.qvector(g, nx), W.qvector(g, ny)
    al, be = W.quaternion(g), W.quaternion(g)
    yd = dev(y)
    q.qgemv(trans, M, N, al, dev(A), M, dev(x), 1, be, yd, 1)
    vec_parity(host(yd), oracle.qgemv(trans, M, N, al, A, M, x, 1, be, y, 1),
               gemv_mag(trans, M, N, al, A, x, 1, be, y, 1), nx, "d", f"qgemv_d {trans} {M}x{N}")
    # beta = 0: y (NaN) not read; alpha = 0: A and x (NaN) not read
    yd = dev(np.full_like(y, np.nan))
    q.qgemv(trans, M, N, al, dev(A), M, dev(x), 1, [0.0] * 4, yd, 1)
    vec_parity(host(yd), oracle.qgemv(trans, M, N, al, A, M, x, 1, np.zeros(4), np.zeros_like(y), 1),
               gemv_mag(trans, M, N, al, A, x, 1, np.zeros(4), y, 1), nx, "d", "qgemv_d beta 0")
    yd = dev(y)
    q.qgemv(trans, M, N, [0.0] * 4, dev(np.full_like(A, np.nan)), M, dev(np.full_like(x, np.nan)), 1, be, yd, 1)
    vec_parity(host(yd), oracle.qgemv(trans, M, N, np.zeros(4), A, M, x, 1, be, y, 1),
               gemv_mag(trans, M, N, np.zeros(4), A, x, 1, be, y, 1), 0, "d", "qgemv_d alpha 0")
