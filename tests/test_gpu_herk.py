"""GPU checks of the Hermitian rank-k update (C-ABI qherk_d / qherk_s)
against the oracle's qherk: the triangle within the path's bars (relative
Frobenius 1e-13 FP64 / 1e-6 FP32 split, globally and per 32 x 32 block, and
every real within its componentwise bound), the other triangle and padding
untouched bit for bit, the diagonal real."""
import numpy as np
import pytest

import oracle
import workloads as W
import paper_1903_05575_amd as q
from tests.gpu_util import assert_parity, bound_f64, bound_split, dev, host, logical, norm1, relfro

pytestmark = pytest.mark.gpu


def tri_mask(n, uplo):
    mu, nu = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return mu >= nu if uplo == "L" else mu <= nu


def problem(seed, n, k, trans, dtype):
    g = W.rng(seed)
    rows, cols = (n, k) if trans == "N" else (k, n)
    A = W.qmatrix(g, rows, cols, ld=rows + 2, dtype=dtype)
    C = W.qmatrix(g, n, n, ld=n + 1, dtype=dtype)
    return A, rows + 2, C, n + 1


def herk_bound(A, n, k, trans, alpha, beta, C, dtype):
    """S = |op(A)|_1 |op(A)|_1^T over kappa; alpha, beta real."""
    a1 = norm1(logical(A, n, k) if trans == "N" else logical(A, k, n).transpose(1, 0, 2))
    c1 = norm1(logical(C, n, n))
    if dtype == "f64":
        return bound_f64(a1 @ a1.T, k, abs(alpha), abs(beta), c1)
    return bound_split(a1 @ a1.T, k, 6, abs(alpha), abs(beta), c1)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("uplo", "LU")
@pytest.mark.parametrize("trans", "NC")
def test_herk(gpu, dtype, uplo, trans):
    n, k = 150, 77
    npd = np.float64 if dtype == "f64" else np.float32
    A, lda, C, ldc = problem(800 + len(uplo + trans) + (dtype == "f32"), n, k, trans, npd)
    alpha, beta = 0.75, -0.5
    want = oracle.qherk(uplo, trans, n, k, alpha, A, lda, beta, C.astype(np.float64), ldc)
    Cd = dev(C)
    q.qherk(uplo, trans, n, k, alpha, dev(A), lda, beta, Cd, ldc)
    got = host(Cd)
    gl, wl, cl = logical(got, n, n), logical(want, n, n), logical(C, n, n)
    m = tri_mask(n, uplo)
    assert_parity(gl, wl, herk_bound(A, n, k, trans, alpha, beta, C, dtype), 1e-13 if dtype == "f64" else 1e-6,
                  mask=m, label=f"herk {dtype} {uplo}{trans}")
    np.testing.assert_array_equal(gl[~m], cl[~m])                 # other triangle untouched
    assert (gl[np.arange(n), np.arange(n), 1:] == 0).all()         # real diagonal
    np.testing.assert_array_equal(got[:, n:], C[:, n:])            # padding untouched


def test_herk_special(gpu):
    n, k = 70, 20
    A, lda, C, ldc = problem(5, n, k, "N", np.float64)
    # alpha == 0, beta == 1: untouched entirely
    Cd = dev(C)
    q.qherk("L", "N", n, k, 0.0, dev(A), lda, 1.0, Cd, ldc)
    np.testing.assert_array_equal(host(Cd), C)
    # beta == 0: C (NaN) not read on the triangle
    Cn = np.full_like(C, np.nan)
    Cd = dev(Cn)
    q.qherk("U", "N", n, k, 1.0, dev(A), lda, 0.0, Cd, ldc)
    got = logical(host(Cd), n, n)
    m = tri_mask(n, "U")
    assert np.isfinite(got[m]).all() and np.isnan(got[~m]).all()
    want = logical(oracle.qherk("U", "N", n, k, 1.0, A, lda, 0.0, np.zeros_like(C), ldc), n, n)
    got[~m] = 0.0
    assert_parity(got, want, herk_bound(A, n, k, "N", 1.0, 0.0, C, "f64"), 1e-13, mask=m, label="herk beta 0")


def test_herk_equals_gemm_triangle(gpu):
    """Off the diagonal, qherk_d equals qgemm_d(N, C) with B = A on the triangle, bitwise
    (same kernel, same summation order)."""
    n, k = 130, 45
    A, lda, C, ldc = problem(6, n, k, "N", np.float64)
    Cg, Ch = dev(C), dev(C)
    Ad = dev(A)
    q.qgemm_d("N", "C", n, n, k, [0.5, 0, 0, 0], Ad, lda, Ad, lda, [2.0, 0, 0, 0], Cg, ldc)
    q.qherk("L", "N", n, k, 0.5, Ad, lda, 2.0, Ch, ldc)
    g, h = logical(host(Cg), n, n), logical(host(Ch), n, n)
    m = tri_mask(n, "L") & ~np.eye(n, dtype=bool)
    np.testing.assert_array_equal(g[m], h[m])
