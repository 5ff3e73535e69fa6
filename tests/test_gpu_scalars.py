"""GPU checks of the general scalar placement (C-ABI qgemm_ex_d / qgemm_ex_s):
aL (sum op(A) aM op(B)) aR + bL C bR against the oracle's qgemm_ex."""
import numpy as np
import pytest

import oracle
import workloads as W
import paper_1903_05575_amd as q
from tests.gpu_util import dev, host, logical, relfro

pytestmark = pytest.mark.gpu


def scalars(seed):
    g = W.rng(seed)
    return [g.uniform(-1, 1, 4) for _ in range(5)]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("opA,opB", [("N", "N"), ("T", "C"), ("C", "T"), ("R", "N"), ("N", "R")])
def test_ex_all_scalars(gpu, dtype, opA, opB):
    M, N, K = 97, 130, 75
    p = W.gemm_problem(4000 + "NTCR".index(opA) * 4 + "NTCR".index(opB), M, N, K, opA, opB, pad=2,
                       dtype=np.float64 if dtype == "f64" else np.float32)
    aL, aM, aR, bL, bR = scalars(17)
    want = oracle.qgemm_ex(opA, opB, M, N, K, aL, aM, aR, p["A"], p["lda"], p["B"], p["ldb"], bL, bR,
                           p["C"].astype(np.float64), p["ldc"])
    C = dev(p["C"])
    q.qgemm_ex(opA, opB, M, N, K, aL, aM, aR, dev(p["A"]), p["lda"], dev(p["B"]), p["ldb"], bL, bR, C, p["ldc"])
    got = host(C)
    err = relfro(logical(got, M, N), logical(want, M, N))
    assert err <= (1e-13 if dtype == "f64" else 1e-6), err
    np.testing.assert_array_equal(got[:, M:], p["C"][:, M:])


@pytest.mark.parametrize("which", ["mid", "right", "beta_right"])
def test_ex_single_placement(gpu, which):
    """One non-default scalar at a time, and the defaults reduce to qgemm_d."""
    M, N, K = 64, 70, 40
    p = W.gemm_problem(41, M, N, K, "N", "N")
    s = np.array([0.2, -0.7, 0.5, 0.1])
    kw = dict(aL=None, aM=None, aR=None, bL=p["beta"], bR=None)
    kw[{"mid": "aM", "right": "aR", "beta_right": "bR"}[which]] = s
    want = oracle.qgemm_ex("N", "N", M, N, K, kw["aL"], kw["aM"], kw["aR"], p["A"], p["lda"], p["B"], p["ldb"],
                           kw["bL"], kw["bR"], p["C"], p["ldc"])
    C = dev(p["C"])
    q.qgemm_ex("N", "N", M, N, K, kw["aL"], kw["aM"], kw["aR"], dev(p["A"]), p["lda"], dev(p["B"]), p["ldb"],
               kw["bL"], kw["bR"], C, p["ldc"])
    assert relfro(logical(host(C), M, N), logical(want, M, N)) <= 1e-13
    # all defaults except bL = beta equals qgemm_d with alpha = 1
    C1, C2 = dev(p["C"]), dev(p["C"])
    q.qgemm_ex("N", "N", M, N, K, None, None, None, dev(p["A"]), p["lda"], dev(p["B"]), p["ldb"], p["beta"], None,
               C1, p["ldc"])
    q.qgemm_d("N", "N", M, N, K, [1, 0, 0, 0], dev(p["A"]), p["lda"], dev(p["B"]), p["ldb"], p["beta"], C2, p["ldc"])
    np.testing.assert_array_equal(host(C1), host(C2))


def test_ex_zero_alpha_skips_product(gpu):
    M, N, K = 30, 20, 10
    p = W.gemm_problem(42, M, N, K, "N", "N")
    aL, aM, aR, bL, bR = scalars(3)
    aM = np.zeros(4)
    A = np.full_like(p["A"], np.nan)
    want = oracle.qgemm_ex("N", "N", M, N, K, aL, aM, aR, A, p["lda"], p["B"], p["ldb"], bL, bR, p["C"], p["ldc"])
    C = dev(p["C"])
    q.qgemm_ex("N", "N", M, N, K, aL, aM, aR, dev(A), p["lda"], dev(p["B"]), p["ldb"], bL, bR, C, p["ldc"])
    got = logical(host(C), M, N)
    assert np.isfinite(got).all()
    np.testing.assert_allclose(got, logical(want, M, N), rtol=1e-14, atol=1e-14)
