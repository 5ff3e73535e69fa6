"""GPU checks of the general scalar placement (C-ABI qgemm_ex_d / qgemm_ex_s):
aL (sum op(A) aM op(B)) aR + bL C bR against the oracle's qgemm_ex.
Bars: relative Frobenius 1e-13 (FP64) / 1e-6 (FP32 split) globally and per
32 x 32 block, every real within its componentwise bound (the middle scalar
scales op(B) as it is staged: five more roundings; the right scalars one more
Hamilton product in the epilogue)."""
import numpy as np
import pytest

import oracle
import workloads as W
import paper_1903_05575_amd as q
from tests.gpu_util import (U64, U_ACC32, assert_parity, bound_f64, bound_split, dev, gamma, gemm_S, host, logical,
                            norm1, qnorm1, relfro, split_pipeline)

pytestmark = pytest.mark.gpu


def ex_bound(p, aL, aM, aR, bL, bR, f64):
    one = np.array([1.0, 0, 0, 0])
    aL, aM, aR, bR = (one if x is None else x for x in (aL, aM, aR, bR))
    bL = np.zeros(4) if bL is None else bL
    S = gemm_S(p) * qnorm1(aM)
    a1 = qnorm1(aL) * qnorm1(aR)
    c1 = norm1(logical(p["C"], p["M"], p["N"]))
    b1 = qnorm1(bL) * qnorm1(bR)
    if f64:
        return bound_f64(S, p["K"], a1, b1, c1, extra=8 + 5 + 4)
    return bound_split(S, p["K"], 6, a1, b1, c1, pre=5, post=10)


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
    assert_parity(logical(got, M, N), logical(want, M, N), ex_bound(p, aL, aM, aR, bL, bR, dtype == "f64"),
                  1e-13 if dtype == "f64" else 1e-6, label=f"ex {dtype} {opA}{opB}")
    np.testing.assert_array_equal(got[:, M:], p["C"][:, M:])


@pytest.mark.parametrize("opA,opB", [("T", "N"), ("T", "C"), ("C", "R")])
def test_ex_s_tl2(gpu, opA, opB):
    """qgemm_ex_s with a transposed A on the TL2 pipeline (2047 x 1000
    outputs), all five scalars."""
    M, N, K = 2047, 1000, 150
    assert split_pipeline(M, N) == "TL2"
    p = W.gemm_problem(4100 + "NTCR".index(opA) * 4 + "NTCR".index(opB), M, N, K, opA, opB, pad=1,
                       dtype=np.float32, dist="normal")
    aL, aM, aR, bL, bR = scalars(18)
    want = oracle.qgemm_ex(opA, opB, M, N, K, aL, aM, aR, p["A"], p["lda"], p["B"], p["ldb"], bL, bR,
                           p["C"].astype(np.float64), p["ldc"])
    C = dev(p["C"])
    q.qgemm_ex(opA, opB, M, N, K, aL, aM, aR, dev(p["A"]), p["lda"], dev(p["B"]), p["ldb"], bL, bR, C, p["ldc"])
    got = host(C)
    assert_parity(logical(got, M, N), logical(want, M, N), ex_bound(p, aL, aM, aR, bL, bR, False), 1e-6,
                  label=f"TL2 ex_s {opA}{opB}")
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
    assert_parity(logical(host(C), M, N), logical(want, M, N), ex_bound(p, *(kw[k] for k in ("aL", "aM", "aR", "bL", "bR")),
                  True), 1e-13, label=f"ex single {which}")
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
    bound = gamma(20, U64) * qnorm1(bL) * qnorm1(bR) * norm1(logical(p["C"], M, N))
    assert_parity(got, logical(want, M, N), bound, 1e-14, label="ex zero middle scalar")
