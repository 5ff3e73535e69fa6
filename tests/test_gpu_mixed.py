"""GPU checks of the mixed-type GEMM (C-ABI qgemm_mixed_d) against the
oracle's qgemm_mixed: every type pair and op pair on ragged sizes spanning
several tiles, padding untouched, the BLAS scalar rules."""
import numpy as np
import pytest

import oracle
import workloads as W
import paper_1903_05575_amd as q
from tests.gpu_util import dev, host, logical, relfro

pytestmark = pytest.mark.gpu

PAIRS = [("Q", "R"), ("R", "Q"), ("Q", "Z"), ("Z", "Q")]


def run(p):
    Cd = dev(p["C"])
    q.qgemm_mixed(p["typeA"], p["typeB"], p["opA"], p["opB"], p["M"], p["N"], p["K"], p["alpha"], dev(p["A"]),
                  p["lda"], dev(p["B"]), p["ldb"], p["beta"], Cd, p["ldc"])
    return host(Cd)


def want(p):
    return oracle.qgemm_mixed(p["typeA"], p["typeB"], p["opA"], p["opB"], p["M"], p["N"], p["K"], p["alpha"],
                              p["A"], p["lda"], p["B"], p["ldb"], p["beta"], p["C"], p["ldc"])


def check(p, tol=1e-13):
    M, N = p["M"], p["N"]
    got, ref = run(p), want(p)
    err = relfro(logical(got, M, N), logical(ref, M, N))
    assert err <= tol, err
    np.testing.assert_array_equal(got[:, M:], p["C"][:, M:])          # padding untouched (NaN)


@pytest.mark.parametrize("tA,tB", PAIRS)
@pytest.mark.parametrize("opA", "NTCR")
@pytest.mark.parametrize("opB", "NTCR")
def test_mixed_ops(gpu, tA, tB, opA, opB):
    seed = 1100 + PAIRS.index((tA, tB)) * 16 + "NTCR".index(opA) * 4 + "NTCR".index(opB)
    check(W.mixed_problem(seed, tA, tB, 70, 150, 45, opA, opB, pad=1))


@pytest.mark.parametrize("tA,tB", PAIRS)
def test_mixed_many_tiles(gpu, tA, tB):
    """Several tiles in both directions and many K-tiles, ragged everywhere."""
    check(W.mixed_problem(1170 + PAIRS.index((tA, tB)), tA, tB, 333, 290, 517, "N", "N", dist="normal", pad=3))


def test_mixed_scalar_rules(gpu):
    """beta = 0: C (NaN) not read; alpha = 0: A, B (NaN) not read, C <- beta C;
    K = 0: C <- beta C; M = 0: nothing touched."""
    p = W.mixed_problem(1180, "Z", "Q", 40, 50, 30, "C", "N")
    nanC = dict(p, C=np.full_like(p["C"], np.nan), beta=np.zeros(4))
    got = run(nanC)
    assert np.isfinite(logical(got, 40, 50)).all()
    assert relfro(logical(got, 40, 50), logical(want(dict(nanC, C=np.zeros_like(p["C"]))), 40, 50)) <= 1e-13
    z = dict(p, A=np.full_like(p["A"], np.nan), B=np.full_like(p["B"], np.nan), alpha=np.zeros(4))
    assert relfro(logical(run(z), 40, 50), logical(want(dict(p, alpha=np.zeros(4))), 40, 50)) <= 1e-15
    k0 = dict(p, K=0)
    assert relfro(logical(run(k0), 40, 50), logical(want(k0), 40, 50)) <= 1e-15
    Cd = dev(p["C"])
    q.qgemm_mixed("Q", "R", "N", "N", 0, 50, 30, p["alpha"], None, 1, None, 30, p["beta"], Cd, p["ldc"])
    np.testing.assert_array_equal(host(Cd), p["C"])


def test_mixed_quaternion_pair_is_qgemm(gpu):
    """Both operands quaternion: the same bits as qgemm_d."""
    p = W.gemm_problem(1190, 100, 90, 80, "T", "C", pad=1)
    Cm, Cg = dev(p["C"]), dev(p["C"])
    A, B = dev(p["A"]), dev(p["B"])
    q.qgemm_mixed("Q", "Q", "T", "C", 100, 90, 80, p["alpha"], A, p["lda"], B, p["ldb"], p["beta"], Cm, p["ldc"])
    q.qgemm_d("T", "C", 100, 90, 80, p["alpha"], A, p["lda"], B, p["ldb"], p["beta"], Cg, p["ldc"])
    np.testing.assert_array_equal(host(Cm), host(Cg))


def as32(p):
    return dict(p, A=p["A"].astype(np.float32), B=p["B"].astype(np.float32), C=p["C"].astype(np.float32))


@pytest.mark.parametrize("tA,tB", PAIRS)
@pytest.mark.parametrize("opA,opB", [("N", "N"), ("T", "C"), ("C", "R"), ("R", "T")])
def test_mixed_f32_storage(gpu, tA, tB, opA, opB):
    """qgemm_mixed_s: float storage, FP64 products; against the oracle on the
    same float inputs the only error is the final rounding of C to float."""
    p = as32(W.mixed_problem(1190 + PAIRS.index((tA, tB)) * 4 + [("N", "N"), ("T", "C"), ("C", "R"), ("R", "T")].index(
        (opA, opB)), tA, tB, 150, 97, 133, opA, opB, dist="normal", pad=1))
    M, N = p["M"], p["N"]
    got, ref = run(p), want(p)
    assert got.dtype == np.float32
    assert relfro(logical(got, M, N), logical(ref, M, N)) <= 1e-7
    np.testing.assert_array_equal(got[:, M:], p["C"][:, M:])


def test_mixed_f32_quaternion_pair_is_qgemm_s(gpu):
    p = W.gemm_problem(1199, 100, 90, 80, "N", "C", dtype=np.float32)
    Cm, Cg = dev(p["C"]), dev(p["C"])
    A, B = dev(p["A"]), dev(p["B"])
    q.qgemm_mixed("Q", "Q", "N", "C", 100, 90, 80, p["alpha"], A, p["lda"], B, p["ldb"], p["beta"], Cm, p["ldc"])
    q.qgemm_s("N", "C", 100, 90, 80, p["alpha"], A, p["lda"], B, p["ldb"], p["beta"], Cg, p["ldc"])
    np.testing.assert_array_equal(host(Cm), host(Cg))
