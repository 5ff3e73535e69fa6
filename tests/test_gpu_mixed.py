"""GPU checks of the mixed-type GEMM (C-ABI qgemm_mixed_d) against the
oracle's qgemm_mixed: every type pair and op pair on ragged sizes spanning
several tiles, padding untouched, the BLAS scalar rules.  Bars: relative
Frobenius 1e-13 (double storage; 1e-7 for float storage, whose only extra
error is the final rounding of C), globally and per 32 x 32 block, and every
real within its componentwise bound (the FP64 bound, plus one FP32 rounding
of the result for float storage)."""
import numpy as np
import pytest

import oracle
import workloads as W
import paper_1903_05575_amd as q
from tests.gpu_util import U32, assert_parity, bound_f64, dev, host, logical, norm1, qnorm1, relfro

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


def typed_norm1(kind, X, op, rows, cols):
    """|op(X)_{r c}|_1 of a real ('R'), complex ('Z') or quaternion ('Q')
    operand whose op() is rows x cols."""
    sr, sc = (rows, cols) if op in "NR" else (cols, rows)
    X = np.asarray(X, dtype=np.float64)
    if kind == "R":
        m = np.abs(X[:sc, :sr]).T
    else:
        m = np.abs(X[:sc, :sr, :]).sum(-1).T
    return m if op in "NR" else m.T


def mixed_bound(p):
    M, N, K = p["M"], p["N"], p["K"]
    a1 = typed_norm1(p["typeA"], p["A"], p["opA"], M, K)
    b1 = typed_norm1(p["typeB"], p["B"], p["opB"], K, N)
    al1, be1, c1 = qnorm1(p["alpha"]), qnorm1(p["beta"]), norm1(logical(p["C"], M, N))
    S = a1 @ b1 if K else np.zeros((M, N))
    b = bound_f64(S, K, al1, be1, c1)
    if np.asarray(p["C"]).dtype == np.float32:
        b = b + 1.01 * U32 * (al1 * S + be1 * np.nan_to_num(c1))
    return b


def check(p, tol=1e-13, label=None):
    M, N = p["M"], p["N"]
    got, ref = run(p), want(p)
    label = label or f"mixed {p['typeA']}{p['typeB']} {p['opA']}{p['opB']} {M}x{N}x{p['K']}"
    assert_parity(logical(got, M, N), logical(ref, M, N), mixed_bound(p), tol, label=label)
    np.testing.assert_array_equal(got[:, M:], p["C"][:, M:])          # padding untouched (NaN)
    return got


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
    zC = dict(nanC, C=np.zeros_like(p["C"]))
    assert_parity(logical(got, 40, 50), logical(want(zC), 40, 50), mixed_bound(zC), 1e-13, label="mixed beta 0")
    z = dict(p, A=np.full_like(p["A"], np.nan), B=np.full_like(p["B"], np.nan), alpha=np.zeros(4))
    za = dict(p, alpha=np.zeros(4))
    assert_parity(logical(run(z), 40, 50), logical(want(za), 40, 50), mixed_bound(za), 1e-15, label="mixed alpha 0")
    k0 = dict(p, K=0)
    assert_parity(logical(run(k0), 40, 50), logical(want(k0), 40, 50), mixed_bound(k0), 1e-15, label="mixed K 0")
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
    got = check(p, 1e-7)
    assert got.dtype == np.float32


def test_mixed_f32_quaternion_pair_is_qgemm_s(gpu):
    p = W.gemm_problem(1199, 100, 90, 80, "N", "C", dtype=np.float32)
    Cm, Cg = dev(p["C"]), dev(p["C"])
    A, B = dev(p["A"]), dev(p["B"])
    q.qgemm_mixed("Q", "Q", "N", "C", 100, 90, 80, p["alpha"], A, p["lda"], B, p["ldb"], p["beta"], Cm, p["ldc"])
    q.qgemm_s("N", "C", 100, 90, 80, p["alpha"], A, p["lda"], B, p["ldb"], p["beta"], Cg, p["ldc"])
    np.testing.assert_array_equal(host(Cm), host(Cg))


@pytest.mark.parametrize("tA,tB", PAIRS)
@pytest.mark.parametrize("opA,opB", [("N", "N"), ("T", "T")])
def test_mixed_f32_many_tiles(gpu, tA, tB, opA, opB):
    """Float storage, several tiles in both directions and many K-tiles (a real
    operand takes 32 x 64 tiles with 8-kappa K-tiles here), ragged everywhere."""
    p = as32(W.mixed_problem(1240 + PAIRS.index((tA, tB)) * 2 + (opA == "T"), tA, tB, 333, 290, 517, opA, opB,
                             dist="normal", pad=3))
    got = check(p, 1e-7)
    assert got.dtype == np.float32
