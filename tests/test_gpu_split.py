"""GPU checks of the FP32 split-BF16 path (C-ABI qgemm_s / qgemm_s_c64)
against the FP64 oracle on the exactly widened FP32 inputs.

The bar for the default 6-term split is a relative Frobenius error <= 1e-6;
3 terms (first order only) is expected near 1e-5 and checked at 3e-5; 9
terms is bounded like 6.  The error of every case is printed.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_1903_05575_amd as q
from tests.gpu_util import dev, host, logical, relfro

pytestmark = pytest.mark.gpu
BOUND = {3: 3e-5, 6: 1e-6, 9: 1e-6}


def f32_problem(seed, M, N, K, opA, opB, pad=0, dist="normal", alpha=None, beta=None):
    p = W.gemm_problem(seed, M, N, K, opA, opB, dist=dist, dtype=np.float32, pad=pad, alpha=alpha, beta=beta)
    return p


def run_gpu(p, terms=6, c64=False):
    A, B = dev(p["A"]), dev(p["B"])
    C = dev(p["C"].astype(np.float64)) if c64 else dev(p["C"])
    q.qgemm_s(p["opA"], p["opB"], p["M"], p["N"], p["K"], p["alpha"], A, p["lda"], B, p["ldb"],
              p["beta"], C, p["ldc"], split_terms=terms)
    return host(C)


def run_oracle(p):
    return oracle.qgemm(p["opA"], p["opB"], p["M"], p["N"], p["K"], p["alpha"], p["A"], p["lda"],
                        p["B"], p["ldb"], p["beta"], p["C"].astype(np.float64), p["ldc"])


@pytest.mark.parametrize("opA", "NTCR")
@pytest.mark.parametrize("opB", "NTCR")
def test_split_ops_ragged(gpu, opA, opB):
    M, N, K = 150, 131, 200
    p = f32_problem(2000 + "NTCR".index(opA) * 4 + "NTCR".index(opB), M, N, K, opA, opB, pad=3)
    want = run_oracle(p)
    got = run_gpu(p)
    err = relfro(logical(got, M, N), logical(want, M, N))
    print(f"split6 {opA}{opB} {M}x{N}x{K}: rel err {err:.3e}")
    assert err <= BOUND[6]
    if got.shape[1] > M:
        np.testing.assert_array_equal(got[:, M:, :], p["C"][:, M:, :])


@pytest.mark.parametrize("terms", [3, 6, 9])
def test_split_terms(gpu, terms):
    M, N, K = 96, 200, 777
    p = f32_problem(31, M, N, K, "N", "C")
    want = run_oracle(p)
    err = relfro(logical(run_gpu(p, terms), M, N), logical(want, M, N))
    print(f"split{terms}: rel err {err:.3e}")
    assert err <= BOUND[terms]


def test_split_c64_output(gpu):
    """FP64 output / beta accumulate: C in float64."""
    M, N, K = 70, 90, 300
    p = f32_problem(41, M, N, K, "C", "N")
    want = run_oracle(p)
    got = run_gpu(p, 6, c64=True)
    err = relfro(logical(got, M, N), logical(want, M, N))
    print(f"split6 c64: rel err {err:.3e}")
    assert got.dtype == np.float64 and err <= BOUND[6]


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (5, 3, 2), (64, 64, 16), (65, 63, 17), (8, 300, 5), (300, 8, 129)])
def test_split_shapes(gpu, M, N, K):
    p = f32_problem(3 * M + 5 * N + 7 * K, M, N, K, "T", "N")
    want = run_oracle(p)
    err = relfro(logical(run_gpu(p), M, N), logical(want, M, N))
    assert err <= BOUND[6], err


def test_split_special(gpu):
    """beta = 0 ignores NaN in C; alpha = 0 leaves A, B unread."""
    M, N, K = 40, 50, 60
    p = f32_problem(5, M, N, K, "N", "N", beta=[0, 0, 0, 0])
    want = run_oracle(p)
    p2 = dict(p)
    p2["C"] = np.full_like(p["C"], np.nan)
    got = run_gpu(p2)
    assert relfro(logical(got, M, N), logical(want, M, N)) <= BOUND[6]
    p3 = f32_problem(6, M, N, K, "N", "N", alpha=[0, 0, 0, 0])
    want = run_oracle(p3)
    p3["A"] = np.full_like(p3["A"], np.nan)
    got = run_gpu(p3)
    np.testing.assert_allclose(logical(got, M, N), logical(want, M, N), rtol=1e-6, atol=1e-6)


@pytest.mark.slow
@pytest.mark.parametrize("scaled", [False, True])
def test_precision_4096_sampled(gpu, scaled):
    """M = N = K = 4096, op N/C, N(0,1) components (and the row-scaled case);
    error against the oracle on a seeded 256-row x 48-column sample of C."""
    p = W.gemm_precision(4096, scaled=scaled)
    got = run_gpu(p)
    g = np.random.default_rng(11 + scaled)
    rows = np.sort(g.choice(4096, 256, replace=False))
    cols = np.sort(g.choice(4096, 48, replace=False))
    want = oracle.qgemm_entries("N", "C", 4096, p["alpha"], p["A"], p["B"], p["beta"],
                                p["C"].astype(np.float64), rows, cols)
    err = relfro(got[cols][:, rows], want)
    print(f"precision 4096 scaled={scaled}: sampled rel err {err:.3e}")
    assert err <= BOUND[6]


@pytest.mark.slow
@pytest.mark.parametrize("opA,opB", [("T", "N"), ("N", "N")])
def test_split_largest_supported_leading_dimension(gpu, opA, opB):
    """The split tiles' 32-bit in-tile offsets allow leading dimensions up to
    2^21 - 1 quaternions for a transposed A or B with op N: exact parity at the
    limit, refusal one past it."""
    ld = (1 << 21) - 1
    M, N, K = 70, 66, 20
    g = W.rng(1520 + (opA == "T"))
    ra, ca = (M, K) if opA == "N" else (K, M)
    A = np.full((ca, ld, 4), np.nan, dtype=np.float32)
    A[:, :ra] = g.standard_normal((ca, ra, 4))
    B = np.full((N, ld, 4), np.nan, dtype=np.float32)
    B[:, :K] = g.standard_normal((N, K, 4))
    C = W.qmatrix(g, M, N, ld=M, dtype=np.float32)
    al, be = W.quaternion(g), W.quaternion(g)
    want = oracle.qgemm(opA, opB, M, N, K, al, A[:, :ra].copy(), ra, B[:, :K].copy(), K, be, C, M)
    Cd, Ad, Bd = dev(C), dev(A), dev(B)
    q.qgemm_s(opA, opB, M, N, K, al, Ad, ld, Bd, ld, be, Cd, M)
    assert relfro(logical(host(Cd), M, N), logical(want, M, N)) <= 1e-6
    lda, ldb = (ld + 1, ld) if opA == "T" else (ld, ld + 1)
    with pytest.raises(q.QGemmError) as e:
        q.qgemm_s(opA, opB, M, N, K, al, Ad, lda, Bd, ldb, be, Cd, M)
    assert e.value.status == 5
