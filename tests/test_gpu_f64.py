"""GPU parity of the FP64 path (C-ABI qgemm_d) against the CPU oracle.

Bar: relative Frobenius error <= 1e-13 over all 4MN reals, and every real
within the componentwise rounding bound (4K+8) u (|alpha| S + |beta| |C|).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_1903_05575_amd as q
from tests.gpu_util import dev, host, logical, relfro, error_bound

pytestmark = pytest.mark.gpu
TOL = 1e-13


def run_gpu(p):
    A, B, C = dev(p["A"]), dev(p["B"]), dev(p["C"])
    q.qgemm_d(p["opA"], p["opB"], p["M"], p["N"], p["K"], p["alpha"], A, p["lda"], B, p["ldb"],
              p["beta"], C, p["ldc"])
    return host(C)


def run_oracle(p):
    return oracle.qgemm(p["opA"], p["opB"], p["M"], p["N"], p["K"], p["alpha"], p["A"], p["lda"],
                        p["B"], p["ldb"], p["beta"], p["C"], p["ldc"])


def check(p, got, want):
    M, N = p["M"], p["N"]
    g, w = logical(got, M, N), logical(want, M, N)
    assert np.isfinite(g).all()
    assert relfro(g, w) <= TOL, relfro(g, w)
    bound = error_bound(p)
    assert (np.abs(g - w) <= bound[..., None] + 1e-300).all()
    # rows beyond M in a padded C are never written
    if got.shape[1] > M:
        np.testing.assert_array_equal(got[:, M:, :], p["C"][:, M:, :])


def test_small_64(gpu):
    p = W.gemm_small()
    check(p, run_gpu(p), run_oracle(p))


@pytest.mark.parametrize("opA", "NTCR")
@pytest.mark.parametrize("opB", "NTCR")
def test_ops_ragged(gpu, opA, opB):
    """All op pairs on a ragged size spanning several 64x64x8 tiles with padded
    leading dimensions and random quaternion alpha, beta."""
    M, N, K = 150, 131, 77
    p = W.gemm_problem(1000 + "NTCR".index(opA) * 4 + "NTCR".index(opB), M, N, K, opA, opB, pad=3)
    check(p, run_gpu(p), run_oracle(p))


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (3, 5, 2), (64, 64, 8), (65, 63, 9), (4, 300, 5),
                                   (300, 4, 130), (17, 1, 300), (128, 192, 256)])
def test_shapes(gpu, M, N, K):
    p = W.gemm_problem(7 * M + 11 * N + 13 * K, M, N, K, "N", "T")
    check(p, run_gpu(p), run_oracle(p))


def test_beta_zero_nan_c(gpu):
    p = W.gemm_problem(5, 70, 66, 20, "C", "N", beta=[0, 0, 0, 0])
    p["C"] = np.full_like(p["C"], np.nan)
    got = run_gpu(p)
    want = run_oracle(p)
    assert np.isfinite(logical(got, 70, 66)).all()
    p["C"] = np.zeros_like(p["C"])
    check(p, got, want)


def test_alpha_zero_and_k_zero(gpu):
    """alpha == 0 or K == 0: C <- beta C, A and B not read (NaN there is harmless)."""
    p = W.gemm_problem(6, 40, 33, 12, "N", "N", alpha=[0, 0, 0, 0])
    p["A"] = np.full_like(p["A"], np.nan)
    p["B"] = np.full_like(p["B"], np.nan)
    got, want = run_gpu(p), run_oracle(p)
    np.testing.assert_allclose(logical(got, 40, 33), logical(want, 40, 33), rtol=1e-15, atol=1e-15)
    p = W.gemm_problem(7, 40, 33, 0, "N", "N")
    got, want = run_gpu(p), run_oracle(p)
    np.testing.assert_allclose(logical(got, 40, 33), logical(want, 40, 33), rtol=1e-15, atol=1e-15)


def test_empty_is_noop(gpu):
    C = dev(np.ones((3, 5, 4)))
    q.qgemm_d("N", "N", 0, 3, 4, [1, 0, 0, 0], None, 1, None, 4, [1, 0, 0, 0], C, 5)
    q.qgemm_d("N", "N", 5, 0, 4, [1, 0, 0, 0], None, 5, None, 4, [1, 0, 0, 0], C, 5)
    assert (host(C) == 1).all()


def test_deterministic(gpu):
    p = W.gemm_problem(8, 200, 190, 300, "T", "C")
    a, b = run_gpu(p), run_gpu(p)
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("n,opA,opB", [(1024, "N", "N"), (1024, "C", "T"), (2048, "T", "C")])
def test_sweep_full(gpu, n, opA, opB):
    """Sweep sizes with the full oracle (element by element)."""
    p = W.gemm_sweep(n, opA, opB)
    check(p, run_gpu(p), run_oracle(p))


@pytest.mark.slow
@pytest.mark.parametrize("opA,opB", [("N", "N"), ("C", "T"), ("T", "C")])
def test_sweep_8192_sampled(gpu, opA, opB):
    """M = N = K = 8192 in the benchmark's launch configuration, checked on a
    seeded sample of 128 rows x 64 columns of C computed by the oracle."""
    n = 8192
    p = W.gemm_sweep(n, opA, opB)
    got = run_gpu(p)
    g = np.random.default_rng(n + len(opA + opB))
    rows = np.sort(g.choice(n, 128, replace=False))
    cols = np.sort(g.choice(n, 64, replace=False))
    want = oracle.qgemm_entries(opA, opB, n, p["alpha"], p["A"], p["B"], p["beta"], p["C"], rows, cols)
    gs = got[cols][:, rows]
    assert relfro(gs, want) <= TOL, relfro(gs, want)
    # componentwise rounding bound on the sample
    a1 = np.abs(p["A"][:, rows, :] if opA in "NR" else p["A"][rows, :n, :].transpose(1, 0, 2)).sum(-1)
    b1 = np.abs(p["B"][cols, :n, :].transpose(1, 0, 2) if opB in "NR" else p["B"][:, cols, :]).sum(-1)
    S = a1.T @ b1                                   # (rows, cols)
    c1 = np.abs(p["C"][cols][:, rows, :]).sum(-1).T
    bound = (4 * n + 8) * 2.0 ** -53 * (np.abs(p["alpha"]).sum() * S + np.abs(p["beta"]).sum() * c1)
    err = np.abs(gs - want).transpose(1, 0, 2)
    assert (err <= bound[..., None]).all()


@pytest.mark.slow
@pytest.mark.parametrize("opA,opB", [("T", "N"), ("N", "N"), ("C", "T")])
def test_largest_supported_leading_dimension(gpu, opA, opB):
    """The largest leading dimension the 32-bit in-tile offsets allow
    (2^20 - 1 quaternions: a 64-wide tile of a transposed A, or of B with op N,
    spans just under 2^31 bytes): exact parity, no offset wrap."""
    ld = (1 << 20) - 1
    M, N, K = 70, 66, 12
    g = W.rng(1500 + "NTC".index(opA) * 3 + "NTC".index(opB))
    ra, ca = (M, K) if opA == "N" else (K, M)
    rb, cb = (K, N) if opB == "N" else (N, K)
    A = np.full((ca, ld, 4), np.nan)
    A[:, :ra] = g.uniform(-1, 1, (ca, ra, 4))
    B = np.full((cb, ld, 4), np.nan)
    B[:, :rb] = g.uniform(-1, 1, (cb, rb, 4))
    C = W.qmatrix(g, M, N, ld=M + 1)
    al, be = W.quaternion(g), W.quaternion(g)
    # the oracle gets the same logical operands, compactly stored
    want = oracle.qgemm(opA, opB, M, N, K, al, A[:, :ra].copy(), ra, B[:, :rb].copy(), rb, be, C, M + 1)
    Cd, Ad, Bd = dev(C), dev(A), dev(B)
    q.qgemm_d(opA, opB, M, N, K, al, Ad, ld, Bd, ld, be, Cd, M + 1)
    assert relfro(logical(host(Cd), M, N), logical(want, M, N)) <= 1e-13
    # one more on the operand whose tile spans the full leading dimension is refused, not wrapped
    lda, ldb = (ld + 1, ld) if opA in "TC" else (ld, ld + 1)
    with pytest.raises(q.QGemmError) as e:
        q.qgemm_d(opA, opB, M, N, K, al, Ad, lda, Bd, ldb, be, Cd, M + 1)
    assert e.value.status == 5


@pytest.mark.parametrize("opA", "NTCR")
@pytest.mark.parametrize("opB", "NTCR")
def test_ops_ragged_full_output_tiles(gpu, opA, opB):
    """Full outputs run 32-row tiles: every op pair, ragged in M, N and K
    (300 x 250 x 37: partial tiles in every dimension; 2040 x 2000 x 29: a
    grid of 64 x 32 tiles whose last tile row holds 24 rows)."""
    for i, (M, N, K) in enumerate(((300, 250, 37), (2040, 2000, 29))):
        p = W.gemm_problem(1600 + 32 * i + "NTCR".index(opA) * 4 + "NTCR".index(opB), M, N, K, opA, opB, pad=1)
        Cd = dev(p["C"])
        q.qgemm_d(opA, opB, M, N, K, p["alpha"], dev(p["A"]), p["lda"], dev(p["B"]), p["ldb"], p["beta"], Cd, p["ldc"])
        want = oracle.qgemm(opA, opB, M, N, K, p["alpha"], p["A"], p["lda"], p["B"], p["ldb"], p["beta"], p["C"],
                            p["ldc"])
        got = host(Cd)
        assert relfro(logical(got, M, N), logical(want, M, N)) <= 1e-13, (M, N, K)
        np.testing.assert_array_equal(got[:, M:], p["C"][:, M:])
