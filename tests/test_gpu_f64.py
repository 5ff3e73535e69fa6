"""GPU parity of the FP64 path (C-ABI qgemm_d) against the CPU oracle.

Bar: relative Frobenius error <= 1e-13 over all 4MN reals and over every
32 x 32 block of outputs, and every real within the componentwise rounding
bound (4K+8) u (|alpha| S + |beta| |C|) of tests/gpu_util.py.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_1903_05575_amd as q
from tests.gpu_util import F64_BAR, assert_parity, bound_f64, dev, error_bound, host, logical, norm1, qnorm1, relfro

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


def check(p, got, want, label="qgemm_d"):
    M, N = p["M"], p["N"]
    assert_parity(logical(got, M, N), logical(want, M, N), error_bound(p), TOL, label=label)
    # rows beyond M in a padded C are never written
    if got.shape[1] > M:
        np.testing.assert_array_equal(got[:, M:, :], p["C"][:, M:, :])


def sampled_bound(p, n, rows, cols):
    """Componentwise bound on a rows x cols sample of an n^3 problem."""
    opA, opB, A, B = p["opA"], p["opB"], p["A"], p["B"]
    a1 = norm1(A[:, rows, :] if opA in "NR" else A[rows, :n, :].transpose(1, 0, 2)).T   # (rows, n)
    b1 = norm1(B[cols, :n, :].transpose(1, 0, 2) if opB in "NR" else B[:, cols, :])      # (n, cols)
    c1 = norm1(p["C"][cols][:, rows, :]).T
    return bound_f64(a1 @ b1, n, qnorm1(p["alpha"]), qnorm1(p["beta"]), c1)


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
    p["A"], p["B"] = np.zeros_like(p["A"]), np.zeros_like(p["B"])
    check(p, got, want, "alpha 0")
    p = W.gemm_problem(7, 40, 33, 0, "N", "N")
    check(p, run_gpu(p), run_oracle(p), "K 0")


def test_empty_is_noop(gpu):
    C = dev(np.ones((3, 5, 4)))
    q.qgemm_d("N", "N", 0, 3, 4, [1, 0, 0, 0], None, 1, None, 4, [1, 0, 0, 0], C, 5)
    q.qgemm_d("N", "N", 5, 0, 4, [1, 0, 0, 0], None, 5, None, 4, [1, 0, 0, 0], C, 5)
    assert (host(C) == 1).all()


def test_deterministic(gpu):
    p = W.gemm_problem(8, 200, 190, 300, "T", "C")
    a, b = run_gpu(p), run_gpu(p)
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("opA,opB", W.OP_PAIRS)
def test_sweep_1024_full(gpu, opA, opB):
    """The 1024^3 sweep cases (all nine op pairs of {N, T, C}) against the full
    oracle, element by element."""
    p = W.gemm_sweep(1024, opA, opB)
    check(p, run_gpu(p), run_oracle(p), f"sweep 1024 {opA}{opB}")


@pytest.mark.slow
@pytest.mark.parametrize("n", [2048, 4096, 8192])
@pytest.mark.parametrize("opA,opB", W.OP_PAIRS)
def test_sweep_sampled(gpu, n, opA, opB):
    """The 2048^3, 4096^3 and 8192^3 sweep cases (all nine op pairs) in the
    benchmark's launch configuration, checked on a seeded sample of 256 rows
    x 128 columns of C that the oracle computes entry by entry."""
    p = W.gemm_sweep(n, opA, opB)
    got = run_gpu(p)
    g = np.random.default_rng(n + 3 * W.OP_PAIRS.index((opA, opB)))
    rows = np.sort(g.choice(n, 256, replace=False))
    cols = np.sort(g.choice(n, 128, replace=False))
    want = oracle.qgemm_entries(opA, opB, n, p["alpha"], p["A"], p["B"], p["beta"], p["C"], rows, cols)
    assert_parity(got[cols][:, rows].transpose(1, 0, 2), want.transpose(1, 0, 2), sampled_bound(p, n, rows, cols),
                  TOL, label=f"sweep {n} {opA}{opB} sampled")


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
    pc = dict(opA=opA, opB=opB, M=M, N=N, K=K, alpha=al, beta=be, A=A[:, :ra], B=B[:, :rb], C=C)
    check(pc, host(Cd), want, f"ld 2^20-1 {opA}{opB}")
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
        check(p, host(Cd), want, f"32-row tiles {opA}{opB} {M}x{N}x{K}")


@pytest.mark.parametrize("opA", "NTCR")
@pytest.mark.parametrize("opB", "NTCR")
def test_tile_width_choice_both_sides(gpu, opA, opB):
    """Full outputs whose 32 x 64 grid fills the block slots poorly take 32 x 32
    tiles with 8-kappa K-tiles (1000 x 1000: 32 x 16 = 512 tiles against 1024
    of 32 x 32); 1100 x 1100 keeps the 32 x 64 tiles (630 of them, no better
    filled by 32 x 32).  Both ragged in M, N and K, padded leading dimensions,
    every op pair: within the bar on every element."""
    for i, (M, N, K) in enumerate(((1000, 1000, 37), (1100, 1100, 29))):
        p = W.gemm_problem(1700 + 32 * i + "NTCR".index(opA) * 4 + "NTCR".index(opB), M, N, K, opA, opB, pad=1)
        check(p, run_gpu(p), run_oracle(p), f"tile width {opA}{opB} {M}x{N}x{K}")
