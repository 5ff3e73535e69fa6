"""GPU checks of the FP32 split-BF16 path (C-ABI qgemm_s / qgemm_s_c64)
against the FP64 oracle on the exactly widened FP32 inputs.

Bars (relative Frobenius, also asserted on every 32 x 32 block of outputs):
1e-6 for the default 6-product split and for 9 products, 3e-5 for 3 products
(first order only); every real is also held to the componentwise bound of
tests/gpu_util.py.  The error of every case is printed.

The single-GEMM launcher picks one of three pipelines from the output size
(the rule is mirrored by gpu_util.split_pipeline and asserted by each test
that targets one):
  TL3  32 x 64 tiles, 8-quaternion K-tiles, two LDS stages -- full outputs
       whose 64-row grid fills the block slots (two per CU) clearly worse;
  TL1  64 x 64 tiles, 16-quaternion K-tiles, one LDS stage -- other grids of
       fewer 64 x 64 tiles than block slots;
  TL2  64 x 64 tiles, 8-quaternion K-tiles, two LDS stages -- grids of at
       least one 64 x 64 tile per block slot.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
import paper_1903_05575_amd as q
from tests.gpu_util import (SPLIT_BAR, assert_parity, bound_split, dev, gemm_S, host, logical, norm1, qnorm1,
                            relfro, split_error_bound, split_pipeline)

pytestmark = pytest.mark.gpu
BOUND = SPLIT_BAR


def f32_problem(seed, M, N, K, opA, opB, pad=0, dist="normal", alpha=None, beta=None):
    return W.gemm_problem(seed, M, N, K, opA, opB, dist=dist, dtype=np.float32, pad=pad, alpha=alpha, beta=beta)


def run_gpu(p, terms=6, c64=False):
    A, B = dev(p["A"]), dev(p["B"])
    C = dev(p["C"].astype(np.float64)) if c64 else dev(p["C"])
    q.qgemm_s(p["opA"], p["opB"], p["M"], p["N"], p["K"], p["alpha"], A, p["lda"], B, p["ldb"],
              p["beta"], C, p["ldc"], split_terms=terms)
    return host(C)


def run_oracle(p):
    return oracle.qgemm(p["opA"], p["opB"], p["M"], p["N"], p["K"], p["alpha"], p["A"], p["lda"],
                        p["B"], p["ldb"], p["beta"], p["C"].astype(np.float64), p["ldc"])


def check(p, got, want, terms=6, c64=False, label="", bar=None):
    M, N = p["M"], p["N"]
    assert_parity(logical(got, M, N), logical(want, M, N), split_error_bound(p, terms, c64),
                  BOUND[terms] if bar is None else bar, label=label or f"split{terms}")
    if got.shape[1] > M:   # rows past M of a padded C are never written
        np.testing.assert_array_equal(got[:, M:, :], np.asarray(p["C"], dtype=got.dtype)[:, M:, :])


@pytest.mark.parametrize("opA", "NTCR")
@pytest.mark.parametrize("opB", "NTCR")
def test_split_ops_ragged(gpu, opA, opB):
    """All op pairs, ragged sizes over several tiles (TL3 here)."""
    M, N, K = 150, 131, 200
    p = f32_problem(2000 + "NTCR".index(opA) * 4 + "NTCR".index(opB), M, N, K, opA, opB, pad=3)
    check(p, run_gpu(p), run_oracle(p), label=f"split6 {opA}{opB} {M}x{N}x{K}")


@pytest.mark.parametrize("opA", "NTCR")
@pytest.mark.parametrize("opB", "NTCR")
def test_split_tl2_ops(gpu, opA, opB):
    """TL2 (64 x 64 tiles, two LDS stages, 8-quaternion K-tiles) for all op
    pairs: 2047 x 1000 gives 32 x 16 = 512 tiles, one per block slot; K = 150
    walks 19 K-tiles with a ragged tail and crosses two accumulation panels."""
    M, N, K = 2047, 1000, 150
    assert split_pipeline(M, N) == "TL2"
    p = f32_problem(2100 + "NTCR".index(opA) * 4 + "NTCR".index(opB), M, N, K, opA, opB, pad=1)
    check(p, run_gpu(p), run_oracle(p), label=f"TL2 split6 {opA}{opB}")


@pytest.mark.parametrize("opA,opB", [("N", "N"), ("T", "N"), ("C", "C"), ("T", "R"), ("R", "T")])
def test_split_tl1_full(gpu, opA, opB):
    """TL1 (64 x 64 tiles, one LDS stage, 16-quaternion K-tiles) on a full
    1200 x 1200 output: 19 x 19 = 361 tiles, fewer than the block slots, and
    the 32-row grid would fill them no better."""
    M, N, K = 1200, 1200, 150
    assert split_pipeline(M, N) == "TL1"
    p = f32_problem(2200 + "NTCR".index(opA) * 4 + "NTCR".index(opB), M, N, K, opA, opB, pad=2)
    check(p, run_gpu(p), run_oracle(p), label=f"TL1 split6 {opA}{opB}")


@pytest.mark.parametrize("terms", [3, 6, 9])
def test_split_terms(gpu, terms):
    M, N, K = 96, 200, 777
    p = f32_problem(31, M, N, K, "N", "C")
    check(p, run_gpu(p, terms), run_oracle(p), terms, label=f"split{terms}")


@pytest.mark.parametrize("terms", [3, 9])
@pytest.mark.parametrize("opA,opB", [("N", "C"), ("T", "N")])
def test_split_terms_tl2(gpu, terms, opA, opB):
    """3 and 9 products on the TL2 pipeline."""
    M, N, K = 2047, 1000, 150
    assert split_pipeline(M, N) == "TL2"
    p = f32_problem(2300 + terms + 10 * (opA == "T"), M, N, K, opA, opB)
    check(p, run_gpu(p, terms), run_oracle(p), terms, label=f"TL2 split{terms} {opA}{opB}")


def test_split_c64_output(gpu):
    """FP64 output / beta accumulate: C in float64."""
    M, N, K = 70, 90, 300
    p = f32_problem(41, M, N, K, "C", "N")
    p["C"] = p["C"].astype(np.float64)
    got = run_gpu(p, 6, c64=True)
    assert got.dtype == np.float64
    check(p, got, run_oracle(p), 6, c64=True, label="split6 c64")


@pytest.mark.parametrize("opA,opB", [("N", "N"), ("T", "C"), ("C", "T")])
def test_split_c64_tl2(gpu, opA, opB):
    """FP64 output on the TL2 pipeline."""
    M, N, K = 2047, 1000, 150
    assert split_pipeline(M, N) == "TL2"
    p = f32_problem(2400 + "NTCR".index(opA) * 4 + "NTCR".index(opB), M, N, K, opA, opB, pad=1)
    p["C"] = p["C"].astype(np.float64)
    check(p, run_gpu(p, 6, c64=True), run_oracle(p), 6, c64=True, label=f"TL2 split6 c64 {opA}{opB}")


@pytest.mark.parametrize("M,N,K", [(90, 70, 0), (90, 70, 50), (2047, 1000, 20)])
def test_split_c64_beta_term_in_fp64(gpu, M, N, K):
    """With the product switched off (alpha = 0, or K = 0) the result is
    beta C formed in FP64 from FP64 C values that FP32 cannot hold: every
    real matches the oracle to the rounding of one Hamilton product in FP64
    (an FP32 beta update would be off by about 1e-8 relative)."""
    g = W.rng(2500 + K)
    p = f32_problem(2501 + K, M, N, K, "N", "N", alpha=[0, 0, 0, 0] if K else None)
    C = W.qmatrix(g, M, N, dist="normal", dtype=np.float64)
    C[:, :M] += 1e-9 * g.standard_normal((N, M, 4))       # below FP32 resolution
    p["C"] = C
    got = run_gpu(p, 6, c64=True)
    want = run_oracle(p)
    gl, wl = logical(got, M, N), logical(want, M, N)
    tol = 8 * 2.0 ** -53 * qnorm1(p["beta"]) * norm1(logical(C, M, N))
    err = np.abs(gl - wl)
    print(f"c64 beta term {M}x{N}x{K}: max |err| / (8 u64 |beta| |C|) = {(err / tol[..., None]).max():.3e}, "
          f"rel err {relfro(gl, wl):.3e}")
    assert (err <= tol[..., None]).all()
    c32 = logical(C.astype(np.float32).astype(np.float64), M, N)
    assert np.abs(c32 - logical(C, M, N)).max() > 1e3 * err.max()   # the data does need FP64


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (5, 3, 2), (64, 64, 16), (65, 63, 17), (8, 300, 5), (300, 8, 129)])
def test_split_shapes(gpu, M, N, K):
    p = f32_problem(3 * M + 5 * N + 7 * K, M, N, K, "T", "N")
    check(p, run_gpu(p), run_oracle(p), label=f"split6 {M}x{N}x{K}")


def test_split_special(gpu):
    """beta = 0 ignores NaN in C; alpha = 0 leaves A, B unread."""
    M, N, K = 40, 50, 60
    p = f32_problem(5, M, N, K, "N", "N", beta=[0, 0, 0, 0])
    want = run_oracle(p)
    p2 = dict(p)
    p2["C"] = np.full_like(p["C"], np.nan)
    check(p, run_gpu(p2), want, label="beta 0, NaN C")
    p3 = f32_problem(6, M, N, K, "N", "N", alpha=[0, 0, 0, 0])
    want = run_oracle(p3)
    p3["A"] = np.full_like(p3["A"], np.nan)
    got = run_gpu(p3)
    np.testing.assert_allclose(logical(got, M, N), logical(want, M, N), rtol=1e-6, atol=1e-6)


@pytest.mark.slow
@pytest.mark.parametrize("scaled", [False, True])
def test_precision_4096_sampled(gpu, scaled):
    """M = N = K = 4096, op N/C, N(0,1) components (and the row-scaled case),
    TL2: error against the oracle on a seeded 256-row x 48-column sample of C."""
    p = W.gemm_precision(4096, scaled=scaled)
    got = run_gpu(p)
    g = np.random.default_rng(11 + scaled)
    rows = np.sort(g.choice(4096, 256, replace=False))
    cols = np.sort(g.choice(4096, 48, replace=False))
    want = oracle.qgemm_entries("N", "C", 4096, p["alpha"], p["A"], p["B"], p["beta"],
                                p["C"].astype(np.float64), rows, cols)
    a1 = norm1(logical(p["A"], 4096, 4096)[rows])                      # op N: rows of A
    b1 = norm1(logical(p["B"], 4096, 4096)[cols]).T                    # op C: op(B)[k, nu] = conj B[nu, k]
    bound = bound_split(a1 @ b1, 4096, 6, qnorm1(p["alpha"]))
    assert_parity(got[cols][:, rows].transpose(1, 0, 2), want.transpose(1, 0, 2), bound, BOUND[6],
                  label=f"precision 4096 scaled={scaled} sampled")


@pytest.mark.slow
@pytest.mark.parametrize("opA,opB", [("T", "N"), ("N", "N")])
def test_split_largest_supported_leading_dimension(gpu, opA, opB):
    """The split tiles' 32-bit in-tile offsets allow leading dimensions up to
    2^21 - 1 quaternions for a transposed A or B with op N: parity at the
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
    p = dict(opA=opA, opB=opB, M=M, N=N, K=K, alpha=al, beta=be, A=A[:, :ra].copy(), lda=ra,
             B=B[:, :K].copy(), ldb=K, C=C, ldc=M)
    want = run_oracle(p)
    Cd, Ad, Bd = dev(C), dev(A), dev(B)
    q.qgemm_s(opA, opB, M, N, K, al, Ad, ld, Bd, ld, be, Cd, M)
    check(p, host(Cd), want, label=f"split6 ld 2^21-1 {opA}{opB}")
    lda, ldb = (ld + 1, ld) if opA == "T" else (ld, ld + 1)
    with pytest.raises(q.QGemmError) as e:
        q.qgemm_s(opA, opB, M, N, K, al, Ad, lda, Bd, ldb, be, Cd, M)
    assert e.value.status == 5
