"""GPU checks of the triangular multiply (C-ABI qtrmm_d / qtrmm_s) against
the oracle's qtrmm.  The unreferenced triangle of A (and a unit diagonal)
hold NaN and C starts as NaN, so a read of any of them shows up; C's padding
must stay untouched.  Bars: relative Frobenius 1e-13 (FP64) / 1e-6 (FP32
split) globally and per 32 x 32 block, every real within its componentwise
bound."""
import numpy as np
import pytest

import oracle
import workloads as W
import paper_1903_05575_amd as q
from tests.gpu_util import assert_parity, bound_f64, bound_split, dev, host, logical, norm1, qnorm1, relfro

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-13, "f32": 1e-6}


def run(t, dtype, split_terms=6):
    npd = np.float64 if dtype == "f64" else np.float32
    Ad, Bd, Cd = dev(t["A"].astype(npd)), dev(t["B"].astype(npd)), dev(t["C"].astype(npd))
    q.qtrmm(t["side"], t["uplo"], t["trans"], t["diag"], t["M"], t["N"], t["alpha"], Ad, t["lda"], Bd, t["ldb"],
            Cd, t["ldc"], split_terms=split_terms)
    return host(Cd)


def want(t, dtype):
    npd = np.float64 if dtype == "f64" else np.float32
    A, B = t["A"].astype(npd), t["B"].astype(npd)       # the oracle sees what the GPU sees
    return oracle.qtrmm(t["side"], t["uplo"], t["trans"], t["diag"], t["M"], t["N"], t["alpha"], A, t["lda"], B,
                        t["ldb"], t["C"], t["ldc"])


def trmm_bound(t, dtype):
    """S = |op(T)|_1 |B|_1 (left) or |B|_1 |op(T)|_1 (right); the unread
    triangle counts as zero and a unit diagonal as 1."""
    M, N = t["M"], t["N"]
    n = M if t["side"] == "L" else N
    t1 = np.nan_to_num(norm1(logical(t["A"], n, n)))
    r = np.arange(n)
    keep = (r[:, None] >= r[None, :]) if t["uplo"] == "L" else (r[:, None] <= r[None, :])
    t1 = np.where(keep, t1, 0.0)
    if t["diag"] == "U":
        t1[r, r] = 1.0
    if t["trans"] in "TC":
        t1 = t1.T
    b1 = norm1(logical(t["B"], M, N))
    S = t1 @ b1 if t["side"] == "L" else b1 @ t1
    if dtype == "f64":
        return bound_f64(S, n, qnorm1(t["alpha"]))
    return bound_split(S, n, 6, qnorm1(t["alpha"]))


def check(t, dtype):
    M, N = t["M"], t["N"]
    got = run(t, dtype)
    ref = want(t, dtype)
    label = f"trmm {dtype} {t['side']}{t['uplo']}{t['trans']}{t['diag']} {M}x{N}"
    assert_parity(logical(got, M, N), logical(ref, M, N), trmm_bound(t, dtype), TOL[dtype], label=label)
    assert np.isnan(got[:, M:]).all()                   # padding rows of C untouched


@pytest.mark.parametrize("side", "LR")
@pytest.mark.parametrize("uplo", "LU")
@pytest.mark.parametrize("trans", "NTCR")
@pytest.mark.parametrize("diag", "NU")
def test_trmm_f64(gpu, side, uplo, trans, diag):
    """Every side / triangle / op / diagonal on ragged sizes spanning several tiles."""
    seed = 900 + "LR".index(side) * 16 + "LU".index(uplo) * 8 + "NTCR".index(trans) * 2 + "NU".index(diag)
    check(W.trmm_problem(seed, side, uplo, trans, diag, 150, 97, pad=2), "f64")


@pytest.mark.parametrize("side", "LR")
@pytest.mark.parametrize("uplo", "LU")
@pytest.mark.parametrize("diag", "NU")
def test_trmm_f64_small_triangles(gpu, side, uplo, diag):
    """Triangles smaller than, equal to and just past one K-tile (4) and one
    32-row tile, where every K-tile a tile reaches crosses the diagonal."""
    for i, (n, other) in enumerate(((1, 3), (3, 5), (4, 4), (5, 2), (31, 7), (32, 33), (33, 9))):
        trans = "NTCR"[i % 4]
        M, N = (n, other) if side == "L" else (other, n)
        seed = 1500 + 50 * i + "LR".index(side) * 4 + "LU".index(uplo) * 2 + "NU".index(diag)
        check(W.trmm_problem(seed, side, uplo, trans, diag, M, N, pad=1), "f64")


@pytest.mark.parametrize("side", "LR")
@pytest.mark.parametrize("uplo", "LU")
@pytest.mark.parametrize("trans", "NC")
@pytest.mark.parametrize("diag", "NU")
def test_trmm_f32(gpu, side, uplo, trans, diag):
    seed = 950 + "LR".index(side) * 8 + "LU".index(uplo) * 4 + "NC".index(trans) * 2 + "NU".index(diag)
    check(W.trmm_problem(seed, side, uplo, trans, diag, 133, 161, dist="normal", pad=1), "f32")


@pytest.mark.parametrize("side,uplo", [("L", "L"), ("L", "U"), ("R", "L"), ("R", "U")])
def test_trmm_f64_many_tiles(gpu, side, uplo):
    """More than 512 output tiles, so the weighted tile order takes full
    rounds of 64 tiles per XCD plus a partial one."""
    M, N = (1536, 1472) if side == "L" else (1472, 1536)
    check(W.trmm_problem(980 + "LR".index(side) * 2 + "LU".index(uplo), side, uplo, "N", "N", M, N), "f64")


@pytest.mark.parametrize("diag", "NU")
def test_trmm_equals_gemm_on_dense_triangle(gpu, diag):
    """With the zeros and the unit diagonal written out, qgemm_d over the
    whole K range gives the same bits: the skipped K-tiles of the triangular
    launch contribute exact zeros in the same summation order."""
    M, N = 200, 130
    t = W.trmm_problem(990 + (diag == "U"), "L", "U", "C", diag, M, N, pad=1)
    D = np.nan_to_num(t["A"].copy())
    r = np.arange(M)
    below = r[None, :] > r[:, None]                      # [col, row]: rows below the diagonal
    D[:, :M][below] = 0.0
    if diag == "U":
        D[r, r] = [1.0, 0.0, 0.0, 0.0]
    Cg = dev(np.zeros_like(t["C"]))
    q.qgemm_d("C", "N", M, N, M, t["alpha"], dev(D), t["lda"], dev(t["B"]), t["ldb"], [0.0] * 4, Cg, t["ldc"])
    got = run(t, "f64")
    np.testing.assert_array_equal(logical(got, M, N), logical(host(Cg), M, N))


def test_trmm_alpha_zero_and_empty(gpu):
    """alpha = 0: C <- 0 with A and B all NaN (not read); M = 0 or N = 0: no-op."""
    t = W.trmm_problem(995, "R", "L", "T", "N", 70, 90)
    t = dict(t, A=np.full_like(t["A"], np.nan), B=np.full_like(t["B"], np.nan), alpha=np.zeros(4))
    got = run(t, "f64")
    assert (logical(got, 70, 90) == 0).all()
    Cd = dev(np.full((3, 5, 4), np.nan))
    q.qtrmm("L", "L", "N", "N", 0, 3, [1, 0, 0, 0], None, 1, None, 1, Cd, 5)
    assert np.isnan(host(Cd)).all()


def test_trmm_overlap_rejected(gpu):
    """C may not alias B (the other tiles still read it): rejected before any launch."""
    t = W.trmm_problem(996, "L", "L", "N", "N", 64, 64)
    Ad, Bd = dev(t["A"]), dev(t["B"])
    with pytest.raises(q.QGemmError) as e:
        q.qtrmm("L", "L", "N", "N", 64, 64, t["alpha"], Ad, t["lda"], Bd, t["ldb"], Bd, t["ldb"])
    assert e.value.status == 1 and e.value.arg == 12
