"""Seeded synthetic inputs for quaternion GEMM.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic, so both the CPU oracle and the GPU path can be fed from it
with identical bits.

The paper times square products with alpha = 1, beta = 0 on unspecified values
(Sec. 5).  The generators below reproduce the shapes and value distributions
of the five workloads this library is measured on:

  * ``gemm_small``      -- FP64, op N/N, 64^3, alpha = 1, beta = 0, N(0,1)
  * ``gemm_sweep``      -- FP64, M=N=K in {1024..8192}, any op pair, lda = stored
                           rows, alpha/beta random quaternions, U[-1,1] entries
  * ``gemm_precision``  -- FP32, 4096^3, op N/C, N(0,1), optionally with the rows
                           of op(A) and the K index of op(B) scaled by 10^U[-3,3]
  * ``grouped``         -- 4096 FP32 problems, M,N,K = round(exp(U[ln 8, ln 512])),
                           op N/N, alpha = 1, beta = 0.5, U[-1,1]
  * ``linear_layer``    -- FP32 X (8192 x 1024), W (1024 x 1024) with Glorot
                           sigma = sqrt(2 / (4*1024 + 4*1024)) = 1/64 per component,
                           upstream gradient N(0,1)

Storage convention: a rows x cols quaternion matrix with leading dimension ld
is an array of shape (cols, ld, 4): column-major, four interleaved components.
"""
import numpy as np

BASE_SEED = 1903055750


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def stored_dims(op, rows, cols):
    """(rows, cols) of the stored operand whose op() is rows x cols."""
    return (rows, cols) if op in ("N", "R") else (cols, rows)


def qmatrix(g, rows, cols, ld=None, dist="normal", dtype=np.float64, sigma=1.0):
    """Random quaternion matrix in storage layout (cols, ld, 4).

    Padding rows (ld > rows) are filled with NaN so that a kernel that reads
    outside the logical matrix shows up in the result."""
    ld = max(rows, 1) if ld is None else ld
    if dist == "normal":
        v = g.standard_normal((cols, rows, 4)) * sigma
    elif dist == "uniform":
        v = g.uniform(-1.0, 1.0, (cols, rows, 4))
    else:
        raise ValueError(dist)
    out = np.full((cols, ld, 4), np.nan, dtype=dtype)
    out[:, :rows, :] = v.astype(dtype)
    return out


def quaternion(g, dist="uniform"):
    if dist == "uniform":
        return g.uniform(-1.0, 1.0, 4)
    return g.standard_normal(4)


def gemm_small(seed=BASE_SEED, n=64):
    g = rng(seed)
    A = qmatrix(g, n, n, dist="normal")
    B = qmatrix(g, n, n, dist="normal")
    C = np.zeros((n, n, 4))
    return dict(opA="N", opB="N", M=n, N=n, K=n, alpha=np.array([1.0, 0, 0, 0]),
                beta=np.zeros(4), A=A, lda=n, B=B, ldb=n, C=C, ldc=n)


def gemm_problem(seed, M, N, K, opA="N", opB="N", dist="uniform", dtype=np.float64,
                 alpha=None, beta=None, pad=0):
    """One problem with random quaternion alpha/beta (components U[-1,1]) unless
    given.  ``pad`` extra rows are added to every leading dimension."""
    g = rng(seed)
    ra, ca = stored_dims(opA, M, K)
    rb, cb = stored_dims(opB, K, N)
    lda, ldb, ldc = max(ra, 1) + pad, max(rb, 1) + pad, max(M, 1) + pad
    A = qmatrix(g, ra, ca, ld=lda, dist=dist, dtype=dtype)
    B = qmatrix(g, rb, cb, ld=ldb, dist=dist, dtype=dtype)
    C = qmatrix(g, M, N, ld=ldc, dist=dist, dtype=dtype)
    al = quaternion(g) if alpha is None else np.asarray(alpha, dtype=np.float64)
    be = quaternion(g) if beta is None else np.asarray(beta, dtype=np.float64)
    return dict(opA=opA, opB=opB, M=M, N=N, K=K, alpha=al, beta=be, A=A, lda=lda,
                B=B, ldb=ldb, C=C, ldc=ldc)


def trmm_problem(seed, side, uplo, trans, diag, M, N, dist="uniform", dtype=np.float64, alpha=None, pad=0):
    """Triangular multiply inputs: a stored n x n A (n = M for side 'L', N for
    side 'R') whose triangle opposite to ``uplo`` holds NaN, as does its
    diagonal when ``diag`` is 'U' (those entries must not be read), B and an
    all-NaN C (written, never read), each leading dimension padded by ``pad``."""
    g = rng(seed)
    n = M if side == "L" else N
    lda, ldb, ldc = max(n, 1) + pad, max(M, 1) + pad, max(M, 1) + pad
    A = qmatrix(g, n, n, ld=lda, dist=dist, dtype=dtype)
    r = np.arange(n)
    unread = (r[None, :] < r[:, None]) if uplo == "L" else (r[None, :] > r[:, None])   # [col, row]
    if diag == "U":
        unread = unread | (r[None, :] == r[:, None])
    A[:, :n, :][unread] = np.nan
    B = qmatrix(g, M, N, ld=ldb, dist=dist, dtype=dtype)
    C = np.full((max(N, 0), ldc, 4), np.nan, dtype=dtype)
    al = quaternion(g) if alpha is None else np.asarray(alpha, dtype=np.float64)
    return dict(side=side, uplo=uplo, trans=trans, diag=diag, M=M, N=N, alpha=al, A=A, lda=lda, B=B, ldb=ldb,
                C=C, ldc=ldc)


def typed_matrix(g, kind, rows, cols, ld=None, dist="uniform", dtype=np.float64):
    """Random matrix of element kind 'R' (real, storage (cols, ld)), 'Z'
    (complex as interleaved (re, im), storage (cols, ld, 2)) or 'Q'
    (quaternion, storage (cols, ld, 4)); padding rows hold NaN."""
    width = {"R": 1, "Z": 2, "Q": 4}[kind]
    ld = max(rows, 1) if ld is None else ld
    v = g.uniform(-1.0, 1.0, (cols, rows, width)) if dist == "uniform" else g.standard_normal((cols, rows, width))
    out = np.full((cols, ld, width), np.nan, dtype=dtype)
    out[:, :rows, :] = v.astype(dtype)
    return out[..., 0] if kind == "R" else out


def mixed_problem(seed, typeA, typeB, M, N, K, opA="N", opB="N", dist="uniform", pad=0):
    """Mixed-type GEMM inputs: A of kind typeA, B of kind typeB (see
    typed_matrix), quaternion C and random quaternion alpha, beta."""
    g = rng(seed)
    ra, ca = stored_dims(opA, M, K)
    rb, cb = stored_dims(opB, K, N)
    lda, ldb, ldc = max(ra, 1) + pad, max(rb, 1) + pad, max(M, 1) + pad
    A = typed_matrix(g, typeA, ra, ca, ld=lda, dist=dist)
    B = typed_matrix(g, typeB, rb, cb, ld=ldb, dist=dist)
    C = qmatrix(g, M, N, ld=ldc, dist=dist)
    return dict(typeA=typeA, typeB=typeB, opA=opA, opB=opB, M=M, N=N, K=K, alpha=quaternion(g),
                beta=quaternion(g), A=A, lda=lda, B=B, ldb=ldb, C=C, ldc=ldc)


def qvector(g, n, inc=1, dist="uniform", dtype=np.float64):
    """n quaternions strided by inc elements, storage shape ((n-1) inc + 1, 4);
    the slots between them hold NaN (never read)."""
    length = (n - 1) * inc + 1 if n > 0 else 1
    out = np.full((length, 4), np.nan, dtype=dtype)
    v = g.uniform(-1.0, 1.0, (n, 4)) if dist == "uniform" else g.standard_normal((n, 4))
    out[::inc][:n] = v.astype(dtype)
    return out


SWEEP_SIZES = (1024, 2048, 4096, 8192)
OP_PAIRS = tuple((a, b) for a in "NTC" for b in "NTC")


def gemm_sweep(n, opA, opB):
    idx = SWEEP_SIZES.index(n) * len(OP_PAIRS) + OP_PAIRS.index((opA, opB)) if n in SWEEP_SIZES else 0
    return gemm_problem(BASE_SEED + 1000 + idx, n, n, n, opA, opB, dist="uniform")


def gemm_precision(n=4096, scaled=False, seed=BASE_SEED + 2):
    """FP32 op N/C; with ``scaled`` the rows of op(A) (M index) and the K index
    of op(B) are multiplied by independent factors 10^U[-3,3]."""
    g = rng(seed + (1 if scaled else 0))
    M = N = K = n
    A = qmatrix(g, M, K, dist="normal", dtype=np.float64)     # op N: stored M x K
    B = qmatrix(g, N, K, dist="normal", dtype=np.float64)     # op C: stored N x K
    if scaled:
        ra = 10.0 ** g.uniform(-3.0, 3.0, M)
        rk = 10.0 ** g.uniform(-3.0, 3.0, K)
        A = A * ra[None, :, None]
        B = B * rk[:, None, None]      # K index of op(B) = stored column of B
    C = np.zeros((N, M, 4), dtype=np.float32)
    return dict(opA="N", opB="C", M=M, N=N, K=K, alpha=np.array([1.0, 0, 0, 0]),
                beta=np.zeros(4), A=A.astype(np.float32), lda=M, B=B.astype(np.float32), ldb=N,
                C=C, ldc=M)


def grouped_sizes(count=4096, lo=8, hi=512, seed=BASE_SEED + 3):
    g = rng(seed)
    mnk = np.rint(np.exp(g.uniform(np.log(lo), np.log(hi), (count, 3)))).astype(np.int64)
    return mnk


def grouped(count=4096, lo=8, hi=512, seed=BASE_SEED + 3, dtype=np.float32):
    """List of problems (op N/N, alpha = 1, beta = 0.5 real), own buffers each."""
    mnk = grouped_sizes(count, lo, hi, seed)
    g = rng(seed + 17)
    probs = []
    for (M, N, K) in mnk:
        M, N, K = int(M), int(N), int(K)
        A = qmatrix(g, M, K, dist="uniform", dtype=dtype)
        B = qmatrix(g, K, N, dist="uniform", dtype=dtype)
        C = qmatrix(g, M, N, dist="uniform", dtype=dtype)
        probs.append(dict(M=M, N=N, K=K, A=A, lda=M, B=B, ldb=K, C=C, ldc=M))
    return dict(opA="N", opB="N", alpha=np.array([1.0, 0, 0, 0]), beta=np.array([0.5, 0, 0, 0]),
                problems=probs)


def linear_layer(rows=8192, fan_in=1024, fan_out=1024, seed=BASE_SEED + 4, dtype=np.float32):
    """Y = X W with X rows x fan_in, W fan_in x fan_out; Glorot sigma from the
    real 4x4-embedding fans (4*fan_in, 4*fan_out)."""
    g = rng(seed)
    sigma = np.sqrt(2.0 / (4 * fan_in + 4 * fan_out))
    X = qmatrix(g, rows, fan_in, dist="normal", dtype=dtype)
    W = qmatrix(g, fan_in, fan_out, dist="normal", dtype=dtype, sigma=sigma)
    dY = qmatrix(g, rows, fan_out, dist="normal", dtype=dtype)
    return dict(M=rows, K=fan_in, N=fan_out, X=X, W=W, dY=dY, sigma=sigma)
