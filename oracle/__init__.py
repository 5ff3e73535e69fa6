"""CPU FP64 oracle for quaternion GEMM -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path never does, and this package never
imports the product package.  The arithmetic lives in ``qgemm_oracle.c``
(plain C, binary64, OpenMP over output columns); this module only marshals
numpy buffers through ctypes.

Storage convention shared with the tests: a quaternion matrix with ``rows``
rows, ``cols`` columns and leading dimension ``ld`` is a float64 numpy array of
shape ``(cols, ld, 4)``: column-major, four interleaved components per element
(Sec. 4 storage; Sec. 3.1 column-major).  Element (mu, nu) component c is
``X[nu, mu, c]``.

op codes: 'N' as stored, 'T' transpose, 'C' conjugate transpose (the paper's
^H), 'R' conjugate without transpose.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qgemm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
OPS = {"N": 0, "T": 1, "C": 2, "R": 3}


def build(force=True):
    """Compile the oracle with gcc (no GPU toolchain involved)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99", "-Wall",
           "-o", _LIB_PATH + ".tmp", _SRC]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        L.oracle_hamilton.argtypes = [dp, dp, dp]
        L.oracle_hamilton.restype = None
        L.oracle_qgemm.argtypes = [ctypes.c_int, ctypes.c_int, i64, i64, i64,
                                   dp, dp, i64, dp, i64, dp, dp, i64]
        L.oracle_qgemm.restype = ctypes.c_int
        L.oracle_qgemm_backward.argtypes = [ctypes.c_int, ctypes.c_int, i64, i64, i64,
                                            dp, dp, i64, dp, i64, dp, i64, dp,
                                            dp, i64, dp, i64, dp, i64]
        L.oracle_qgemm_backward.restype = ctypes.c_int
        L.oracle_qgemm_ex.argtypes = [ctypes.c_int, ctypes.c_int, i64, i64, i64, dp, dp, dp,
                                      dp, i64, dp, i64, dp, dp, dp, i64]
        L.oracle_qgemm_ex.restype = ctypes.c_int
        L.oracle_qherk.argtypes = [ctypes.c_int, ctypes.c_int, i64, i64, ctypes.c_double, dp, i64,
                                   ctypes.c_double, dp, i64]
        L.oracle_qherk.restype = ctypes.c_int
        L.oracle_qtrmm.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, i64, i64, dp,
                                   dp, i64, dp, i64, dp, i64]
        L.oracle_qtrmm.restype = ctypes.c_int
        L.oracle_qgemm_mixed.argtypes = [ctypes.c_int] * 4 + [i64, i64, i64, dp, dp, i64, dp, i64, dp, dp, i64]
        L.oracle_qgemm_mixed.restype = ctypes.c_int
        L.oracle_qaxpy.argtypes = [i64, dp, dp, i64, dp, i64]
        L.oracle_qaxpy.restype = ctypes.c_int
        L.oracle_qdot.argtypes = [ctypes.c_int, i64, dp, i64, dp, i64, dp]
        L.oracle_qdot.restype = ctypes.c_int
        L.oracle_qgemv.argtypes = [ctypes.c_int, i64, i64, dp, dp, i64, dp, i64, dp, dp, i64]
        L.oracle_qgemv.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def set_threads(n):
    lib().oracle_set_threads(int(n))


def max_threads():
    return int(lib().oracle_max_threads())


def hamilton(p, q):
    """Hamilton product p q of two 4-vectors (Eq. quaternion_prod)."""
    p, q = _f64(p), _f64(q)
    out = np.zeros(4)
    lib().oracle_hamilton(_ptr(p), _ptr(q), _ptr(out))
    return out


def stored_shape(op, rows, cols):
    """(rows, cols) of the stored matrix whose op() is rows x cols."""
    return (rows, cols) if op in ("N", "R") else (cols, rows)


def qgemm(opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc):
    """Return alpha*op(A)*op(B) + beta*C as a new (N, ldc, 4) array.

    A, B, C are storage arrays (see module docstring); C is not modified.
    FP32 inputs are widened exactly to FP64."""
    A, B = _f64(A), _f64(B)
    out = _f64(C).copy()
    rc = lib().oracle_qgemm(OPS[opA], OPS[opB], M, N, K, _ptr(_f64(alpha)), _ptr(A), lda,
                            _ptr(B), ldb, _ptr(_f64(beta)), _ptr(out), ldc)
    if rc != 0:
        raise RuntimeError(f"oracle_qgemm failed ({rc})")
    return out


def qgemm_ex(opA, opB, M, N, K, aL, aM, aR, A, lda, B, ldb, bL, bR, C, ldc):
    """Return aL (sum op(A) aM op(B)) aR + bL C bR as a new (N, ldc, 4) array
    (general scalar placement); a scalar given as None is the default (unit,
    or zero for bL)."""
    A, B = _f64(A), _f64(B)
    out = _f64(C).copy()
    q = [None if x is None else _f64(x) for x in (aL, aM, aR, bL, bR)]
    rc = lib().oracle_qgemm_ex(OPS[opA], OPS[opB], M, N, K, *[_ptr(x) for x in q[:3]], _ptr(A), lda,
                               _ptr(B), ldb, _ptr(q[3]), _ptr(q[4]), _ptr(out), ldc)
    if rc != 0:
        raise RuntimeError(f"oracle_qgemm_ex failed ({rc})")
    return out


def qherk(uplo, trans, n, k, alpha, A, lda, beta, C, ldc):
    """Hermitian rank-k update on the triangle uplo ('L' or 'U') of C:
    alpha op(A) op(A)^H + beta C with op = trans ('N' or 'C'), alpha and beta
    real.  Returns a new (n, ldc, 4) array."""
    A = _f64(A)
    out = _f64(C).copy()
    rc = lib().oracle_qherk({"L": 0, "U": 1}[uplo], OPS[trans], n, k, float(alpha), _ptr(A), lda,
                            float(beta), _ptr(out), ldc)
    if rc != 0:
        raise RuntimeError(f"oracle_qherk failed ({rc})")
    return out


def qtrmm(side, uplo, trans, diag, M, N, alpha, A, lda, B, ldb, C, ldc):
    """Triangular multiply alpha op(T) B (side 'L') or alpha B op(T) (side
    'R'), T the triangle uplo ('L'/'U') of A with unit diagonal when diag is
    'U'.  C only supplies the shape (N, ldc, 4) and the padding of the
    result, which is returned as a new array."""
    A = _f64(A)
    B = _f64(B)
    out = _f64(C).copy()
    rc = lib().oracle_qtrmm({"L": 0, "R": 1}[side], {"L": 0, "U": 1}[uplo], OPS[trans], {"N": 0, "U": 1}[diag],
                            M, N, _ptr(_f64(alpha)), _ptr(A), lda, _ptr(B), ldb,
                            _ptr(out), ldc)
    if rc != 0:
        raise RuntimeError(f"oracle_qtrmm failed ({rc})")
    return out


TYPES = {"R": 1, "Z": 2, "Q": 4}


def qgemm_mixed(typeA, typeB, opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc):
    """Mixed-type GEMM: typeA/typeB in 'R' (real, shape (cols, ld)), 'Z'
    (complex, (cols, ld, 2)), 'Q' (quaternion, (cols, ld, 4)); the result is
    a new quaternion (N, ldc, 4) array."""
    A, B = _f64(A), _f64(B)
    out = _f64(C).copy()
    rc = lib().oracle_qgemm_mixed(TYPES[typeA], TYPES[typeB], OPS[opA], OPS[opB], M, N, K, _ptr(_f64(alpha)),
                                  _ptr(A), lda, _ptr(B), ldb, _ptr(_f64(beta)), _ptr(out), ldc)
    if rc != 0:
        raise RuntimeError(f"oracle_qgemm_mixed failed ({rc})")
    return out


def qaxpy(n, alpha, x, incx, y, incy):
    """alpha x + y over n strided quaternions; x, y are (len, 4) arrays.  Returns a new y."""
    x = _f64(x)
    out = _f64(y).copy()
    if lib().oracle_qaxpy(n, _ptr(_f64(alpha)), _ptr(x), incx, _ptr(out), incy) != 0:
        raise RuntimeError("oracle_qaxpy failed")
    return out


def qdot(conj, n, x, incx, y, incy):
    """sum x_i y_i (conj: sum conj(x_i) y_i) as a length-4 array."""
    r = np.zeros(4)
    if lib().oracle_qdot(int(bool(conj)), n, _ptr(_f64(x)), incx, _ptr(_f64(y)), incy, _ptr(r)) != 0:
        raise RuntimeError("oracle_qdot failed")
    return r


def qgemv(trans, M, N, alpha, A, lda, x, incx, beta, y, incy):
    """alpha op(A) x + beta y with A stored M x N; returns a new y."""
    out = _f64(y).copy()
    if lib().oracle_qgemv(OPS[trans], M, N, _ptr(_f64(alpha)), _ptr(_f64(A)), lda, _ptr(_f64(x)), incx,
                          _ptr(_f64(beta)), _ptr(out), incy) != 0:
        raise RuntimeError("oracle_qgemv failed")
    return out


def qgemm_backward(opA, opB, M, N, K, alpha, A, lda, B, ldb, G, ldg, beta,
                   want_dA=True, want_dB=True, want_dC0=True):
    """Gradients (dA, dB, dC0) of <G, alpha*op(A)*op(B) + beta*C0>, each in the
    stored layout of its operand with the smallest leading dimension."""
    A, B, G = _f64(A), _f64(B), _f64(G)
    ra, ca = stored_shape(opA, M, K)
    rb, cb = stored_shape(opB, K, N)
    dA = np.zeros((ca, max(ra, 1), 4)) if want_dA else None
    dB = np.zeros((cb, max(rb, 1), 4)) if want_dB else None
    dC0 = np.zeros((N, max(M, 1), 4)) if want_dC0 else None
    rc = lib().oracle_qgemm_backward(OPS[opA], OPS[opB], M, N, K, _ptr(_f64(alpha)), _ptr(A), lda,
                                     _ptr(B), ldb, _ptr(G), ldg, _ptr(_f64(beta)),
                                     _ptr(dA), max(ra, 1), _ptr(dB), max(rb, 1), _ptr(dC0), max(M, 1))
    if rc != 0:
        raise RuntimeError(f"oracle_qgemm_backward failed ({rc})")
    return dA, dB, dC0


def qgemm_entries(opA, opB, K, alpha, A, B, beta, C, rows, cols):
    """Oracle values of selected output rows x cols of alpha*op(A)*op(B)+beta*C.

    A, B, C are full storage arrays; only the needed slices are passed to the C
    routine (pure index selection, no arithmetic here).  Returns an array of
    shape (len(cols), len(rows), 4)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    # rows of op(A): columns of the stored A for N/R, stored rows otherwise
    As = A[:, rows, :] if opA in ("N", "R") else A[rows, :, :]
    Bs = B[cols, :, :] if opB in ("N", "R") else B[:, cols, :]
    Cs = C[cols][:, rows, :]
    As, Bs, Cs = _f64(As), _f64(Bs), _f64(Cs)
    m, n = len(rows), len(cols)
    return qgemm(opA, opB, m, n, K, alpha, As, As.shape[1], Bs, Bs.shape[1], beta, Cs, Cs.shape[1])
