"""ctypes binding of libqgemm.so (argument marshalling only).

Every step of the computation runs in the HIP kernels behind the C ABI
declared in include/qgemm.h; this module converts Python arguments to the
C types, checks that tensors are large enough for the sizes passed, and turns
status codes into exceptions.  There is no fallback: if the library is
missing or cannot be loaded, every call raises.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqgemm.so")

OPS = {"N": 0, "T": 1, "C": 2, "R": 3}
STATUS = {0: "QGEMM_OK", 1: "QGEMM_ERR_INVALID_ARG", 2: "QGEMM_ERR_MISALIGNED", 3: "QGEMM_ERR_HIP",
          4: "QGEMM_ERR_ALLOC", 5: "QGEMM_ERR_UNSUPPORTED"}


class QGemmError(RuntimeError):
    def __init__(self, status, arg, where):
        self.status = status
        self.arg = arg
        super().__init__(f"{where}: {STATUS.get(status, status)} (argument {arg})")


_lib = None

_i64 = ctypes.c_int64
_int = ctypes.c_int
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)

class Problem(ctypes.Structure):
    """Mirror of qgemm_problem_t (include/qgemm.h)."""
    _fields_ = [("M", ctypes.c_int64), ("N", ctypes.c_int64), ("K", ctypes.c_int64),
                ("lda", ctypes.c_int64), ("ldb", ctypes.c_int64), ("ldc", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("B", ctypes.c_void_p), ("C", ctypes.c_void_p)]


_SIGNATURES = {
    "qgemm_status_string": ([_int], ctypes.c_char_p),
    "qgemm_last_invalid_arg": ([], _int),
    "qgemm_d": ([_int, _int, _i64, _i64, _i64, _dp, _vp, _i64, _vp, _i64, _dp, _vp, _i64, _vp], _int),
    "qgemm_s": ([_int, _int, _i64, _i64, _i64, _dp, _vp, _i64, _vp, _i64, _dp, _vp, _i64, _int, _vp], _int),
    "qgemm_s_c64": ([_int, _int, _i64, _i64, _i64, _dp, _vp, _i64, _vp, _i64, _dp, _vp, _i64, _int, _vp], _int),
    "qgemm_ex_d": ([_int, _int, _i64, _i64, _i64, _dp, _dp, _dp, _vp, _i64, _vp, _i64, _dp, _dp, _vp, _i64,
                    _vp], _int),
    "qgemm_ex_s": ([_int, _int, _i64, _i64, _i64, _dp, _dp, _dp, _vp, _i64, _vp, _i64, _dp, _dp, _vp, _i64,
                    _int, _vp], _int),
    "qherk_d": ([_int, _int, _i64, _i64, ctypes.c_double, _vp, _i64, ctypes.c_double, _vp, _i64, _vp], _int),
    "qherk_s": ([_int, _int, _i64, _i64, ctypes.c_double, _vp, _i64, ctypes.c_double, _vp, _i64, _int, _vp], _int),
    "qtrmm_d": ([_int, _int, _int, _int, _i64, _i64, _dp, _vp, _i64, _vp, _i64, _vp, _i64, _vp], _int),
    "qtrmm_s": ([_int, _int, _int, _int, _i64, _i64, _dp, _vp, _i64, _vp, _i64, _vp, _i64, _int, _vp], _int),
    "qgemm_mixed_d": ([_int, _int, _int, _int, _i64, _i64, _i64, _dp, _vp, _i64, _vp, _i64, _dp, _vp, _i64, _vp],
                      _int),
    "qgemm_mixed_s": ([_int, _int, _int, _int, _i64, _i64, _i64, _dp, _vp, _i64, _vp, _i64, _dp, _vp, _i64, _vp],
                      _int),
    "qaxpy_d": ([_i64, _dp, _vp, _i64, _vp, _i64, _vp], _int),
    "qaxpy_s": ([_i64, _dp, _vp, _i64, _vp, _i64, _vp], _int),
    "qdot_d": ([_int, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _vp], _int),
    "qdot_s": ([_int, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _vp], _int),
    "qdot_d_noalloc": ([_int, _i64, _vp, _i64, _vp, _i64, _vp, _vp], _int),
    "qgemv_d": ([_int, _i64, _i64, _dp, _vp, _i64, _vp, _i64, _dp, _vp, _i64, _vp], _int),
    "qgemv_s": ([_int, _i64, _i64, _dp, _vp, _i64, _vp, _i64, _dp, _vp, _i64, _vp], _int),
    "qgemm_batched_plan_create": ([ctypes.POINTER(_vp), _int, _int, _int, _i64, ctypes.POINTER(Problem), _dp,
                                   _dp, _int, _int], _int),
    "qgemm_batched_run": ([_vp, _vp], _int),
    "qgemm_batched_plan_destroy": ([_vp], _int),
    "qgemm_batched_plan_info": ([_vp, ctypes.POINTER(_i64), ctypes.POINTER(_int), ctypes.POINTER(_i64)], _int),
    "qgemm_last_invalid_problem": ([], _i64),
    "qgemm_batched_set_tile_table": ([_vp], _int),
    "qgemm_batched_get_tile_table": ([_vp], _int),
    "qgemm_backward_d": ([_int, _int, _i64, _i64, _i64, _dp, _vp, _i64, _vp, _i64, _vp, _i64, _dp,
                          _vp, _i64, _vp, _i64, _vp, _i64, _vp], _int),
    "qgemm_backward_s": ([_int, _int, _i64, _i64, _i64, _dp, _vp, _i64, _vp, _i64, _vp, _i64, _dp,
                          _vp, _i64, _vp, _i64, _vp, _i64, _int, _vp], _int),
}


def lib():
    """Load libqgemm.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1903_05575_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGNATURES)


def _q4(x):
    a = (ctypes.c_double * 4)(*[float(v) for v in x])
    return ctypes.cast(a, _dp), a


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _check_storage(t, rows, cols, ld, dtype, name, width=4):
    """A stored rows x cols operand needs (cols-1)*ld + rows elements of
    `width` reals (4 for a quaternion)."""
    if rows == 0 or cols == 0:
        return
    if t is None:
        raise ValueError(f"{name} is None")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    need = width * ((cols - 1) * ld + rows)
    if t.numel() < need:
        raise ValueError(f"{name} holds {t.numel()} reals, needs {need}")


def _stored(op, rows, cols):
    return (rows, cols) if op in ("N", "R") else (cols, rows)


def _raise(rc, where):
    if rc != 0:
        raise QGemmError(rc, lib().qgemm_last_invalid_arg(), where)


def qgemm_d(opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream=None):
    """C <- alpha op(A) op(B) + beta C in binary64 (C-ABI qgemm_d).
    A, B, C are float64 GPU tensors in column-major interleaved storage."""
    ra, ca = _stored(opA, M, K)
    rb, cb = _stored(opB, K, N)
    if M and N and K:
        _check_storage(A, ra, ca, lda, torch.float64, "A")
        _check_storage(B, rb, cb, ldb, torch.float64, "B")
    _check_storage(C, M, N, ldc, torch.float64, "C")
    pa, _ka = _q4(alpha)
    pb, _kb = _q4(beta)
    rc = lib().qgemm_d(OPS[opA], OPS[opB], M, N, K, pa, _ptr(A), lda, _ptr(B), ldb, pb, _ptr(C), ldc,
                       _stream(stream))
    _raise(rc, "qgemm_d")


def qgemm_s(opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, split_terms=6, stream=None):
    """C <- alpha op(A) op(B) + beta C for FP32 storage, computed as split-BF16
    products (split_terms in {3, 6, 9}) on the BF16 matrix cores with FP32
    accumulation (C-ABI qgemm_s).  If C is float64 the result and the beta
    term are formed in FP64 (C-ABI qgemm_s_c64)."""
    ra, ca = _stored(opA, M, K)
    rb, cb = _stored(opB, K, N)
    if M and N and K:
        _check_storage(A, ra, ca, lda, torch.float32, "A")
        _check_storage(B, rb, cb, ldb, torch.float32, "B")
    c64 = C is not None and C.dtype == torch.float64
    _check_storage(C, M, N, ldc, torch.float64 if c64 else torch.float32, "C")
    pa, _ka = _q4(alpha)
    pb, _kb = _q4(beta)
    fn = lib().qgemm_s_c64 if c64 else lib().qgemm_s
    rc = fn(OPS[opA], OPS[opB], M, N, K, pa, _ptr(A), lda, _ptr(B), ldb, pb, _ptr(C), ldc, int(split_terms),
            _stream(stream))
    _raise(rc, "qgemm_s_c64" if c64 else "qgemm_s")


def qgemm_backward(opA, opB, M, N, K, alpha, A, lda, B, ldb, G, ldg, beta,
                   dA=None, ldda=1, dB=None, lddb=1, dC0=None, lddc0=1, split_terms=6, stream=None):
    """Gradients of <G, alpha op(A) op(B) + beta C0> with respect to the stored
    A, B and C0, written (overwritten) into dA, dB, dC0 when given (C-ABI
    qgemm_backward_d for float64 tensors, qgemm_backward_s for float32)."""
    dtype = G.dtype
    ra, ca = _stored(opA, M, K)
    rb, cb = _stored(opB, K, N)
    _check_storage(G, M, N, ldg, dtype, "G")
    if dB is not None:
        _check_storage(A, ra, ca, lda, dtype, "A")
        _check_storage(dB, rb, cb, lddb, dtype, "dB")
    if dA is not None:
        _check_storage(B, rb, cb, ldb, dtype, "B")
        _check_storage(dA, ra, ca, ldda, dtype, "dA")
    if dC0 is not None:
        _check_storage(dC0, M, N, lddc0, dtype, "dC0")
    pa, _ka = _q4(alpha)
    pb, _kb = _q4(beta)
    args = [OPS[opA], OPS[opB], M, N, K, pa, _ptr(A), lda, _ptr(B), ldb, _ptr(G), ldg, pb,
            _ptr(dA), ldda, _ptr(dB), lddb, _ptr(dC0), lddc0]
    if dtype == torch.float64:
        rc = lib().qgemm_backward_d(*args, _stream(stream))
        _raise(rc, "qgemm_backward_d")
    elif dtype == torch.float32:
        rc = lib().qgemm_backward_s(*args, int(split_terms), _stream(stream))
        _raise(rc, "qgemm_backward_s")
    else:
        raise ValueError(f"unsupported dtype {dtype}")


TILE_CLASSES = ((32, 64), (64, 32), (32, 32), (16, 64))
DTYPES = {torch.float32: 0, torch.float64: 1}    # QGEMM_DTYPE_F32 / QGEMM_DTYPE_F64


def tile_table():
    """The tile table of FP32 grouped plans in effect, as a list of 32 classes
    indexed [M bucket][N bucket][K bucket] (C-ABI qgemm_batched_get_tile_table)."""
    buf = (ctypes.c_ubyte * 32)()
    _raise(lib().qgemm_batched_get_tile_table(ctypes.cast(buf, _vp)), "qgemm_batched_get_tile_table")
    return list(buf)


def set_tile_table(table):
    """Install a tile table for plans created afterwards (32 classes, or None
    for the compiled-in table; C-ABI qgemm_batched_set_tile_table)."""
    if table is None:
        _raise(lib().qgemm_batched_set_tile_table(None), "qgemm_batched_set_tile_table")
        return
    table = list(table)
    if len(table) != 32:
        raise ValueError("a tile table has 32 entries")
    buf = (ctypes.c_ubyte * 32)(*table)
    _raise(lib().qgemm_batched_set_tile_table(ctypes.cast(buf, _vp)), "qgemm_batched_set_tile_table")


class GroupedPlan:
    """A grouped (batched) quaternion GEMM plan (C-ABI
    qgemm_batched_plan_create / _run / _plan_destroy).

    problems: sequence of dicts with GPU tensors A, B, C of `dtype` (float32:
    split-BF16 path; float64: FP64 path) and the ints M, N, K, lda, ldb, ldc.
    The tensors must outlive the plan; the plan keeps references to them.
    run() enqueues one persistent launch on the current (or given) stream and
    may be captured in a CUDA/HIP graph.  split_terms applies to float32
    plans only."""

    def __init__(self, problems, opA="N", opB="N", alpha=(1, 0, 0, 0), beta=(0, 0, 0, 0), split_terms=6,
                 tile_class=-1, dtype=torch.float32):
        self._handle = None
        self._keep = []
        if dtype not in DTYPES:
            raise ValueError(f"unsupported dtype {dtype}")
        if dtype == torch.float64:
            split_terms = 0
        arr = (Problem * max(1, len(problems)))()
        for i, pr in enumerate(problems):
            M, N, K = pr["M"], pr["N"], pr["K"]
            ra, ca = _stored(opA, M, K)
            rb, cb = _stored(opB, K, N)
            if M and N and K:
                _check_storage(pr["A"], ra, ca, pr["lda"], dtype, f"problems[{i}].A")
                _check_storage(pr["B"], rb, cb, pr["ldb"], dtype, f"problems[{i}].B")
            _check_storage(pr["C"], M, N, pr["ldc"], dtype, f"problems[{i}].C")
            arr[i] = Problem(M, N, K, pr["lda"], pr["ldb"], pr["ldc"],
                             pr["A"].data_ptr() if pr.get("A") is not None else None,
                             pr["B"].data_ptr() if pr.get("B") is not None else None,
                             pr["C"].data_ptr() if pr.get("C") is not None else None)
            self._keep.append((pr.get("A"), pr.get("B"), pr.get("C")))
        pa, _ka = _q4(alpha)
        pb, _kb = _q4(beta)
        h = ctypes.c_void_p()
        rc = lib().qgemm_batched_plan_create(ctypes.byref(h), DTYPES[dtype], OPS[opA], OPS[opB], len(problems),
                                             arr, pa, pb, int(split_terms), int(tile_class))
        if rc != 0:
            bad = lib().qgemm_last_invalid_problem()
            raise QGemmError(rc, lib().qgemm_last_invalid_arg(), f"qgemm_batched_plan_create (problem {bad})")
        self._handle = h

    def run(self, stream=None):
        rc = lib().qgemm_batched_run(self._handle, _stream(stream))
        _raise(rc, "qgemm_batched_run")

    def info(self):
        n = ctypes.c_int64()
        g = ctypes.c_int()
        cls = (ctypes.c_int64 * len(TILE_CLASSES))()
        _raise(lib().qgemm_batched_plan_info(self._handle, ctypes.byref(n), ctypes.byref(g), cls),
               "qgemm_batched_plan_info")
        return {"work_items": n.value, "grid": g.value, "tiles_per_class": list(cls)}

    def close(self):
        if self._handle is not None:
            lib().qgemm_batched_plan_destroy(self._handle)
            self._handle = None
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _q4_opt(x):
    if x is None:
        return None, None
    return _q4(x)


def qgemm_ex(opA, opB, M, N, K, alpha_left, alpha_mid, alpha_right, A, lda, B, ldb, beta_left, beta_right,
             C, ldc, split_terms=6, stream=None):
    """C <- aL (sum op(A) aM op(B)) aR + bL C bR (C-ABI qgemm_ex_d for float64
    tensors, qgemm_ex_s for float32).  A scalar given as None takes its default
    (unit; zero for beta_left)."""
    dtype = C.dtype
    ra, ca = _stored(opA, M, K)
    rb, cb = _stored(opB, K, N)
    if M and N and K:
        _check_storage(A, ra, ca, lda, dtype, "A")
        _check_storage(B, rb, cb, ldb, dtype, "B")
    _check_storage(C, M, N, ldc, dtype, "C")
    q = [_q4_opt(x) for x in (alpha_left, alpha_mid, alpha_right, beta_left, beta_right)]
    ptrs = [x[0] for x in q]
    args = [OPS[opA], OPS[opB], M, N, K, ptrs[0], ptrs[1], ptrs[2], _ptr(A), lda, _ptr(B), ldb, ptrs[3], ptrs[4],
            _ptr(C), ldc]
    if dtype == torch.float64:
        rc = lib().qgemm_ex_d(*args, _stream(stream))
        _raise(rc, "qgemm_ex_d")
    elif dtype == torch.float32:
        rc = lib().qgemm_ex_s(*args, int(split_terms), _stream(stream))
        _raise(rc, "qgemm_ex_s")
    else:
        raise ValueError(f"unsupported dtype {dtype}")


def qherk(uplo, trans, N, K, alpha, A, lda, beta, C, ldc, split_terms=6, stream=None):
    """Hermitian rank-k update on the triangle uplo ('L' or 'U') of C:
    alpha op(A) op(A)^H + beta C, op = trans ('N' or 'C'), alpha and beta real
    (C-ABI qherk_d for float64 tensors, qherk_s for float32)."""
    dtype = C.dtype
    rows, cols = (N, K) if trans == "N" else (K, N)
    if N and K:
        _check_storage(A, rows, cols, lda, dtype, "A")
    _check_storage(C, N, N, ldc, dtype, "C")
    args = [{"L": 0, "U": 1}[uplo], OPS[trans], N, K, float(alpha), _ptr(A), lda, float(beta), _ptr(C), ldc]
    if dtype == torch.float64:
        _raise(lib().qherk_d(*args, _stream(stream)), "qherk_d")
    elif dtype == torch.float32:
        _raise(lib().qherk_s(*args, int(split_terms), _stream(stream)), "qherk_s")
    else:
        raise ValueError(f"unsupported dtype {dtype}")


def qtrmm(side, uplo, trans, diag, M, N, alpha, A, lda, B, ldb, C, ldc, split_terms=6, stream=None):
    """Triangular multiply C <- alpha op(T) B (side 'L') or alpha B op(T)
    (side 'R'), T the triangle uplo ('L'/'U') of A, unit diagonal when diag
    is 'U' (C-ABI qtrmm_d for float64 tensors, qtrmm_s for float32).  C is
    written only and must not overlap A or B."""
    dtype = C.dtype
    n = M if side == "L" else N
    if M and N:
        _check_storage(A, n, n, lda, dtype, "A")
        _check_storage(B, M, N, ldb, dtype, "B")
    _check_storage(C, M, N, ldc, dtype, "C")
    pa, _ka = _q4(alpha)
    args = [{"L": 0, "R": 1}[side], {"L": 0, "U": 1}[uplo], OPS[trans], {"N": 0, "U": 1}[diag], M, N, pa,
            _ptr(A), lda, _ptr(B), ldb, _ptr(C), ldc]
    if dtype == torch.float64:
        _raise(lib().qtrmm_d(*args, _stream(stream)), "qtrmm_d")
    elif dtype == torch.float32:
        _raise(lib().qtrmm_s(*args, int(split_terms), _stream(stream)), "qtrmm_s")
    else:
        raise ValueError(f"unsupported dtype {dtype}")


TYPES = {"R": 1, "Z": 2, "Q": 4}


def qgemm_mixed(typeA, typeB, opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream=None):
    """Mixed-type GEMM (C-ABI qgemm_mixed_d for float64 tensors, qgemm_mixed_s
    for float32): one of A, B real ('R', tensor (cols, ld)) or complex ('Z',
    (cols, ld, 2)), the other quaternion ('Q', (cols, ld, 4)); C quaternion."""
    dtype = C.dtype
    ra, ca = _stored(opA, M, K)
    rb, cb = _stored(opB, K, N)
    if M and N and K:
        _check_storage(A, ra, ca, lda, dtype, "A", TYPES[typeA])
        _check_storage(B, rb, cb, ldb, dtype, "B", TYPES[typeB])
    _check_storage(C, M, N, ldc, dtype, "C")
    pa, _ka = _q4(alpha)
    pb, _kb = _q4(beta)
    name = "qgemm_mixed_" + _suffix(dtype)
    rc = getattr(lib(), name)(TYPES[typeA], TYPES[typeB], OPS[opA], OPS[opB], M, N, K, pa, _ptr(A), lda, _ptr(B), ldb,
                              pb, _ptr(C), ldc, _stream(stream))
    _raise(rc, name)


DOT_WORK_DOUBLES = 4096      # QGEMM_DOT_WORK_DOUBLES of include/qgemm.h


def _check_vector(t, n, inc, dtype, name):
    """n quaternions strided by inc need ((n-1) inc + 1) * 4 reals."""
    if n == 0:
        return
    _check_storage(t, 1, n, inc, dtype, name)


def _suffix(dtype):
    if dtype == torch.float64:
        return "d"
    if dtype == torch.float32:
        return "s"
    raise ValueError(f"unsupported dtype {dtype}")


def qaxpy(n, alpha, x, incx, y, incy, stream=None):
    """y_i <- alpha x_i + y_i over n quaternions (C-ABI qaxpy_d / qaxpy_s)."""
    _check_vector(x, n, incx, y.dtype, "x")
    _check_vector(y, n, incy, y.dtype, "y")
    pa, _ka = _q4(alpha)
    name = "qaxpy_" + _suffix(y.dtype)
    _raise(getattr(lib(), name)(n, pa, _ptr(x), incx, _ptr(y), incy, _stream(stream)), name)


def qdot(n, x, incx, y, incy, conj=False, result=None, work=None, stream=None):
    """sum x_i y_i (conj: sum conj(x_i) y_i) into the device tensor `result`
    (4 reals, allocated when None) through a device workspace `work` of
    DOT_WORK_DOUBLES doubles (allocated when None).  Returns `result`."""
    dtype = x.dtype if x is not None else torch.float64
    _check_vector(x, n, incx, dtype, "x")
    _check_vector(y, n, incy, dtype, "y")
    if result is None:
        result = torch.empty(4, dtype=dtype, device="cuda")
    if work is None and n > 0:
        work = torch.empty(DOT_WORK_DOUBLES, dtype=torch.float64, device="cuda")
    if work is not None and (work.dtype != torch.float64 or work.numel() < DOT_WORK_DOUBLES):
        raise ValueError(f"work must hold {DOT_WORK_DOUBLES} float64 values")
    name = "qdot_" + _suffix(dtype)
    _raise(getattr(lib(), name)(int(bool(conj)), n, _ptr(x), incx, _ptr(y), incy, _ptr(result), _ptr(work),
                                _stream(stream)), name)
    return result


def qgemv(trans, M, N, alpha, A, lda, x, incx, beta, y, incy, stream=None):
    """y <- alpha op(A) x + beta y, A stored M x N (C-ABI qgemv_d / qgemv_s)."""
    dtype = y.dtype
    tr = trans in ("T", "C")
    nx, ny = (M, N) if tr else (N, M)
    if M and N:
        _check_storage(A, M, N, lda, dtype, "A")
        _check_vector(x, nx, incx, dtype, "x")
        _check_vector(y, ny, incy, dtype, "y")
    pa, _ka = _q4(alpha)
    pb, _kb = _q4(beta)
    name = "qgemv_" + _suffix(dtype)
    _raise(getattr(lib(), name)(OPS[trans], M, N, pa, _ptr(A), lda, _ptr(x), incx, pb, _ptr(y), incy,
                                _stream(stream)), name)
