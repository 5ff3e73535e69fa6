"""Host-only checks of the C ABI (no GPU needed): the library loads, exports
every symbol of include/qgemm.h, and its argument validation rejects bad
calls before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "qgemm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(q[a-z]+_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    import paper_1903_05575_amd as q
    return q.lib()


def test_exports_all_declared(L):
    syms = header_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(L, s), s
    import paper_1903_05575_amd._lib as lb
    assert set(lb.exported_symbols()) == set(syms)


def q4(*v):
    return (ctypes.c_double * 4)(*v)


ONE = q4(1, 0, 0, 0)
FAKE = 0x10000        # aligned, never dereferenced: validation fails first
FAR_A, FAR_B, FAR_C = 1 << 40, 2 << 40, 3 << 40   # disjoint however large the leading dimensions


def call_d(L, opA=0, opB=0, M=4, N=4, K=4, alpha=ONE, A=FAR_A, lda=4, B=FAR_B, ldb=4, beta=ONE, C=FAR_C, ldc=4):
    return L.qgemm_d(opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, None)


@pytest.mark.parametrize("kw,arg,status", [
    (dict(opA=7), 1, 1), (dict(opB=-1), 2, 1), (dict(M=-1), 3, 1), (dict(N=-2), 4, 1), (dict(K=-3), 5, 1),
    (dict(M=1 << 31), 3, 5), (dict(alpha=None), 6, 1), (dict(lda=3), 8, 1), (dict(ldb=3), 10, 1),
    (dict(beta=None), 11, 1), (dict(ldc=3), 13, 1), (dict(A=None), 7, 1), (dict(B=None), 9, 1),
    (dict(C=None), 12, 1), (dict(A=FAR_A + 8), 7, 2), (dict(B=FAR_B + 16), 9, 2), (dict(C=FAR_C + 24), 12, 2),
])
def test_validation_d(L, kw, arg, status):
    rc = call_d(L, **kw)
    assert rc == status
    assert L.qgemm_last_invalid_arg() == arg


def test_transposed_ld_rules(L):
    # op T on A: stored K x M -> lda >= K
    assert call_d(L, opA=1, M=8, K=5, lda=4) == 1 and L.qgemm_last_invalid_arg() == 8
    # op C on B: stored N x K -> ldb >= N
    assert call_d(L, opB=2, N=9, K=4, ldb=8) == 1 and L.qgemm_last_invalid_arg() == 10
    # op T on A with lda = K is valid (N = 0: nothing is launched)
    assert call_d(L, opA=1, M=8, K=4, lda=4, ldc=8, N=0) == 0
    # K == 0 or alpha == 0: A and B may be NULL
    assert call_d(L, K=0, A=None, B=None, N=0) == 0
    assert call_d(L, alpha=q4(0, 0, 0, 0), A=None, B=None, N=0) == 0


def test_validation_s_split_terms(L):
    rc = L.qgemm_s(0, 0, 4, 4, 4, ONE, FAKE, 4, FAKE_B, 4, ONE, FAKE_C, 4, 5, None)
    assert rc == 1 and L.qgemm_last_invalid_arg() == 14
    rc = L.qgemm_s(0, 0, 4, 4, 4, ONE, FAKE + 8, 4, FAKE_B, 4, ONE, FAKE_C, 4, 6, None)
    assert rc == 2 and L.qgemm_last_invalid_arg() == 7


def test_validation_s_c64_alignment(L):
    """qgemm_s_c64 asks 16-byte alignment of its float A and B (as qgemm_s)
    and 32-byte alignment of its double C: a sub-matrix view of A or B offset
    by one float quaternion is accepted (the call then stops at the bad
    split_terms, argument 14); C offset by 16 bytes is refused."""
    for fn in (L.qgemm_s, L.qgemm_s_c64):
        rc = fn(0, 0, 4, 4, 4, ONE, FAKE + 16, 4, FAKE_B + 16, 4, ONE, FAKE_C, 4, 5, None)
        assert rc == 1 and L.qgemm_last_invalid_arg() == 14
        rc = fn(0, 0, 4, 4, 4, ONE, FAKE + 8, 4, FAKE_B, 4, ONE, FAKE_C, 4, 6, None)
        assert rc == 2 and L.qgemm_last_invalid_arg() == 7
        rc = fn(0, 0, 4, 4, 4, ONE, FAKE, 4, FAKE_B + 8, 4, ONE, FAKE_C, 4, 6, None)
        assert rc == 2 and L.qgemm_last_invalid_arg() == 9
    rc = L.qgemm_s_c64(0, 0, 4, 4, 4, ONE, FAKE, 4, FAKE_B, 4, ONE, FAKE_C + 16, 4, 6, None)
    assert rc == 2 and L.qgemm_last_invalid_arg() == 12
    rc = L.qgemm_s(0, 0, 4, 4, 4, ONE, FAKE, 4, FAKE_B, 4, ONE, FAKE_C + 16, 4, 5, None)
    assert rc == 1 and L.qgemm_last_invalid_arg() == 14


def test_validation_backward(L):
    rc = L.qgemm_backward_d(0, 0, 4, 4, 4, ONE, FAKE, 4, FAKE, 4, FAKE, 3, ONE, FAKE, 4, FAKE, 4, FAKE, 4, None)
    assert rc == 1 and L.qgemm_last_invalid_arg() == 12
    rc = L.qgemm_backward_s(0, 0, 4, 4, 4, ONE, FAKE, 4, FAKE, 4, FAKE, 4, ONE, FAKE, 4, FAKE, 4, FAKE, 4, 4, None)
    assert rc == 1 and L.qgemm_last_invalid_arg() == 20
    rc = L.qgemm_backward_d(0, 1, 4, 4, 4, ONE, FAKE, 4, FAKE, 4, FAKE, 4, ONE, FAKE, 4, FAKE, 3, None, 0, None)
    assert rc == 1 and L.qgemm_last_invalid_arg() == 17


def test_batched_plan_validation(L):
    import paper_1903_05575_amd._lib as lb
    probs = (lb.Problem * 3)()
    for i in range(3):
        probs[i] = lb.Problem(4, 4, 4, 4, 4, 4, FAKE, FAKE_B, FAKE_C + 4096 * i)
    probs[1].ldb = 2
    h = ctypes.c_void_p()
    rc = L.qgemm_batched_plan_create(ctypes.byref(h), 0, 0, 0, 3, probs, ONE, ONE, 6, -1)
    assert rc == 1 and L.qgemm_last_invalid_arg() == 10 and L.qgemm_last_invalid_problem() == 1
    probs[1].ldb = 4
    probs[2].C = FAKE + 4
    rc = L.qgemm_batched_plan_create(ctypes.byref(h), 0, 0, 0, 3, probs, ONE, ONE, 6, -1)
    assert rc == 2 and L.qgemm_last_invalid_arg() == 12 and L.qgemm_last_invalid_problem() == 2
    rc = L.qgemm_batched_plan_create(ctypes.byref(h), 0, 0, 0, 3, probs, ONE, ONE, 6, 4)   # classes are 0..3
    assert rc == 1 and L.qgemm_last_invalid_arg() == 10
    probs[2].C = FAKE_B + 64                     # C of problem 2 inside its B
    rc = L.qgemm_batched_plan_create(ctypes.byref(h), 0, 0, 0, 3, probs, ONE, ONE, 6, -1)
    assert rc == 1 and L.qgemm_last_invalid_arg() == 12 and L.qgemm_last_invalid_problem() == 2
    assert L.qgemm_batched_run(None, None) == 1
    assert L.qgemm_batched_plan_destroy(None) == 0


def test_batched_plan_dtype_validation(L):
    """dtype is argument 2 (QGEMM_DTYPE_F32 = 0, QGEMM_DTYPE_F64 = 1); FP64
    plans take split_terms 0 and the one tile class 0, and ask FP64 alignment
    (32 bytes) of every array."""
    import paper_1903_05575_amd._lib as lb
    probs = (lb.Problem * 2)()
    for i in range(2):
        probs[i] = lb.Problem(4, 4, 4, 4, 4, 4, FAKE, FAKE_B, FAKE_C + 4096 * i)
    h = ctypes.c_void_p()
    rc = L.qgemm_batched_plan_create(ctypes.byref(h), 2, 0, 0, 2, probs, ONE, ONE, 0, -1)
    assert rc == 1 and L.qgemm_last_invalid_arg() == 2
    rc = L.qgemm_batched_plan_create(ctypes.byref(h), 1, 4, 0, 2, probs, ONE, ONE, 0, -1)
    assert rc == 1 and L.qgemm_last_invalid_arg() == 3
    rc = L.qgemm_batched_plan_create(ctypes.byref(h), 1, 0, 0, 2, probs, ONE, ONE, 6, -1)
    assert rc == 1 and L.qgemm_last_invalid_arg() == 9
    rc = L.qgemm_batched_plan_create(ctypes.byref(h), 1, 0, 0, 2, probs, ONE, ONE, 0, 1)
    assert rc == 1 and L.qgemm_last_invalid_arg() == 10
    probs[1].A = FAKE + 16                       # one float quaternion: misaligned for double
    rc = L.qgemm_batched_plan_create(ctypes.byref(h), 1, 0, 0, 2, probs, ONE, ONE, 0, -1)
    assert rc == 2 and L.qgemm_last_invalid_arg() == 7 and L.qgemm_last_invalid_problem() == 1
    probs[1].A = FAKE
    probs[0].lda = 3                             # M = 4 rows of A under op N
    rc = L.qgemm_batched_plan_create(ctypes.byref(h), 1, 0, 0, 2, probs, ONE, ONE, 0, -1)
    assert rc == 1 and L.qgemm_last_invalid_arg() == 8 and L.qgemm_last_invalid_problem() == 0
    assert h.value is None


def test_tile_table_get_set(L):
    """The FP32 grouped tile table: read back what was installed, refuse an
    entry above 3 (argument 1) without changing the table, restore with NULL."""
    import paper_1903_05575_amd._lib as lb
    built_in = lb.tile_table()
    assert len(built_in) == 32 and all(0 <= c <= 3 for c in built_in)
    custom = [(i * 7) % 4 for i in range(32)]
    lb.set_tile_table(custom)
    assert lb.tile_table() == custom
    bad = (ctypes.c_ubyte * 32)(*([0] * 31 + [4]))
    assert L.qgemm_batched_set_tile_table(ctypes.cast(bad, ctypes.c_void_p)) == 1
    assert L.qgemm_last_invalid_arg() == 1
    assert lb.tile_table() == custom
    lb.set_tile_table(None)
    assert lb.tile_table() == built_in
    assert L.qgemm_batched_get_tile_table(None) == 1


def test_tile_table_header_matches_tuner():
    """tile_table.inc is what the tuner writes: 32 classes in 0..3 and the hash
    of the kernel sources it was tuned on."""
    import re as _re
    txt = open(os.path.join(ROOT, "paper_1903_05575_amd", "csrc", "tile_table.inc")).read()
    body = txt[txt.index("kTileTable"):]
    vals = [int(v) for v in _re.findall(r"\b(\d)\b", body[body.index("=") + 1:])]
    assert len(vals) == 32 and all(0 <= v <= 3 for v in vals)
    assert _re.search(r"kernel_source_sha:\s*[0-9a-f]{16}", txt)


def test_status_strings(L):
    for code, name in [(0, b"QGEMM_OK"), (1, b"QGEMM_ERR_INVALID_ARG"), (2, b"QGEMM_ERR_MISALIGNED"),
                       (3, b"QGEMM_ERR_HIP"), (4, b"QGEMM_ERR_ALLOC"), (5, b"QGEMM_ERR_UNSUPPORTED")]:
        assert L.qgemm_status_string(code) == name
    assert L.qgemm_status_string(99) == b"QGEMM_ERR_UNKNOWN"


def test_python_binding_checks_storage():
    """The binding refuses tensors too small for the sizes passed (host check)."""
    import torch
    import paper_1903_05575_amd as q
    from paper_1903_05575_amd import _lib
    with pytest.raises(ValueError):
        _lib._check_storage(torch.zeros(3, 4, 4), 4, 4, 4, torch.float32, "A")


def test_split_unsupported_leading_dimension(L):
    """The split-BF16 tiles address a K-tile with 32-bit offsets: a transposed
    operand with lda >= 2^21 quaternions is refused as unsupported (host check)."""
    big = 1 << 21
    rc = L.qgemm_s(1, 0, 4, 4, 4, ONE, FAR_A, big, FAR_B, 4, ONE, FAR_C, 4, 6, None)
    assert rc == 5 and L.qgemm_last_invalid_arg() == 8
    rc = L.qgemm_s(0, 0, 4, 4, 4, ONE, FAR_A, 4, FAR_B, big * 4, ONE, FAR_C, 4, 6, None)
    assert rc == 5 and L.qgemm_last_invalid_arg() == 10


def test_f64_unsupported_leading_dimension(L):
    """The FP64 tiles address a K-tile with 32-bit offsets: a transposed A with
    lda >= 2^20 quaternions is refused as unsupported (host check)."""
    rc = call_d(L, opA=1, lda=1 << 20)
    assert rc == 5 and L.qgemm_last_invalid_arg() == 8


def test_validation_ex(L):
    """qgemm_ex_* argument numbering: 9 A, 10 lda, 11 B, 12 ldb, 15 C, 16 ldc, 17 split."""
    n = None
    rc = L.qgemm_ex_d(0, 0, 4, 4, 4, ONE, n, n, FAKE, 3, FAKE, 4, ONE, n, FAKE, 4, n)
    assert rc == 1 and L.qgemm_last_invalid_arg() == 10
    rc = L.qgemm_ex_d(0, 0, 4, 4, 4, n, n, n, FAKE, 4, FAKE, 4, n, n, FAKE + 8, 4, n)
    assert rc == 2 and L.qgemm_last_invalid_arg() == 15
    rc = L.qgemm_ex_d(0, 0, 4, 4, 4, n, n, n, FAKE, 4, FAKE, 4, n, n, FAKE, 2, n)
    assert rc == 1 and L.qgemm_last_invalid_arg() == 16
    rc = L.qgemm_ex_s(0, 0, 4, 4, 4, n, n, n, FAR_A, 4, FAR_B, 4, n, n, FAR_C, 4, 7, n)
    assert rc == 1 and L.qgemm_last_invalid_arg() == 17
    # a zero middle scalar: A and B are not read, so NULL is accepted (N = 0: nothing launched)
    rc = L.qgemm_ex_d(0, 0, 4, 0, 4, n, q4(0, 0, 0, 0), n, None, 4, None, 4, n, n, FAKE, 4, n)
    assert rc == 0


def test_validation_herk(L):
    """qherk_* argument numbering: 1 uplo, 2 trans, 3 N, 4 K, 6 A, 7 lda, 9 C, 10 ldc, 11 split."""
    d = ctypes.c_double
    assert L.qherk_d(2, 0, 4, 4, d(1.0), FAKE, 4, d(0.0), FAKE, 4, None) == 1 and L.qgemm_last_invalid_arg() == 1
    assert L.qherk_d(0, 1, 4, 4, d(1.0), FAKE, 4, d(0.0), FAKE, 4, None) == 1 and L.qgemm_last_invalid_arg() == 2
    assert L.qherk_d(0, 0, 4, 4, d(1.0), FAKE, 3, d(0.0), FAKE, 4, None) == 1 and L.qgemm_last_invalid_arg() == 7
    # trans C: A is K x N, lda >= K
    assert L.qherk_d(0, 2, 8, 4, d(1.0), FAKE, 4, d(0.0), FAKE, 7, None) == 1 and L.qgemm_last_invalid_arg() == 10
    assert L.qherk_d(1, 2, 8, 4, d(1.0), FAKE + 8, 4, d(0.0), FAKE, 8, None) == 2 and L.qgemm_last_invalid_arg() == 6
    assert L.qherk_s(0, 0, 4, 4, d(1.0), FAKE, 4, d(0.0), FAKE, 4, 5, None) == 1 and L.qgemm_last_invalid_arg() == 11
    # alpha == 0 with beta == 1: nothing to do, nothing is read
    assert L.qherk_d(0, 0, 4, 4, d(0.0), None, 4, d(1.0), None, 4, None) == 0


FAKE_B, FAKE_C = 0x20000, 0x30000    # disjoint from FAKE for 4 x 4 operands


def call_trmm(L, side=0, uplo=0, trans=0, diag=0, M=4, N=4, alpha=ONE, A=FAKE, lda=4, B=FAKE_B, ldb=4,
              C=FAKE_C, ldc=4):
    return L.qtrmm_d(side, uplo, trans, diag, M, N, alpha, A, lda, B, ldb, C, ldc, None)


@pytest.mark.parametrize("kw,arg,status", [
    (dict(side=2), 1, 1), (dict(uplo=-1), 2, 1), (dict(trans=4), 3, 1), (dict(diag=2), 4, 1),
    (dict(M=-1), 5, 1), (dict(N=-1), 6, 1), (dict(M=1 << 31), 5, 5), (dict(alpha=None), 7, 1),
    (dict(lda=3), 9, 1), (dict(side=1, N=8, ldc=4, lda=4), 9, 1), (dict(ldb=3), 11, 1), (dict(ldc=3), 13, 1),
    (dict(A=None), 8, 1), (dict(B=None), 10, 1), (dict(C=None), 12, 1),
    (dict(A=FAKE + 8), 8, 2), (dict(B=FAKE_B + 16), 10, 2), (dict(C=FAKE_C + 24), 12, 2),
    (dict(C=FAKE_B), 12, 1), (dict(C=FAKE + 256), 12, 1), (dict(B=FAKE_C + 480), 12, 1),
])
def test_validation_trmm(L, kw, arg, status):
    """qtrmm_* argument numbering: 1 side, 2 uplo, 3 trans, 4 diag, 5 M, 6 N,
    7 alpha, 8 A, 9 lda (>= order of the triangle), 10 B, 11 ldb, 12 C
    (also: C overlapping A or B), 13 ldc, 14 split_terms."""
    assert call_trmm(L, **kw) == status
    assert L.qgemm_last_invalid_arg() == arg


def test_validation_trmm_s_and_quick_return(L):
    assert L.qtrmm_s(0, 0, 0, 0, 4, 4, ONE, FAKE, 4, FAKE_B, 4, FAKE_C, 4, 5, None) == 1
    assert L.qgemm_last_invalid_arg() == 14
    assert L.qtrmm_s(0, 0, 0, 0, 4, 4, ONE, FAKE + 8, 4, FAKE_B, 4, FAKE_C, 4, 6, None) == 2
    assert L.qgemm_last_invalid_arg() == 8
    # empty output: nothing read or written
    assert call_trmm(L, M=0, A=None, B=None, C=None) == 0
    assert call_trmm(L, N=0, A=None, B=None, C=None) == 0


def call_mixed(L, tA=4, tB=1, opA=0, opB=0, M=4, N=4, K=4, alpha=ONE, A=FAKE, lda=4, B=FAKE_B, ldb=4, beta=ONE,
               C=FAKE_C, ldc=4):
    return L.qgemm_mixed_d(tA, tB, opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, None)


@pytest.mark.parametrize("kw,arg,status", [
    (dict(tA=3), 1, 1), (dict(tB=0), 2, 1), (dict(tA=1, tB=2), 2, 1), (dict(opA=5), 3, 1), (dict(opB=-1), 4, 1),
    (dict(M=-1), 5, 1), (dict(K=-1), 7, 1), (dict(alpha=None), 8, 1), (dict(lda=3), 10, 1), (dict(ldb=3), 12, 1),
    (dict(beta=None), 13, 1), (dict(ldc=3), 15, 1), (dict(A=None), 9, 1), (dict(B=None), 11, 1),
    (dict(C=None), 14, 1), (dict(A=FAKE + 8), 9, 2), (dict(tA=2, tB=4, A=FAKE + 8), 9, 2),
    (dict(B=FAKE_B + 4), 11, 2), (dict(C=FAKE_C + 16), 14, 2),
])
def test_validation_mixed(L, kw, arg, status):
    """qgemm_mixed_d numbering: 1 typeA, 2 typeB, then as qgemm_d shifted by two;
    the element of each operand sets its alignment (8, 16, 32 bytes)."""
    assert call_mixed(L, **kw) == status
    assert L.qgemm_last_invalid_arg() == arg


def test_mixed_real_alignment_is_one_double(L):
    # a real B at an 8-byte offset is aligned; the call then fails later on the misaligned quaternion C
    assert call_mixed(L, B=FAKE_B + 8, C=FAKE_C + 8) == 2 and L.qgemm_last_invalid_arg() == 14


def test_validation_level12(L):
    """qaxpy_*: 1 n, 2 alpha, 3 x, 4 incx, 5 y, 6 incy.  qdot_*: 1 conj, 2 n,
    3 x, 4 incx, 5 y, 6 incy, 7 result, 8 work.  qgemv_*: 1 trans, 2 M, 3 N,
    4 alpha, 5 A, 6 lda, 7 x, 8 incx, 9 beta, 10 y, 11 incy."""
    def ax(*a):
        return L.qaxpy_d(*a, None), L.qgemm_last_invalid_arg()
    assert ax(-1, ONE, FAKE, 1, FAKE_B, 1) == (1, 1)
    assert ax(4, None, FAKE, 1, FAKE_B, 1) == (1, 2)
    assert ax(4, ONE, FAKE, 0, FAKE_B, 1) == (1, 4)
    assert ax(4, ONE, FAKE, 1, FAKE_B, -1) == (1, 6)
    assert ax(4, ONE, None, 1, FAKE_B, 1) == (1, 3)
    assert ax(4, ONE, FAKE, 1, None, 1) == (1, 5)
    assert ax(4, ONE, FAKE + 16, 1, FAKE_B, 1) == (2, 3)
    assert ax(4, ONE, FAKE, 2, FAKE + 32, 2) == (1, 5)            # interleaved x and y overlap
    assert ax(0, ONE, None, 1, None, 1) == (0, 0)                 # nothing to do
    assert ax(4, q4(0, 0, 0, 0), None, 1, None, 1) == (0, 0)      # alpha = 0: y untouched
    assert L.qaxpy_s(4, ONE, FAKE + 8, 1, FAKE_B, 1, None) == 2 and L.qgemm_last_invalid_arg() == 3

    def dot(*a):
        return L.qdot_d(*a, None), L.qgemm_last_invalid_arg()
    assert dot(2, 4, FAKE, 1, FAKE_B, 1, FAKE_C, 0x40000) == (1, 1)
    assert dot(0, -4, FAKE, 1, FAKE_B, 1, FAKE_C, 0x40000) == (1, 2)
    assert dot(0, 4, FAKE, 0, FAKE_B, 1, FAKE_C, 0x40000) == (1, 4)
    assert dot(0, 4, FAKE, 1, FAKE_B, 0, FAKE_C, 0x40000) == (1, 6)
    assert dot(0, 4, FAKE, 1, FAKE_B, 1, None, 0x40000) == (1, 7)
    assert dot(0, 4, FAKE, 1, FAKE_B, 1, FAKE_C, None) == (1, 8)
    assert dot(0, 4, FAKE + 8, 1, FAKE_B, 1, FAKE_C, 0x40000) == (2, 3)
    assert dot(0, 4, FAKE, 1, FAKE_B, 1, FAKE_C + 4, 0x40000) == (2, 7)

    def gv(trans=0, M=4, N=4, alpha=ONE, A=FAKE, lda=4, x=FAKE_B, incx=1, beta=ONE, y=FAKE_C, incy=1):
        return L.qgemv_d(trans, M, N, alpha, A, lda, x, incx, beta, y, incy, None), L.qgemm_last_invalid_arg()
    assert gv(trans=4) == (1, 1)
    assert gv(M=-1) == (1, 2)
    assert gv(N=-1) == (1, 3)
    assert gv(alpha=None) == (1, 4)
    assert gv(lda=3) == (1, 6)
    assert gv(incx=0) == (1, 8)
    assert gv(beta=None) == (1, 9)
    assert gv(incy=0) == (1, 11)
    assert gv(A=None) == (1, 5)
    assert gv(x=None) == (1, 7)
    assert gv(y=None) == (1, 10)
    assert gv(y=FAKE_B) == (1, 10)                                # y aliases x
    assert gv(y=FAKE + 64) == (1, 10)                             # y inside A
    assert gv(A=FAKE + 8) == (2, 5)
    assert gv(M=0, A=None, x=None, y=None) == (0, 0)
    assert gv(alpha=q4(0, 0, 0, 0), A=None, x=None, y=None) == (0, 0)   # alpha = 0, beta = 1


def test_outputs_must_not_overlap_inputs(L):
    """Every output is checked against the address ranges of what the call
    reads (the kernels write some tiles while others still read)."""
    # qgemm_d: C inside A (4 x 4 doubles quaternions span 512 bytes), C inside B, C == A
    assert call_d(L, A=FAKE, C=FAKE + 256) == 1 and L.qgemm_last_invalid_arg() == 12
    assert call_d(L, B=FAKE, C=FAKE + 256) == 1 and L.qgemm_last_invalid_arg() == 12
    assert call_d(L, A=FAKE, B=FAKE, C=FAKE_C, M=0) == 0          # empty output: nothing to check
    # qgemm_s / qgemm_ex_d / qgemm_mixed_d
    assert L.qgemm_s(0, 0, 4, 4, 4, ONE, FAKE, 4, FAKE_B, 4, ONE, FAKE_B + 64, 4, 6, None) == 1
    assert L.qgemm_last_invalid_arg() == 12
    assert L.qgemm_ex_d(0, 0, 4, 4, 4, ONE, None, None, FAKE, 4, FAKE_B, 4, ONE, None, FAKE, 4, None) == 1
    assert L.qgemm_last_invalid_arg() == 15
    assert call_mixed(L, C=FAKE) == 1 and L.qgemm_last_invalid_arg() == 14
    assert call_mixed(L, tA=1, tB=4, A=FAKE_C + 96, lda=4) == 1 and L.qgemm_last_invalid_arg() == 14
    # qherk_d: C over A
    d = ctypes.c_double
    assert L.qherk_d(0, 0, 4, 4, d(1.0), FAKE, 4, d(0.0), FAKE + 32, 4, None) == 1
    assert L.qgemm_last_invalid_arg() == 9
    # backward: dA over G, dB over A, dC0 over dA
    G = 0x50000
    args = lambda dA, dB, dC0: (0, 0, 4, 4, 4, ONE, FAKE, 4, FAKE_B, 4, G, 4, ONE, dA, 4, dB, 4, dC0, 4, None)
    assert L.qgemm_backward_d(*args(G + 32, None, None)) == 1 and L.qgemm_last_invalid_arg() == 14
    assert L.qgemm_backward_d(*args(None, FAKE, None)) == 1 and L.qgemm_last_invalid_arg() == 16
    assert L.qgemm_backward_d(*args(0x60000, None, 0x60000 + 128)) == 1 and L.qgemm_last_invalid_arg() == 18


def test_leading_dimensions_beyond_64bit_offsets_refused(L):
    """A leading dimension whose matrix would span more than 2^62 bytes is
    refused as unsupported (every offset the kernels form stays exact)."""
    huge = 1 << 60
    assert call_d(L, ldc=huge) == 5 and L.qgemm_last_invalid_arg() == 13
    assert call_d(L, lda=huge) == 5 and L.qgemm_last_invalid_arg() == 8
    assert L.qgemv_d(0, 4, 4, ONE, FAR_A, huge, FAR_B, 1, ONE, FAR_C, 1, None) == 5
    assert L.qgemm_last_invalid_arg() == 6
    assert L.qaxpy_d(4, ONE, FAR_A, huge, FAR_B, 1, None) == 5 and L.qgemm_last_invalid_arg() == 4
    assert call_mixed(L, tA=4, tB=1, A=FAR_A, B=FAR_B, C=FAR_C, ldb=huge) == 5 and L.qgemm_last_invalid_arg() == 12


def test_validation_mixed_s(L):
    """qgemm_mixed_s: float storage, element alignment 4 / 8 / 16 bytes."""
    args = lambda tA, tB, A, B, C: (tA, tB, 0, 0, 4, 4, 4, ONE, A, 4, B, 4, ONE, C, 4, None)
    assert L.qgemm_mixed_s(*args(4, 1, FAR_A + 8, FAR_B, FAR_C)) == 2 and L.qgemm_last_invalid_arg() == 9
    assert L.qgemm_mixed_s(*args(4, 1, FAR_A, FAR_B + 2, FAR_C)) == 2 and L.qgemm_last_invalid_arg() == 11
    assert L.qgemm_mixed_s(*args(2, 4, FAR_A + 4, FAR_B, FAR_C)) == 2 and L.qgemm_last_invalid_arg() == 9
    assert L.qgemm_mixed_s(*args(4, 1, FAR_A, FAR_B, FAR_C + 8)) == 2 and L.qgemm_last_invalid_arg() == 14
    assert L.qgemm_mixed_s(*args(1, 1, FAR_A, FAR_B, FAR_C)) == 1 and L.qgemm_last_invalid_arg() == 2


def test_tile_table_threads(L):
    """Concurrent installs and reads of the tile table from several host
    threads: every read returns one of the tables installed, whole."""
    import threading
    import paper_1903_05575_amd._lib as lb
    tables = [[c] * 32 for c in range(4)]
    seen = []
    errors = []

    def worker(k):
        try:
            for i in range(200):
                lb.set_tile_table(tables[(k + i) % 4])
                t = lb.tile_table()
                seen.append(tuple(t))
        except Exception as e:          # noqa: BLE001 -- reported below
            errors.append(e)

    th = [threading.Thread(target=worker, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    lb.set_tile_table(None)
    assert not errors
    assert set(seen) <= {tuple(t) for t in tables}


def test_batched_plan_leading_dimension_limit(L):
    """A problem whose leading dimension is beyond the 32-bit in-tile offsets
    of its tile is refused when the plan is made (QGEMM_ERR_UNSUPPORTED,
    argument 6 = the problem list, with its index), for FP32 and FP64 plans;
    nothing is allocated before that check."""
    import paper_1903_05575_amd._lib as lb
    h = ctypes.c_void_p()
    for dtype, big in ((0, 1 << 24), (1, 1 << 23)):
        probs = (lb.Problem * 2)()
        probs[0] = lb.Problem(4, 4, 4, 4, 4, 4, FAR_A, FAR_B, FAR_C)
        probs[1] = lb.Problem(4, 4, 4, big, 4, 4, FAR_A + (1 << 36), FAR_B + (1 << 36), FAR_C + (1 << 36))
        rc = L.qgemm_batched_plan_create(ctypes.byref(h), dtype, 1, 0, 2, probs, ONE, ONE, 0, -1)
        assert rc == 5 and L.qgemm_last_invalid_arg() == 6 and L.qgemm_last_invalid_problem() == 1, (dtype, rc)
        assert h.value is None
