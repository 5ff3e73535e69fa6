// C-ABI layer of libqgemm.so: argument validation (host only, before any HIP
// call), quick returns, and dispatch to the kernels.  See include/qgemm.h.
#include "qgemm_internal.hpp"

#include "../../include/qgemm.h"

#include <stdint.h>

#include <new>

namespace {

thread_local int g_bad_arg = 0;
thread_local int64_t g_bad_problem = -1;

qgemm_status_t fail(qgemm_status_t s, int arg)
{
    g_bad_arg = arg;
    return s;
}

bool valid_op(int op) { return op >= QGEMM_OP_N && op <= QGEMM_OP_R; }
bool op_transposes(int op) { return op == QGEMM_OP_T || op == QGEMM_OP_C; }
bool op_conjugates(int op) { return op == QGEMM_OP_C || op == QGEMM_OP_R; }
bool is_zero4(const double *q) { return q[0] == 0.0 && q[1] == 0.0 && q[2] == 0.0 && q[3] == 0.0; }

constexpr int64_t kMaxDim = 0x7fffffff;

// Whether the bytes spanned by two column-major matrices overlap: X is xrows x
// xcols with leading dimension ldx and xbytes per element, likewise Y.  Empty
// matrices overlap nothing.
bool ranges_overlap(const void *X, int64_t ldx, int64_t xrows, int64_t xcols, int64_t xbytes, const void *Y,
                    int64_t ldy, int64_t yrows, int64_t ycols, int64_t ybytes)
{
    if (!X || !Y || xrows <= 0 || xcols <= 0 || yrows <= 0 || ycols <= 0) return false;
    const __int128 x0 = (__int128)reinterpret_cast<uintptr_t>(X), y0 = (__int128)reinterpret_cast<uintptr_t>(Y);
    const __int128 x1 = x0 + ((__int128)ldx * (xcols - 1) + xrows) * xbytes;
    const __int128 y1 = y0 + ((__int128)ldy * (ycols - 1) + yrows) * ybytes;
    return x0 < y1 && y0 < x1;
}

// Whether a rows x cols matrix with leading dimension ld and ebytes per
// element spans at most 2^62 bytes, so that every element offset the kernels
// form in 64 bits is exact.  (Larger leading dimensions are refused as
// unsupported.)
bool extent_fits(int64_t ld, int64_t rows, int64_t cols, int64_t ebytes)
{
    if (rows <= 0 || cols <= 0) return true;
    return ((__int128)ld * (cols - 1) + rows) * ebytes <= ((__int128)1 << 62);
}
static_assert(QGEMM_DOT_WORK_DOUBLES >= 4 * qg::kDotParts, "dot workspace holds every partial sum");

// Validate a GEMM call.  Argument numbering follows the public signatures:
// 1 opA, 2 opB, 3 M, 4 N, 5 K, 6 alpha, 7 A, 8 lda, 9 B, 10 ldb, 11 beta,
// 12 C, 13 ldc.  `align` is the byte size of one element of C (and the
// alignment asked of C); `ab_bytes` the byte size of one element of A and B
// (the alignment asked of them, and the element size of the check that C
// overlaps neither); 0: A and B are aligned to `align` and the caller checks
// the overlap.
qgemm_status_t validate(int opA, int opB, int64_t M, int64_t N, int64_t K, const double *alpha,
                        const void *A, int64_t lda, const void *B, int64_t ldb, const double *beta,
                        const void *C, int64_t ldc, uintptr_t align, int64_t ab_bytes)
{
    g_bad_arg = 0;
    if (!valid_op(opA)) return fail(QGEMM_ERR_INVALID_ARG, 1);
    if (!valid_op(opB)) return fail(QGEMM_ERR_INVALID_ARG, 2);
    if (M < 0) return fail(QGEMM_ERR_INVALID_ARG, 3);
    if (N < 0) return fail(QGEMM_ERR_INVALID_ARG, 4);
    if (K < 0) return fail(QGEMM_ERR_INVALID_ARG, 5);
    if (M > kMaxDim) return fail(QGEMM_ERR_UNSUPPORTED, 3);
    if (N > kMaxDim) return fail(QGEMM_ERR_UNSUPPORTED, 4);
    if (K > kMaxDim) return fail(QGEMM_ERR_UNSUPPORTED, 5);
    if (!alpha) return fail(QGEMM_ERR_INVALID_ARG, 6);
    const int64_t rows_a = op_transposes(opA) ? K : M;
    const int64_t rows_b = op_transposes(opB) ? N : K;
    if (lda < (rows_a > 1 ? rows_a : 1)) return fail(QGEMM_ERR_INVALID_ARG, 8);
    if (ldb < (rows_b > 1 ? rows_b : 1)) return fail(QGEMM_ERR_INVALID_ARG, 10);
    if (!beta) return fail(QGEMM_ERR_INVALID_ARG, 11);
    if (ldc < (M > 1 ? M : 1)) return fail(QGEMM_ERR_INVALID_ARG, 13);
    if (M == 0 || N == 0) return QGEMM_OK;
    const bool reads_ab = K > 0 && !is_zero4(alpha);
    {
        const int64_t eb = ab_bytes ? ab_bytes : (int64_t)align;
        if (reads_ab && !extent_fits(lda, rows_a, op_transposes(opA) ? M : K, eb)) return fail(QGEMM_ERR_UNSUPPORTED, 8);
        if (reads_ab && !extent_fits(ldb, rows_b, op_transposes(opB) ? K : N, eb)) return fail(QGEMM_ERR_UNSUPPORTED, 10);
        if (!extent_fits(ldc, M, N, (int64_t)align)) return fail(QGEMM_ERR_UNSUPPORTED, 13);
    }
    if (reads_ab && !A) return fail(QGEMM_ERR_INVALID_ARG, 7);
    if (reads_ab && !B) return fail(QGEMM_ERR_INVALID_ARG, 9);
    if (!C) return fail(QGEMM_ERR_INVALID_ARG, 12);
    const uintptr_t ab_align = ab_bytes ? (uintptr_t)ab_bytes : align;
    if (reads_ab && (reinterpret_cast<uintptr_t>(A) % ab_align)) return fail(QGEMM_ERR_MISALIGNED, 7);
    if (reads_ab && (reinterpret_cast<uintptr_t>(B) % ab_align)) return fail(QGEMM_ERR_MISALIGNED, 9);
    if (reinterpret_cast<uintptr_t>(C) % align) return fail(QGEMM_ERR_MISALIGNED, 12);
    // C is written by some tiles while others still read A and B
    if (reads_ab && ab_bytes) {
        const int64_t cols_a = op_transposes(opA) ? M : K, cols_b = op_transposes(opB) ? K : N;
        if (ranges_overlap(C, ldc, M, N, (int64_t)align, A, lda, rows_a, cols_a, ab_bytes) ||
            ranges_overlap(C, ldc, M, N, (int64_t)align, B, ldb, rows_b, cols_b, ab_bytes))
            return fail(QGEMM_ERR_INVALID_ARG, 12);
    }
    return QGEMM_OK;
}

template <typename T>
qg::GemmDesc<T> make_desc(int opA, int opB, int64_t M, int64_t N, int64_t K, const double *alpha,
                          const T *A, int64_t lda, const T *B, int64_t ldb, const double *beta,
                          T *C, int64_t ldc)
{
    qg::GemmDesc<T> d{};
    d.A = A;
    d.B = B;
    d.C = C;
    d.lda = lda;
    d.ldb = ldb;
    d.ldc = ldc;
    d.M = (int)M;
    d.N = (int)N;
    d.K = (int)K;
    d.opA_t = op_transposes(opA);
    d.conjA = op_conjugates(opA);
    d.opB_t = op_transposes(opB);
    d.conjB = op_conjugates(opB);
    d.has_bscale = false;
    d.store_t = false;
    d.store_conj = false;
    d.has_right = false;
    d.uplo = 0;
    d.herm_diag = false;
    d.tri = 0;
    d.tri_lower = false;
    d.tri_unit = false;
    for (int i = 0; i < 4; ++i) {
        d.alpha[i] = alpha[i];
        d.beta[i] = beta[i];
        d.bscale[i] = i == 0 ? 1.0 : 0.0;
        d.alpha_r[i] = i == 0 ? 1.0 : 0.0;
        d.beta_r[i] = i == 0 ? 1.0 : 0.0;
    }
    return d;
}

// op of the stored operand that yields op(X)^H, for the gradient:
// N -> C, T -> R (conj only), C -> N, R -> T.
int adjoint_op(int op)
{
    switch (op) {
    case QGEMM_OP_N: return QGEMM_OP_C;
    case QGEMM_OP_T: return QGEMM_OP_R;
    case QGEMM_OP_C: return QGEMM_OP_N;
    default: return QGEMM_OP_T;
    }
}

// Gradient of L = <G, alpha op(A) op(B) + beta C0> (real inner product of the
// components) with respect to the stored A, B and C0.  For quaternions
// <x, q y> = <conj(q) x, y> and <x, y q> = <x conj(q), y> (the 4 x 4 matrices
// of left and right multiplication by q are transposed by conjugating q), so
// <G, alpha a b> = <conj(alpha) G conj(b), a> = <conj(a) conj(alpha) G, b>
// term by term, and summing over the products of each output:
//   d op(A) = conj(alpha) G op(B)^H                (left scalar)
//   d op(B) = op(A)^H (conj(alpha) G)              (scalar between the factors)
//   dC0     = conj(beta) G
// and dX is d op(X) mapped back through op: N as is, T transposed, C
// conjugate-transposed, R conjugated.  Each map is applied by the store of the
// GEMM epilogue; the middle scalar is applied to op(B) as it is staged.
template <typename T>
qgemm_status_t backward_impl(int opA, int opB, int64_t M, int64_t N, int64_t K, const double *alpha, const T *A,
                             int64_t lda, const T *B, int64_t ldb, const T *G, int64_t ldg, const double *beta,
                             T *dA, int64_t ldda, T *dB, int64_t lddb, T *dC0, int64_t lddc0, int split_terms,
                             hipStream_t stream)
{
    constexpr uintptr_t align = 4 * sizeof(T);
    g_bad_arg = 0;
    if (!valid_op(opA)) return fail(QGEMM_ERR_INVALID_ARG, 1);
    if (!valid_op(opB)) return fail(QGEMM_ERR_INVALID_ARG, 2);
    if (M < 0) return fail(QGEMM_ERR_INVALID_ARG, 3);
    if (N < 0) return fail(QGEMM_ERR_INVALID_ARG, 4);
    if (K < 0) return fail(QGEMM_ERR_INVALID_ARG, 5);
    if (M > kMaxDim) return fail(QGEMM_ERR_UNSUPPORTED, 3);
    if (N > kMaxDim) return fail(QGEMM_ERR_UNSUPPORTED, 4);
    if (K > kMaxDim) return fail(QGEMM_ERR_UNSUPPORTED, 5);
    if (!alpha) return fail(QGEMM_ERR_INVALID_ARG, 6);
    const int64_t rows_a = op_transposes(opA) ? K : M;
    const int64_t rows_b = op_transposes(opB) ? N : K;
    if (lda < (rows_a > 1 ? rows_a : 1)) return fail(QGEMM_ERR_INVALID_ARG, 8);
    if (ldb < (rows_b > 1 ? rows_b : 1)) return fail(QGEMM_ERR_INVALID_ARG, 10);
    if (ldg < (M > 1 ? M : 1)) return fail(QGEMM_ERR_INVALID_ARG, 12);
    if (!beta) return fail(QGEMM_ERR_INVALID_ARG, 13);
    if (dA && ldda < (rows_a > 1 ? rows_a : 1)) return fail(QGEMM_ERR_INVALID_ARG, 15);
    if (dB && lddb < (rows_b > 1 ? rows_b : 1)) return fail(QGEMM_ERR_INVALID_ARG, 17);
    if (dC0 && lddc0 < (M > 1 ? M : 1)) return fail(QGEMM_ERR_INVALID_ARG, 19);
    if (split_terms == 0) split_terms = 6;
    if (split_terms != 3 && split_terms != 6 && split_terms != 9) return fail(QGEMM_ERR_INVALID_ARG, 20);
    const bool need_a = dA && M > 0 && K > 0;
    const bool need_b = dB && K > 0 && N > 0;
    const bool need_c = dC0 && M > 0 && N > 0;
    const bool reads_g = (need_a || need_b) ? (M > 0 && N > 0) : need_c;
    if (reads_g && !G) return fail(QGEMM_ERR_INVALID_ARG, 11);
    if (need_a && N > 0 && !B) return fail(QGEMM_ERR_INVALID_ARG, 9);
    if (need_b && M > 0 && !A) return fail(QGEMM_ERR_INVALID_ARG, 7);
    auto misaligned = [&](const void *p) { return p && (reinterpret_cast<uintptr_t>(p) % align) != 0; };
    if (misaligned(A)) return fail(QGEMM_ERR_MISALIGNED, 7);
    if (misaligned(B)) return fail(QGEMM_ERR_MISALIGNED, 9);
    if (misaligned(G)) return fail(QGEMM_ERR_MISALIGNED, 11);
    if (misaligned(dA)) return fail(QGEMM_ERR_MISALIGNED, 14);
    if (misaligned(dB)) return fail(QGEMM_ERR_MISALIGNED, 16);
    if (misaligned(dC0)) return fail(QGEMM_ERR_MISALIGNED, 18);
    {
        constexpr int64_t qb = 4 * sizeof(T);
        const int64_t cols_a = op_transposes(opA) ? M : K, cols_b = op_transposes(opB) ? K : N;
        if (!extent_fits(lda, rows_a, cols_a, qb)) return fail(QGEMM_ERR_UNSUPPORTED, 8);
        if (!extent_fits(ldb, rows_b, cols_b, qb)) return fail(QGEMM_ERR_UNSUPPORTED, 10);
        if (!extent_fits(ldg, M, N, qb)) return fail(QGEMM_ERR_UNSUPPORTED, 12);
        if (dA && !extent_fits(ldda, rows_a, cols_a, qb)) return fail(QGEMM_ERR_UNSUPPORTED, 15);
        if (dB && !extent_fits(lddb, rows_b, cols_b, qb)) return fail(QGEMM_ERR_UNSUPPORTED, 17);
        if (dC0 && !extent_fits(lddc0, M, N, qb)) return fail(QGEMM_ERR_UNSUPPORTED, 19);
    }
    {
        // every output is written while the other gradient launch may still read the inputs
        struct Span {
            const void *p;
            int64_t ld, rows, cols;
        };
        const int64_t cols_a = op_transposes(opA) ? M : K, cols_b = op_transposes(opB) ? K : N;
        const Span in[3] = {{A, lda, rows_a, cols_a}, {B, ldb, rows_b, cols_b}, {G, ldg, M, N}};
        const Span out[3] = {{need_a ? dA : nullptr, ldda, rows_a, cols_a},
                             {need_b ? dB : nullptr, lddb, rows_b, cols_b},
                             {need_c ? dC0 : nullptr, lddc0, M, N}};
        const int out_arg[3] = {14, 16, 18};
        constexpr int64_t qb = 4 * sizeof(T);
        for (int o = 0; o < 3; ++o) {
            for (int i = 0; i < 3; ++i)
                if (ranges_overlap(out[o].p, out[o].ld, out[o].rows, out[o].cols, qb, in[i].p, in[i].ld, in[i].rows,
                                   in[i].cols, qb))
                    return fail(QGEMM_ERR_INVALID_ARG, out_arg[o]);
            for (int j = 0; j < o; ++j)
                if (ranges_overlap(out[o].p, out[o].ld, out[o].rows, out[o].cols, qb, out[j].p, out[j].ld,
                                   out[j].rows, out[j].cols, qb))
                    return fail(QGEMM_ERR_INVALID_ARG, out_arg[o]);
        }
    }
    {
        // the two gradient GEMMs read (G, op(B)^H) and (op(A)^H, G) through the GEMM tiles
        auto ok = [](int64_t l1, int64_t l2, bool t1, bool t2) {
            return sizeof(T) == 4 ? qg::split_ld_supported(l1, l2, t1, t2) : qg::f64_ld_supported(l1, l2, t1, t2);
        };
        if (!ok(ldg, ldb, false, !op_transposes(opB)) || !ok(lda, ldg, !op_transposes(opA), false))
            return fail(QGEMM_ERR_UNSUPPORTED, 8);
    }
    if ((need_a && (dA == (const T *)A || dA == (const T *)B || dA == (const T *)G)) ||
        (need_b && (dB == (const T *)A || dB == (const T *)B || dB == (const T *)G)))
        return fail(QGEMM_ERR_INVALID_ARG, need_a ? 14 : 16);

    const double one[4] = {1.0, 0.0, 0.0, 0.0};
    const double zero[4] = {0.0, 0.0, 0.0, 0.0};
    const double ca[4] = {alpha[0], -alpha[1], -alpha[2], -alpha[3]};
    auto launch = [&](qg::GemmDesc<T> &d) -> hipError_t {
        if constexpr (sizeof(T) == 8) return qg::launch_qgemm_f64(d, stream);
        else return qg::launch_qgemm_bf16x3(d, nullptr, split_terms, qg::kSplitPanel, stream);
    };
    if (need_a) {
        // d op(A) (M x K) = conj(alpha) G (M x N) op(B)^H (N x K)
        auto d = make_desc<T>(QGEMM_OP_N, adjoint_op(opB), M, K, N, ca, G, ldg, B, ldb, zero, dA, ldda);
        d.store_t = op_transposes(opA);
        d.store_conj = op_conjugates(opA);
        if (launch(d) != hipSuccess) return QGEMM_ERR_HIP;
    }
    if (need_b) {
        // d op(B) (K x N) = op(A)^H (K x M) (conj(alpha) G) (M x N)
        auto d = make_desc<T>(adjoint_op(opA), QGEMM_OP_N, K, N, M, one, A, lda, G, ldg, zero, dB, lddb);
        d.has_bscale = !(ca[0] == 1.0 && ca[1] == 0.0 && ca[2] == 0.0 && ca[3] == 0.0);
        for (int i = 0; i < 4; ++i) d.bscale[i] = ca[i];
        d.store_t = op_transposes(opB);
        d.store_conj = op_conjugates(opB);
        if (launch(d) != hipSuccess) return QGEMM_ERR_HIP;
    }
    if (need_c) {
        const double cb[4] = {beta[0], -beta[1], -beta[2], -beta[3]};
        if (qg::launch_scale_left<T>(G, ldg, dC0, lddc0, (int)M, (int)N, cb, stream) != hipSuccess)
            return QGEMM_ERR_HIP;
    }
    return QGEMM_OK;
}

bool is_one4(const double *q) { return q[0] == 1.0 && q[1] == 0.0 && q[2] == 0.0 && q[3] == 0.0; }

// General scalar placement C <- aL (sum op(A) aM op(B)) aR + bL C bR (the left,
// middle and right scalar products of Sec. 2.2).  NULL scalars take their
// defaults (unit; zero for bL).  Argument numbering of the public calls:
// 1 opA, 2 opB, 3 M, 4 N, 5 K, 6 aL, 7 aM, 8 aR, 9 A, 10 lda, 11 B, 12 ldb,
// 13 bL, 14 bR, 15 C, 16 ldc, 17 split_terms (FP32 only).
template <typename T>
qgemm_status_t ex_impl(int opA, int opB, int64_t M, int64_t N, int64_t K, const double *aL, const double *aM,
                       const double *aR, const T *A, int64_t lda, const T *B, int64_t ldb, const double *bL,
                       const double *bR, T *C, int64_t ldc, int split_terms, hipStream_t stream)
{
    static const double one[4] = {1.0, 0.0, 0.0, 0.0};
    static const double zero[4] = {0.0, 0.0, 0.0, 0.0};
    const double *l = aL ? aL : one, *m = aM ? aM : one, *r = aR ? aR : one;
    const double *bl = bL ? bL : zero, *br = bR ? bR : one;
    // the product vanishes when any alpha is zero: validate as for alpha = 0
    const bool az = is_zero4(l) || is_zero4(m) || is_zero4(r);
    qgemm_status_t s = validate(opA, opB, M, N, K, az ? zero : l, A, lda, B, ldb, bl, C, ldc, 4 * sizeof(T),
                                4 * sizeof(T));
    if (s != QGEMM_OK) {
        static const int remap[14] = {0, 1, 2, 3, 4, 5, 6, 9, 10, 11, 12, 13, 15, 16};
        g_bad_arg = remap[g_bad_arg];
        return s;
    }
    if (sizeof(T) == 4) {
        if (split_terms == 0) split_terms = 6;
        if (split_terms != 3 && split_terms != 6 && split_terms != 9) return fail(QGEMM_ERR_INVALID_ARG, 17);
    }
    if (M == 0 || N == 0) return QGEMM_OK;
    const bool ld_ok = sizeof(T) == 4 ? qg::split_ld_supported(lda, ldb, op_transposes(opA), op_transposes(opB))
                                      : qg::f64_ld_supported(lda, ldb, op_transposes(opA), op_transposes(opB));
    if (!ld_ok) return fail(QGEMM_ERR_UNSUPPORTED, op_transposes(opA) ? 10 : 12);
    auto d = make_desc<T>(opA, opB, M, N, K, az ? zero : l, A, lda, B, ldb, bl, C, ldc);
    d.has_bscale = !az && !is_one4(m);
    d.has_right = !(is_one4(r) && is_one4(br));
    for (int i = 0; i < 4; ++i) {
        d.bscale[i] = m[i];
        d.alpha_r[i] = r[i];
        d.beta_r[i] = br[i];
    }
    hipError_t e;
    if constexpr (sizeof(T) == 8) e = qg::launch_qgemm_f64(d, stream);
    else e = qg::launch_qgemm_bf16x3(d, nullptr, split_terms, qg::kSplitPanel, stream);
    return e == hipSuccess ? QGEMM_OK : QGEMM_ERR_HIP;
}

// Hermitian rank-k update on one triangle of C (BLAS HERK convention, alpha
// and beta real): trans N: C <- alpha A A^H + beta C (A n x k); trans C:
// C <- alpha A^H A + beta C (A k x n).  The GEMM kernels run with B = A and
// the adjoint op; tiles outside the triangle exit at once and the epilogue
// writes only the triangle, with a real diagonal.
// Arguments: 1 uplo, 2 trans, 3 N, 4 K, 5 alpha, 6 A, 7 lda, 8 beta, 9 C,
// 10 ldc, 11 split_terms (FP32 only).
template <typename T>
qgemm_status_t herk_impl(int uplo, int trans, int64_t N, int64_t K, double alpha, const T *A, int64_t lda,
                         double beta, T *C, int64_t ldc, int split_terms, hipStream_t stream)
{
    constexpr uintptr_t align = 4 * sizeof(T);
    g_bad_arg = 0;
    if (uplo != QGEMM_LOWER && uplo != QGEMM_UPPER) return fail(QGEMM_ERR_INVALID_ARG, 1);
    if (trans != QGEMM_OP_N && trans != QGEMM_OP_C) return fail(QGEMM_ERR_INVALID_ARG, 2);
    if (N < 0) return fail(QGEMM_ERR_INVALID_ARG, 3);
    if (K < 0) return fail(QGEMM_ERR_INVALID_ARG, 4);
    if (N > kMaxDim) return fail(QGEMM_ERR_UNSUPPORTED, 3);
    if (K > kMaxDim) return fail(QGEMM_ERR_UNSUPPORTED, 4);
    const int64_t rows_a = trans == QGEMM_OP_N ? N : K;
    if (lda < (rows_a > 1 ? rows_a : 1)) return fail(QGEMM_ERR_INVALID_ARG, 7);
    if (ldc < (N > 1 ? N : 1)) return fail(QGEMM_ERR_INVALID_ARG, 10);
    if (sizeof(T) == 4) {
        if (split_terms == 0) split_terms = 6;
        if (split_terms != 3 && split_terms != 6 && split_terms != 9) return fail(QGEMM_ERR_INVALID_ARG, 11);
    }
    if (N == 0) return QGEMM_OK;
    if ((alpha == 0.0 || K == 0) && beta == 1.0) return QGEMM_OK;     // nothing to update
    const bool reads_a = K > 0 && alpha != 0.0;
    if (reads_a && !A) return fail(QGEMM_ERR_INVALID_ARG, 6);
    if (!C) return fail(QGEMM_ERR_INVALID_ARG, 9);
    if (reads_a && (reinterpret_cast<uintptr_t>(A) % align)) return fail(QGEMM_ERR_MISALIGNED, 6);
    if (reinterpret_cast<uintptr_t>(C) % align) return fail(QGEMM_ERR_MISALIGNED, 9);
    if (reads_a && !extent_fits(lda, rows_a, trans == QGEMM_OP_N ? K : N, 4 * sizeof(T)))
        return fail(QGEMM_ERR_UNSUPPORTED, 7);
    if (!extent_fits(ldc, N, N, 4 * sizeof(T))) return fail(QGEMM_ERR_UNSUPPORTED, 10);
    if (reads_a && ranges_overlap(C, ldc, N, N, 4 * sizeof(T), A, lda, rows_a, trans == QGEMM_OP_N ? K : N,
                                  4 * sizeof(T)))
        return fail(QGEMM_ERR_INVALID_ARG, 9);
    const bool ta = trans == QGEMM_OP_C;
    const bool ld_ok = sizeof(T) == 4 ? qg::split_ld_supported(lda, lda, ta, !ta) : qg::f64_ld_supported(lda, lda, ta, !ta);
    if (!ld_ok) return fail(QGEMM_ERR_UNSUPPORTED, 7);
    const double al[4] = {alpha, 0.0, 0.0, 0.0};
    const double be[4] = {beta, 0.0, 0.0, 0.0};
    auto d = make_desc<T>(trans, adjoint_op(trans), N, N, K, al, A, lda, A, lda, be, C, ldc);
    d.uplo = uplo == QGEMM_LOWER ? 1 : 2;
    d.herm_diag = true;
    hipError_t e;
    if constexpr (sizeof(T) == 8) e = qg::launch_qgemm_f64(d, stream);
    else e = qg::launch_qgemm_bf16x3(d, nullptr, split_terms, qg::kSplitPanel, stream);
    return e == hipSuccess ? QGEMM_OK : QGEMM_ERR_HIP;
}

// Triangular multiply on the GEMM kernels: the triangular matrix is op(A)
// (side left, K = M) or op(B) (side right, K = N) of one GEMM launch with
// beta = 0.  Argument numbering as in include/qgemm.h.
template <typename T>
qgemm_status_t trmm_impl(int side, int uplo, int trans, int diag, int64_t M, int64_t N, const double *alpha,
                         const T *A, int64_t lda, const T *B, int64_t ldb, T *C, int64_t ldc, int split_terms,
                         hipStream_t stream)
{
    constexpr uintptr_t align = 4 * sizeof(T);
    g_bad_arg = 0;
    if (side != QGEMM_SIDE_LEFT && side != QGEMM_SIDE_RIGHT) return fail(QGEMM_ERR_INVALID_ARG, 1);
    if (uplo != QGEMM_LOWER && uplo != QGEMM_UPPER) return fail(QGEMM_ERR_INVALID_ARG, 2);
    if (!valid_op(trans)) return fail(QGEMM_ERR_INVALID_ARG, 3);
    if (diag != QGEMM_NON_UNIT && diag != QGEMM_UNIT) return fail(QGEMM_ERR_INVALID_ARG, 4);
    if (M < 0) return fail(QGEMM_ERR_INVALID_ARG, 5);
    if (N < 0) return fail(QGEMM_ERR_INVALID_ARG, 6);
    if (M > kMaxDim) return fail(QGEMM_ERR_UNSUPPORTED, 5);
    if (N > kMaxDim) return fail(QGEMM_ERR_UNSUPPORTED, 6);
    if (!alpha) return fail(QGEMM_ERR_INVALID_ARG, 7);
    const int64_t n = side == QGEMM_SIDE_LEFT ? M : N;
    if (lda < (n > 1 ? n : 1)) return fail(QGEMM_ERR_INVALID_ARG, 9);
    if (ldb < (M > 1 ? M : 1)) return fail(QGEMM_ERR_INVALID_ARG, 11);
    if (ldc < (M > 1 ? M : 1)) return fail(QGEMM_ERR_INVALID_ARG, 13);
    if (sizeof(T) == 4) {
        if (split_terms == 0) split_terms = 6;
        if (split_terms != 3 && split_terms != 6 && split_terms != 9) return fail(QGEMM_ERR_INVALID_ARG, 14);
    }
    if (M == 0 || N == 0) return QGEMM_OK;
    const bool reads_ab = !is_zero4(alpha);
    if (reads_ab && !A) return fail(QGEMM_ERR_INVALID_ARG, 8);
    if (reads_ab && !B) return fail(QGEMM_ERR_INVALID_ARG, 10);
    if (!C) return fail(QGEMM_ERR_INVALID_ARG, 12);
    if (reads_ab && (reinterpret_cast<uintptr_t>(A) % align)) return fail(QGEMM_ERR_MISALIGNED, 8);
    if (reads_ab && (reinterpret_cast<uintptr_t>(B) % align)) return fail(QGEMM_ERR_MISALIGNED, 10);
    if (reinterpret_cast<uintptr_t>(C) % align) return fail(QGEMM_ERR_MISALIGNED, 12);
    if (reads_ab && !extent_fits(lda, n, n, 4 * sizeof(T))) return fail(QGEMM_ERR_UNSUPPORTED, 9);
    if (reads_ab && !extent_fits(ldb, M, N, 4 * sizeof(T))) return fail(QGEMM_ERR_UNSUPPORTED, 11);
    if (!extent_fits(ldc, M, N, 4 * sizeof(T))) return fail(QGEMM_ERR_UNSUPPORTED, 13);
    // C is written while A and B are still read by other tiles: no overlap
    if (reads_ab && (ranges_overlap(C, ldc, M, N, 4 * sizeof(T), A, lda, n, n, 4 * sizeof(T)) ||
                     ranges_overlap(C, ldc, M, N, 4 * sizeof(T), B, ldb, M, N, 4 * sizeof(T))))
        return fail(QGEMM_ERR_INVALID_ARG, 12);
    const bool left = side == QGEMM_SIDE_LEFT;
    const bool ta = left ? op_transposes(trans) : false, tb = left ? false : op_transposes(trans);
    const bool ld_ok = sizeof(T) == 4 ? qg::split_ld_supported(left ? lda : ldb, left ? ldb : lda, ta, tb)
                                      : qg::f64_ld_supported(left ? lda : ldb, left ? ldb : lda, ta, tb);
    if (!ld_ok) return fail(QGEMM_ERR_UNSUPPORTED, 9);
    const double zero[4] = {0.0, 0.0, 0.0, 0.0};
    auto d = left ? make_desc<T>(trans, QGEMM_OP_N, M, N, M, alpha, A, lda, B, ldb, zero, C, ldc)
                  : make_desc<T>(QGEMM_OP_N, trans, M, N, N, alpha, B, ldb, A, lda, zero, C, ldc);
    d.tri = left ? 1 : 2;
    d.tri_lower = (uplo == QGEMM_LOWER) != op_transposes(trans);   // the triangle after the op
    d.tri_unit = diag == QGEMM_UNIT;
    hipError_t e;
    if constexpr (sizeof(T) == 8) e = qg::launch_qgemm_f64(d, stream);
    else e = qg::launch_qgemm_bf16x3(d, nullptr, split_terms, qg::kSplitPanel, stream);
    return e == hipSuccess ? QGEMM_OK : QGEMM_ERR_HIP;
}

// Bytes spanned by n strided quaternions of `qbytes` bytes each.
bool vec_overlap(const void *X, int64_t nx, int64_t incx, const void *Y, int64_t ny, int64_t incy, int64_t qbytes)
{
    return ranges_overlap(X, incx, 1, nx, qbytes, Y, incy, 1, ny, qbytes);
}

template <typename T>
qgemm_status_t axpy_impl(int64_t n, const double *alpha, const T *x, int64_t incx, T *y, int64_t incy,
                         hipStream_t stream)
{
    constexpr uintptr_t align = 4 * sizeof(T);
    g_bad_arg = 0;
    if (n < 0) return fail(QGEMM_ERR_INVALID_ARG, 1);
    if (!alpha) return fail(QGEMM_ERR_INVALID_ARG, 2);
    if (incx < 1) return fail(QGEMM_ERR_INVALID_ARG, 4);
    if (incy < 1) return fail(QGEMM_ERR_INVALID_ARG, 6);
    if (n == 0 || is_zero4(alpha)) return QGEMM_OK;
    if (!x) return fail(QGEMM_ERR_INVALID_ARG, 3);
    if (!y) return fail(QGEMM_ERR_INVALID_ARG, 5);
    if (reinterpret_cast<uintptr_t>(x) % align) return fail(QGEMM_ERR_MISALIGNED, 3);
    if (reinterpret_cast<uintptr_t>(y) % align) return fail(QGEMM_ERR_MISALIGNED, 5);
    if (!extent_fits(incx, 1, n, 4 * sizeof(T))) return fail(QGEMM_ERR_UNSUPPORTED, 4);
    if (!extent_fits(incy, 1, n, 4 * sizeof(T))) return fail(QGEMM_ERR_UNSUPPORTED, 6);
    if (!(x == y && incx == incy) && vec_overlap(x, n, incx, y, n, incy, 4 * sizeof(T)))
        return fail(QGEMM_ERR_INVALID_ARG, 5);
    return qg::launch_qaxpy<T>(n, alpha, x, incx, y, incy, stream) == hipSuccess ? QGEMM_OK : QGEMM_ERR_HIP;
}

// own_work: the partial sums go to the library's file-scope workspace
// (qdot_d_noalloc) instead of the caller's `work`, whose address is looked up
// only after every argument has been validated.
template <typename T>
qgemm_status_t dot_impl(int conj, int64_t n, const T *x, int64_t incx, const T *y, int64_t incy, T *result,
                        double *work, hipStream_t stream, bool own_work = false)
{
    constexpr uintptr_t align = 4 * sizeof(T);
    g_bad_arg = 0;
    if (conj != 0 && conj != 1) return fail(QGEMM_ERR_INVALID_ARG, 1);
    if (n < 0) return fail(QGEMM_ERR_INVALID_ARG, 2);
    if (incx < 1) return fail(QGEMM_ERR_INVALID_ARG, 4);
    if (incy < 1) return fail(QGEMM_ERR_INVALID_ARG, 6);
    if (!result) return fail(QGEMM_ERR_INVALID_ARG, 7);
    if (reinterpret_cast<uintptr_t>(result) % sizeof(T)) return fail(QGEMM_ERR_MISALIGNED, 7);
    if (n > 0) {
        if (!x) return fail(QGEMM_ERR_INVALID_ARG, 3);
        if (!y) return fail(QGEMM_ERR_INVALID_ARG, 5);
        if (!own_work && !work) return fail(QGEMM_ERR_INVALID_ARG, 8);
        if (reinterpret_cast<uintptr_t>(x) % align) return fail(QGEMM_ERR_MISALIGNED, 3);
        if (reinterpret_cast<uintptr_t>(y) % align) return fail(QGEMM_ERR_MISALIGNED, 5);
        if (!own_work && reinterpret_cast<uintptr_t>(work) % sizeof(double)) return fail(QGEMM_ERR_MISALIGNED, 8);
        if (!extent_fits(incx, 1, n, 4 * sizeof(T))) return fail(QGEMM_ERR_UNSUPPORTED, 4);
        if (!extent_fits(incy, 1, n, 4 * sizeof(T))) return fail(QGEMM_ERR_UNSUPPORTED, 6);
        if (own_work) {
            int cap = 0;
            if (qg::dot_scratch(&work, &cap) != hipSuccess) return QGEMM_ERR_HIP;
            if (cap < 4 * qg::kDotParts) return QGEMM_ERR_UNSUPPORTED;   // cannot happen: sized for kDotParts
        }
    }
    return qg::launch_qdot<T>(conj == 1, n, x, incx, y, incy, result, work, stream) == hipSuccess ? QGEMM_OK
                                                                                                : QGEMM_ERR_HIP;
}

template <typename T>
qgemm_status_t gemv_impl(int trans, int64_t M, int64_t N, const double *alpha, const T *A, int64_t lda, const T *x,
                         int64_t incx, const double *beta, T *y, int64_t incy, hipStream_t stream)
{
    constexpr uintptr_t align = 4 * sizeof(T);
    g_bad_arg = 0;
    if (!valid_op(trans)) return fail(QGEMM_ERR_INVALID_ARG, 1);
    if (M < 0) return fail(QGEMM_ERR_INVALID_ARG, 2);
    if (N < 0) return fail(QGEMM_ERR_INVALID_ARG, 3);
    if (M > kMaxDim) return fail(QGEMM_ERR_UNSUPPORTED, 2);
    if (N > kMaxDim) return fail(QGEMM_ERR_UNSUPPORTED, 3);
    if (!alpha) return fail(QGEMM_ERR_INVALID_ARG, 4);
    if (lda < (M > 1 ? M : 1)) return fail(QGEMM_ERR_INVALID_ARG, 6);
    if (incx < 1) return fail(QGEMM_ERR_INVALID_ARG, 8);
    if (!beta) return fail(QGEMM_ERR_INVALID_ARG, 9);
    if (incy < 1) return fail(QGEMM_ERR_INVALID_ARG, 11);
    if (M == 0 || N == 0) return QGEMM_OK;
    const bool alpha_zero = is_zero4(alpha);
    if (alpha_zero && beta[0] == 1.0 && beta[1] == 0.0 && beta[2] == 0.0 && beta[3] == 0.0) return QGEMM_OK;
    const bool tr = trans == QGEMM_OP_T || trans == QGEMM_OP_C;
    const int64_t nx = tr ? M : N, ny = tr ? N : M;
    if (!alpha_zero && !A) return fail(QGEMM_ERR_INVALID_ARG, 5);
    if (!alpha_zero && !x) return fail(QGEMM_ERR_INVALID_ARG, 7);
    if (!y) return fail(QGEMM_ERR_INVALID_ARG, 10);
    if (!alpha_zero && (reinterpret_cast<uintptr_t>(A) % align)) return fail(QGEMM_ERR_MISALIGNED, 5);
    if (!alpha_zero && (reinterpret_cast<uintptr_t>(x) % align)) return fail(QGEMM_ERR_MISALIGNED, 7);
    if (reinterpret_cast<uintptr_t>(y) % align) return fail(QGEMM_ERR_MISALIGNED, 10);
    if (!alpha_zero && !extent_fits(lda, M, N, 4 * sizeof(T))) return fail(QGEMM_ERR_UNSUPPORTED, 6);
    if (!alpha_zero && !extent_fits(incx, 1, nx, 4 * sizeof(T))) return fail(QGEMM_ERR_UNSUPPORTED, 8);
    if (!extent_fits(incy, 1, ny, 4 * sizeof(T))) return fail(QGEMM_ERR_UNSUPPORTED, 11);
    if (!alpha_zero && (vec_overlap(x, nx, incx, y, ny, incy, 4 * sizeof(T)) ||
                        ranges_overlap(A, lda, M, N, 4 * sizeof(T), y, incy, 1, ny, 4 * sizeof(T))))
        return fail(QGEMM_ERR_INVALID_ARG, 10);
    return qg::launch_qgemv<T>(trans, (int)M, (int)N, alpha, A, lda, x, incx, beta, y, incy, stream) == hipSuccess
               ? QGEMM_OK
               : QGEMM_ERR_HIP;
}

// Mixed-type GEMM (one operand real or complex, the other quaternion) for
// double (T = double) or float (T = float) storage; FP64 arithmetic either
// way.  Argument numbering as in include/qgemm.h: 1 typeA, 2 typeB, then as
// qgemm_d shifted by two.
template <typename T>
qgemm_status_t mixed_impl(int typeA, int typeB, int opA, int opB, int64_t M, int64_t N, int64_t K,
                          const double *alpha, const T *A, int64_t lda, const T *B, int64_t ldb, const double *beta,
                          T *C, int64_t ldc, hipStream_t stream)
{
    constexpr int64_t rb = sizeof(T);   // bytes of one real
    g_bad_arg = 0;
    auto valid_type = [](int t) { return t == QGEMM_REAL || t == QGEMM_COMPLEX || t == QGEMM_QUATERNION; };
    if (!valid_type(typeA)) return fail(QGEMM_ERR_INVALID_ARG, 1);
    if (!valid_type(typeB)) return fail(QGEMM_ERR_INVALID_ARG, 2);
    if (typeA != QGEMM_QUATERNION && typeB != QGEMM_QUATERNION) return fail(QGEMM_ERR_INVALID_ARG, 2);
    qgemm_status_t s = validate(opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, rb, 0);
    if (s != QGEMM_OK) return fail(s, g_bad_arg + 2);
    if (M == 0 || N == 0) return QGEMM_OK;
    const bool reads_ab = K > 0 && !is_zero4(alpha);
    if (reads_ab && (reinterpret_cast<uintptr_t>(A) % (uintptr_t)(rb * typeA))) return fail(QGEMM_ERR_MISALIGNED, 9);
    if (reads_ab && (reinterpret_cast<uintptr_t>(B) % (uintptr_t)(rb * typeB))) return fail(QGEMM_ERR_MISALIGNED, 11);
    if (reinterpret_cast<uintptr_t>(C) % (uintptr_t)(4 * rb)) return fail(QGEMM_ERR_MISALIGNED, 14);
    if (!extent_fits(ldc, M, N, 4 * rb)) return fail(QGEMM_ERR_UNSUPPORTED, 15);
    if (reads_ab) {
        const int64_t ra = op_transposes(opA) ? K : M, ca = op_transposes(opA) ? M : K;
        const int64_t rbb = op_transposes(opB) ? N : K, cb = op_transposes(opB) ? K : N;
        if (!extent_fits(lda, ra, ca, rb * typeA)) return fail(QGEMM_ERR_UNSUPPORTED, 10);
        if (!extent_fits(ldb, rbb, cb, rb * typeB)) return fail(QGEMM_ERR_UNSUPPORTED, 12);
        if (ranges_overlap(C, ldc, M, N, 4 * rb, A, lda, ra, ca, rb * typeA) ||
            ranges_overlap(C, ldc, M, N, 4 * rb, B, ldb, rbb, cb, rb * typeB))
            return fail(QGEMM_ERR_INVALID_ARG, 14);
    }
    if (typeA == QGEMM_QUATERNION && typeB == QGEMM_QUATERNION) {
        if constexpr (sizeof(T) == 8) s = qgemm_d(opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, stream);
        else s = qgemm_s(opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, 6, stream);
        return s == QGEMM_OK ? s : fail(s, g_bad_arg + 2);
    }
    qg::MixedDesc d{};
    const bool right = typeB == QGEMM_QUATERNION;   // quaternion is the right factor: out = C^T
    d.f32 = sizeof(T) == 4;
    d.right = right;
    d.C = C;
    d.ldc = ldc;
    d.K = (int)K;
    if (!right) {
        d.X = A; d.ldx = lda; d.P = (int)M; d.xt = op_transposes(opA); d.conjX = op_conjugates(opA);
        d.Y = B; d.ldy = ldb; d.Q = (int)N; d.yt = op_transposes(opB); d.conjY = typeB == QGEMM_COMPLEX && op_conjugates(opB);
        d.kc = typeB;
    } else {
        d.X = B; d.ldx = ldb; d.P = (int)N; d.xt = !op_transposes(opB); d.conjX = op_conjugates(opB);
        d.Y = A; d.ldy = lda; d.Q = (int)M; d.yt = !op_transposes(opA); d.conjY = typeA == QGEMM_COMPLEX && op_conjugates(opA);
        d.kc = typeA;
    }
    for (int i = 0; i < 4; ++i) {
        d.alpha[i] = alpha[i];
        d.beta[i] = beta[i];
    }
    if (!qg::mixed_ld_supported(d.ldx, d.ldy, d.xt, d.yt, d.kc, (int)rb))
        return fail(QGEMM_ERR_UNSUPPORTED, right ? 12 : 10);
    if (qg::launch_qgemm_mixed_f64(d, stream) != hipSuccess) return QGEMM_ERR_HIP;
    return QGEMM_OK;
}

}  // namespace

extern "C" {

const char *qgemm_status_string(int status)
{
    switch (status) {
    case QGEMM_OK: return "QGEMM_OK";
    case QGEMM_ERR_INVALID_ARG: return "QGEMM_ERR_INVALID_ARG";
    case QGEMM_ERR_MISALIGNED: return "QGEMM_ERR_MISALIGNED";
    case QGEMM_ERR_HIP: return "QGEMM_ERR_HIP";
    case QGEMM_ERR_ALLOC: return "QGEMM_ERR_ALLOC";
    case QGEMM_ERR_UNSUPPORTED: return "QGEMM_ERR_UNSUPPORTED";
    default: return "QGEMM_ERR_UNKNOWN";
    }
}

int qgemm_last_invalid_arg(void) { return g_bad_arg; }

qgemm_status_t qgemm_d(int opA, int opB, int64_t M, int64_t N, int64_t K, const double *alpha,
                       const double *A, int64_t lda, const double *B, int64_t ldb, const double *beta,
                       double *C, int64_t ldc, void *stream)
{
    qgemm_status_t s = validate(opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, 32, 32);
    if (s != QGEMM_OK || M == 0 || N == 0) return s;
    if (!qg::f64_ld_supported(lda, ldb, op_transposes(opA), op_transposes(opB)))
        return fail(QGEMM_ERR_UNSUPPORTED, op_transposes(opA) ? 8 : 10);
    const auto d = make_desc<double>(opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    if (qg::launch_qgemm_f64(d, static_cast<hipStream_t>(stream)) != hipSuccess) return QGEMM_ERR_HIP;
    return QGEMM_OK;
}

static qgemm_status_t split_common(int opA, int opB, int64_t M, int64_t N, int64_t K, const double *alpha,
                                   const float *A, int64_t lda, const float *B, int64_t ldb, const double *beta,
                                   float *C, double *C64, int64_t ldc, int split_terms, void *stream)
{
    const void *Cv = C64 ? static_cast<const void *>(C64) : static_cast<const void *>(C);
    qgemm_status_t s = validate(opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, Cv, ldc, C64 ? 32 : 16, 16);
    if (s != QGEMM_OK) return s;
    if (split_terms == 0) split_terms = 6;
    if (split_terms != 3 && split_terms != 6 && split_terms != 9) return fail(QGEMM_ERR_INVALID_ARG, 14);
    if (M == 0 || N == 0) return QGEMM_OK;
    if (!qg::split_ld_supported(lda, ldb, op_transposes(opA), op_transposes(opB)))
        return fail(QGEMM_ERR_UNSUPPORTED, op_transposes(opA) ? 8 : 10);
    auto d = make_desc<float>(opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    if (qg::launch_qgemm_bf16x3(d, C64, split_terms, qg::kSplitPanel, static_cast<hipStream_t>(stream)) != hipSuccess)
        return QGEMM_ERR_HIP;
    return QGEMM_OK;
}

qgemm_status_t qgemm_s(int opA, int opB, int64_t M, int64_t N, int64_t K, const double *alpha,
                       const float *A, int64_t lda, const float *B, int64_t ldb, const double *beta,
                       float *C, int64_t ldc, int split_terms, void *stream)
{
    return split_common(opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, nullptr, ldc, split_terms, stream);
}

qgemm_status_t qgemm_s_c64(int opA, int opB, int64_t M, int64_t N, int64_t K, const double *alpha,
                           const float *A, int64_t lda, const float *B, int64_t ldb, const double *beta,
                           double *C, int64_t ldc, int split_terms, void *stream)
{
    return split_common(opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, nullptr, C, ldc, split_terms, stream);
}

qgemm_status_t qgemm_ex_d(int opA, int opB, int64_t M, int64_t N, int64_t K, const double *alpha_left,
                          const double *alpha_mid, const double *alpha_right, const double *A, int64_t lda,
                          const double *B, int64_t ldb, const double *beta_left, const double *beta_right,
                          double *C, int64_t ldc, void *stream)
{
    return ex_impl<double>(opA, opB, M, N, K, alpha_left, alpha_mid, alpha_right, A, lda, B, ldb, beta_left,
                           beta_right, C, ldc, 6, static_cast<hipStream_t>(stream));
}

qgemm_status_t qgemm_ex_s(int opA, int opB, int64_t M, int64_t N, int64_t K, const double *alpha_left,
                          const double *alpha_mid, const double *alpha_right, const float *A, int64_t lda,
                          const float *B, int64_t ldb, const double *beta_left, const double *beta_right,
                          float *C, int64_t ldc, int split_terms, void *stream)
{
    return ex_impl<float>(opA, opB, M, N, K, alpha_left, alpha_mid, alpha_right, A, lda, B, ldb, beta_left,
                          beta_right, C, ldc, split_terms, static_cast<hipStream_t>(stream));
}

qgemm_status_t qherk_d(int uplo, int trans, int64_t N, int64_t K, double alpha, const double *A, int64_t lda,
                       double beta, double *C, int64_t ldc, void *stream)
{
    return herk_impl<double>(uplo, trans, N, K, alpha, A, lda, beta, C, ldc, 6, static_cast<hipStream_t>(stream));
}

qgemm_status_t qherk_s(int uplo, int trans, int64_t N, int64_t K, double alpha, const float *A, int64_t lda,
                       double beta, float *C, int64_t ldc, int split_terms, void *stream)
{
    return herk_impl<float>(uplo, trans, N, K, alpha, A, lda, beta, C, ldc, split_terms,
                            static_cast<hipStream_t>(stream));
}

qgemm_status_t qtrmm_d(int side, int uplo, int trans, int diag, int64_t M, int64_t N, const double *alpha,
                       const double *A, int64_t lda, const double *B, int64_t ldb, double *C, int64_t ldc,
                       void *stream)
{
    return trmm_impl<double>(side, uplo, trans, diag, M, N, alpha, A, lda, B, ldb, C, ldc, 6,
                             static_cast<hipStream_t>(stream));
}

qgemm_status_t qtrmm_s(int side, int uplo, int trans, int diag, int64_t M, int64_t N, const double *alpha,
                       const float *A, int64_t lda, const float *B, int64_t ldb, float *C, int64_t ldc,
                       int split_terms, void *stream)
{
    return trmm_impl<float>(side, uplo, trans, diag, M, N, alpha, A, lda, B, ldb, C, ldc, split_terms,
                            static_cast<hipStream_t>(stream));
}

qgemm_status_t qgemm_mixed_d(int typeA, int typeB, int opA, int opB, int64_t M, int64_t N, int64_t K,
                             const double *alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                             const double *beta, double *C, int64_t ldc, void *stream)
{
    return mixed_impl<double>(typeA, typeB, opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                              static_cast<hipStream_t>(stream));
}

qgemm_status_t qgemm_mixed_s(int typeA, int typeB, int opA, int opB, int64_t M, int64_t N, int64_t K,
                             const double *alpha, const float *A, int64_t lda, const float *B, int64_t ldb,
                             const double *beta, float *C, int64_t ldc, void *stream)
{
    return mixed_impl<float>(typeA, typeB, opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                             static_cast<hipStream_t>(stream));
}

qgemm_status_t qaxpy_d(int64_t n, const double *alpha, const double *x, int64_t incx, double *y, int64_t incy,
                       void *stream)
{
    return axpy_impl<double>(n, alpha, x, incx, y, incy, static_cast<hipStream_t>(stream));
}

qgemm_status_t qaxpy_s(int64_t n, const double *alpha, const float *x, int64_t incx, float *y, int64_t incy,
                       void *stream)
{
    return axpy_impl<float>(n, alpha, x, incx, y, incy, static_cast<hipStream_t>(stream));
}

qgemm_status_t qdot_d(int conj, int64_t n, const double *x, int64_t incx, const double *y, int64_t incy,
                      double *result, double *work, void *stream)
{
    return dot_impl<double>(conj, n, x, incx, y, incy, result, work, static_cast<hipStream_t>(stream));
}

qgemm_status_t qdot_s(int conj, int64_t n, const float *x, int64_t incx, const float *y, int64_t incy,
                      float *result, double *work, void *stream)
{
    return dot_impl<float>(conj, n, x, incx, y, incy, result, work, static_cast<hipStream_t>(stream));
}

qgemm_status_t qdot_d_noalloc(int conj, int64_t n, const double *x, int64_t incx, const double *y, int64_t incy,
                              double *result, void *stream)
{
    return dot_impl<double>(conj, n, x, incx, y, incy, result, nullptr, static_cast<hipStream_t>(stream), true);
}

qgemm_status_t qgemv_d(int trans, int64_t M, int64_t N, const double *alpha, const double *A, int64_t lda,
                       const double *x, int64_t incx, const double *beta, double *y, int64_t incy, void *stream)
{
    return gemv_impl<double>(trans, M, N, alpha, A, lda, x, incx, beta, y, incy, static_cast<hipStream_t>(stream));
}

qgemm_status_t qgemv_s(int trans, int64_t M, int64_t N, const double *alpha, const float *A, int64_t lda,
                       const float *x, int64_t incx, const double *beta, float *y, int64_t incy, void *stream)
{
    return gemv_impl<float>(trans, M, N, alpha, A, lda, x, incx, beta, y, incy, static_cast<hipStream_t>(stream));
}

qgemm_status_t qgemm_backward_d(int opA, int opB, int64_t M, int64_t N, int64_t K, const double *alpha,
                                const double *A, int64_t lda, const double *B, int64_t ldb, const double *G,
                                int64_t ldg, const double *beta, double *dA, int64_t ldda, double *dB,
                                int64_t lddb, double *dC0, int64_t lddc0, void *stream)
{
    return backward_impl<double>(opA, opB, M, N, K, alpha, A, lda, B, ldb, G, ldg, beta, dA, ldda, dB, lddb, dC0,
                                 lddc0, 6, static_cast<hipStream_t>(stream));
}

qgemm_status_t qgemm_backward_s(int opA, int opB, int64_t M, int64_t N, int64_t K, const double *alpha,
                                const float *A, int64_t lda, const float *B, int64_t ldb, const float *G,
                                int64_t ldg, const double *beta, float *dA, int64_t ldda, float *dB, int64_t lddb,
                                float *dC0, int64_t lddc0, int split_terms, void *stream)
{
    return backward_impl<float>(opA, opB, M, N, K, alpha, A, lda, B, ldb, G, ldg, beta, dA, ldda, dB, lddb, dC0,
                                lddc0, split_terms, static_cast<hipStream_t>(stream));
}

int64_t qgemm_last_invalid_problem(void) { return g_bad_problem; }

struct qgemm_plan_s {
    qg::GroupedPlan *impl;
};

qgemm_status_t qgemm_batched_plan_create(qgemm_plan_t *plan, int dtype, int opA, int opB, int64_t count,
                                         const qgemm_problem_t *problems, const double *alpha,
                                         const double *beta, int split_terms, int tile_class)
{
    g_bad_arg = 0;
    g_bad_problem = -1;
    if (!plan) return fail(QGEMM_ERR_INVALID_ARG, 1);
    *plan = nullptr;
    if (dtype != QGEMM_DTYPE_F32 && dtype != QGEMM_DTYPE_F64) return fail(QGEMM_ERR_INVALID_ARG, 2);
    const bool f64 = dtype == QGEMM_DTYPE_F64;
    if (!valid_op(opA)) return fail(QGEMM_ERR_INVALID_ARG, 3);
    if (!valid_op(opB)) return fail(QGEMM_ERR_INVALID_ARG, 4);
    if (count < 0 || count > kMaxDim) return fail(QGEMM_ERR_INVALID_ARG, 5);
    if (count > 0 && !problems) return fail(QGEMM_ERR_INVALID_ARG, 6);
    if (!alpha) return fail(QGEMM_ERR_INVALID_ARG, 7);
    if (!beta) return fail(QGEMM_ERR_INVALID_ARG, 8);
    if (f64) {
        if (split_terms != 0) return fail(QGEMM_ERR_INVALID_ARG, 9);   // FP64 plans do not split
        if (tile_class >= qg::kGroupedClassesF64) return fail(QGEMM_ERR_INVALID_ARG, 10);
    } else {
        if (split_terms == 0) split_terms = 6;
        if (split_terms != 3 && split_terms != 6 && split_terms != 9) return fail(QGEMM_ERR_INVALID_ARG, 9);
        if (tile_class >= qg::kGroupedClasses) return fail(QGEMM_ERR_INVALID_ARG, 10);
    }
    const uintptr_t esz = f64 ? 32 : 16;   // bytes per quaternion
    for (int64_t i = 0; i < count; ++i) {
        const qgemm_problem_t &q = problems[i];
        qgemm_status_t s = validate(opA, opB, q.M, q.N, q.K, alpha, q.A, q.lda, q.B, q.ldb, beta, q.C, q.ldc, esz,
                                    (int64_t)esz);
        if (s != QGEMM_OK) {
            g_bad_problem = i;
            return s;
        }
    }
    qg::GroupedPlan *impl = nullptr;
    int rc;
    try {   // host containers may throw; nothing crosses the C ABI
        rc = qg::grouped_plan_create(&impl, f64, op_transposes(opA), op_transposes(opB), op_conjugates(opA),
                                     op_conjugates(opB), split_terms, alpha, beta, count, problems, tile_class);
    } catch (const std::bad_alloc &) {
        return QGEMM_ERR_ALLOC;
    } catch (...) {
        return QGEMM_ERR_HIP;
    }
    if (rc < 0) {
        g_bad_problem = -(int64_t)rc - 1;
        return fail(QGEMM_ERR_UNSUPPORTED, 6);
    }
    if (rc != QGEMM_OK) return fail((qgemm_status_t)rc, rc == QGEMM_ERR_UNSUPPORTED ? 6 : 0);
    qgemm_plan_s *h = new (std::nothrow) qgemm_plan_s{impl};
    if (!h) {
        qg::grouped_plan_destroy(impl);
        return QGEMM_ERR_ALLOC;
    }
    *plan = h;
    return QGEMM_OK;
}

qgemm_status_t qgemm_batched_set_tile_table(const unsigned char *table)
{
    g_bad_arg = 0;
    if (table)
        for (int i = 0; i < qg::kTileTableCells; ++i)
            if (table[i] >= qg::kGroupedClasses) return fail(QGEMM_ERR_INVALID_ARG, 1);
    qg::grouped_set_table(table);
    return QGEMM_OK;
}

qgemm_status_t qgemm_batched_get_tile_table(unsigned char *table)
{
    g_bad_arg = 0;
    if (!table) return fail(QGEMM_ERR_INVALID_ARG, 1);
    qg::grouped_get_table(table);
    return QGEMM_OK;
}

qgemm_status_t qgemm_batched_run(qgemm_plan_t plan, void *stream)
{
    g_bad_arg = 0;
    if (!plan || !plan->impl) return fail(QGEMM_ERR_INVALID_ARG, 1);
    return (qgemm_status_t)qg::grouped_plan_run(plan->impl, static_cast<hipStream_t>(stream));
}

qgemm_status_t qgemm_batched_plan_destroy(qgemm_plan_t plan)
{
    if (!plan) return QGEMM_OK;
    qg::grouped_plan_destroy(plan->impl);
    delete plan;
    return QGEMM_OK;
}

qgemm_status_t qgemm_batched_plan_info(qgemm_plan_t plan, int64_t *work_items, int *grid, int64_t *class_counts)
{
    g_bad_arg = 0;
    if (!plan || !plan->impl) return fail(QGEMM_ERR_INVALID_ARG, 1);
    qg::grouped_plan_info(plan->impl, work_items, grid, class_counts);
    return QGEMM_OK;
}

}  // extern "C"
