/*
 * qgemm.h -- C ABI of the MI355X (gfx950) quaternion GEMM library libqgemm.so.
 *
 * Operation (Williams-Young & Li, Sec. 3.1, Eq. general_gemm, over the
 * quaternions of Sec. 2):
 *
 *     C <- alpha * op(A) * op(B) + beta * C
 *
 * where the product is the Hamilton product (Sec. 2.1, Eq. quaternion_prod),
 * the matrix product is (PQ)_{mu nu} = sum_k P_{mu k} Q_{k nu}, and the
 * scalars alpha and beta multiply from the LEFT (Sec. 2.2, left scalar
 * products; Sec. 3.1 notes alpha may not be moved across a quaternion
 * product).  op(A) is M x K, op(B) is K x N, C is M x N.
 *
 * Storage (Sec. 3.1 column-major; Sec. 4 quaternion = four contiguous reals):
 *   element (mu, nu) of a matrix X with leading dimension ldx occupies the
 *   four reals X[4*(mu + nu*ldx) + c], c = 0..3 = (q0, q1, q2, q3).
 *   Leading dimensions are counted in quaternions, not reals.
 *
 * op codes (the paper defines ^T and the conjugate transpose ^H,
 * Sec. 2.2; the R code is this library's conjugate-without-transpose):
 *   QGEMM_OP_N  op(X) = X                 stored rows x cols = op rows x cols
 *   QGEMM_OP_T  op(X) = X^T (no conj)     stored = cols x rows
 *   QGEMM_OP_C  op(X) = X^H = conj(X)^T   stored = cols x rows
 *   QGEMM_OP_R  op(X) = conj(X)           stored = rows x cols
 *
 * Common conventions for every entry point below:
 *   - Matrix pointers are DEVICE pointers owned by the caller.  The library
 *     keeps no reference to them once the stream-ordered work is done.
 *   - alpha, beta (and any other scalar) are HOST pointers to 4 doubles
 *     (q0..q3), read during the call and passed to the kernel by value.
 *   - stream is a hipStream_t (NULL = the default stream).  Every call is
 *     asynchronous with respect to the host: it validates, enqueues and
 *     returns.  Results are visible after the stream is synchronised.
 *   - Validation happens on the host before any HIP call.  A rejected call
 *     enqueues nothing and sets a thread-local 1-based argument index
 *     readable with qgemm_last_invalid_arg().
 *   - Requirements: M, N, K >= 0 and < 2^31; ld of a stored operand >=
 *     max(1, its stored rows); ldc >= max(1, M); base pointers aligned to one
 *     quaternion (32 bytes for double, 16 bytes for float).
 *   - Quick returns: M == 0 or N == 0 does nothing.  K == 0 or alpha == 0
 *     (all four components) computes C <- beta * C without reading A or B.
 *     beta == 0 (all four components) never reads C, so NaN/Inf there do not
 *     propagate.
 *   - Aliasing: C must not overlap A or B.
 *   - Errors are returned as status codes; nothing aborts or throws across
 *     the ABI.  QGEMM_ERR_HIP means a HIP launch error was reported.
 */
#ifndef QGEMM_H
#define QGEMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QGEMM_OP_N = 0,
    QGEMM_OP_T = 1,
    QGEMM_OP_C = 2,
    QGEMM_OP_R = 3
} qgemm_op_t;

typedef enum {
    QGEMM_OK = 0,
    QGEMM_ERR_INVALID_ARG = 1,
    QGEMM_ERR_MISALIGNED = 2,
    QGEMM_ERR_HIP = 3,
    QGEMM_ERR_ALLOC = 4,
    QGEMM_ERR_UNSUPPORTED = 5
} qgemm_status_t;

/* Human-readable name of a status code (static storage, never NULL). */
const char *qgemm_status_string(int status);

/* 1-based index of the argument that made the last call on this thread
 * return QGEMM_ERR_INVALID_ARG or QGEMM_ERR_MISALIGNED; 0 if none. */
int qgemm_last_invalid_arg(void);

/*
 * qgemm_d -- binary64 quaternion GEMM on FP64 MFMA.
 * Computes C <- alpha op(A) op(B) + beta C (Sec. 3.1, Eq. general_gemm)
 * with every real multiply-add in binary64 and binary64 accumulation.
 * A, B, C: device arrays of double as described above.
 * Arguments (1-based index used by qgemm_last_invalid_arg):
 *   1 opA, 2 opB, 3 M, 4 N, 5 K, 6 alpha, 7 A, 8 lda, 9 B, 10 ldb,
 *   11 beta, 12 C, 13 ldc, 14 stream.
 */
qgemm_status_t qgemm_d(int opA, int opB, int64_t M, int64_t N, int64_t K,
                       const double *alpha, const double *A, int64_t lda,
                       const double *B, int64_t ldb, const double *beta,
                       double *C, int64_t ldc, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* QGEMM_H */
