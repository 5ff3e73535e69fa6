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
 *     quaternion (32 bytes for double, 16 bytes for float).  A matrix may
 *     span at most 2^62 bytes ((ld (cols - 1) + rows) elements); the GEMM
 *     tiles further address one K-tile of an operand with 32-bit offsets,
 *     which bounds the leading dimension of a transposed A or of B with op
 *     N / R (about 2^20 quaternions in double, 2^21 in float).  Beyond these
 *     limits a call returns QGEMM_ERR_UNSUPPORTED.
 *   - Quick returns: M == 0 or N == 0 does nothing.  K == 0 or alpha == 0
 *     (all four components) computes C <- beta * C without reading A or B.
 *     beta == 0 (all four components) never reads C, so NaN/Inf there do not
 *     propagate.
 *   - Aliasing: an output must not overlap any array the call reads (C vs A
 *     and B; each gradient vs A, B, G and the other gradients).  Checked from
 *     the address ranges the sizes and leading dimensions span:
 *     QGEMM_ERR_INVALID_ARG with the output's argument index.
 *   - Errors are returned as status codes; nothing aborts or throws across
 *     the ABI.  QGEMM_ERR_HIP means a HIP launch error was reported.
 *   - Threads and devices: calls from several host threads are safe; each
 *     call runs on the calling thread's current device (set up once per
 *     device on first use) and on the given stream, in stream order.
 *   - Graph capture: every entry point except qgemm_batched_plan_create and
 *     qgemm_batched_plan_destroy only launches kernels (no allocation, host
 *     copy, memset or synchronisation), so its work may be captured into a
 *     hipGraph and replayed; scalars are frozen into the captured launch.
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
    QGEMM_LOWER = 0,
    QGEMM_UPPER = 1
} qgemm_uplo_t;

typedef enum {
    QGEMM_REAL = 1,
    QGEMM_COMPLEX = 2,
    QGEMM_QUATERNION = 4
} qgemm_type_t;

typedef enum {
    QGEMM_SIDE_LEFT = 0,
    QGEMM_SIDE_RIGHT = 1
} qgemm_side_t;

typedef enum {
    QGEMM_NON_UNIT = 0,
    QGEMM_UNIT = 1
} qgemm_diag_t;

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

/*
 * qgemm_s -- FP32-stored quaternion GEMM as split-BF16 products on the BF16
 * matrix cores with FP32 accumulation (an extension of the paper's FP64
 * method, Sec. 4, to lower-precision matrix units).
 * Computes C <- alpha op(A) op(B) + beta C with A, B, C device arrays of
 * float.  Each FP32 component is split into three BF16 pieces (round to
 * nearest even on successive residuals); split_terms selects the piece
 * products formed: 3 (first order), 6 (default, all products down to 2^-16
 * relative) or 9 (all); 0 means 6.  Accumulation is FP32 in two levels (an
 * inner accumulator flushed every 64 quaternions of K).  alpha and beta are
 * applied in FP32.  Inputs must be finite with |x| below the BF16 overflow
 * threshold (about 3.39e38).
 * Arguments: 1 opA, 2 opB, 3 M, 4 N, 5 K, 6 alpha, 7 A, 8 lda, 9 B, 10 ldb,
 *            11 beta, 12 C, 13 ldc, 14 split_terms, 15 stream.
 */
qgemm_status_t qgemm_s(int opA, int opB, int64_t M, int64_t N, int64_t K,
                       const double *alpha, const float *A, int64_t lda,
                       const float *B, int64_t ldb, const double *beta,
                       float *C, int64_t ldc, int split_terms, void *stream);

/*
 * qgemm_s_c64 -- as qgemm_s, but C is an array of double: the accumulated
 * product is widened and alpha, beta and the update of C are done in FP64
 * (for callers that keep the result in double).  C must be 32-byte aligned
 * (one double quaternion); A and B, arrays of float, 16-byte aligned as in
 * qgemm_s.
 */
qgemm_status_t qgemm_s_c64(int opA, int opB, int64_t M, int64_t N, int64_t K,
                           const double *alpha, const float *A, int64_t lda,
                           const float *B, int64_t ldb, const double *beta,
                           double *C, int64_t ldc, int split_terms, void *stream);

/*
 * qgemm_ex_d / qgemm_ex_s -- general scalar placement.  Because quaternion
 * scalars do not commute with matrices, the left, right and middle scalar
 * products differ (Sec. 2.2: qQ, Qq and PqQ).  These calls compute
 *     C <- aL * ( sum_k op(A)_{mu k} * aM * op(B)_{k nu} ) * aR + bL * C * bR
 * with aL = alpha_left, aM = alpha_mid, aR = alpha_right, bL = beta_left,
 * bR = beta_right (host arrays of 4 doubles).  A NULL scalar takes its default:
 * the unit quaternion for aL, aM, aR and bR, zero for bL.  With aM = aR = bR =
 * unit this is qgemm_d / qgemm_s.  aM multiplies every element of op(B) (after
 * the op) from the left as the tile is staged; aR and bR are applied in the
 * epilogue.  Any of aL, aM, aR zero: the product is not formed (A, B not
 * read); bL zero: C is not read.  Precision as qgemm_d (FP64) and qgemm_s
 * (split-BF16, scalars applied in FP32; aM is applied to op(B) in FP32 before
 * the split).
 * Arguments: 1 opA, 2 opB, 3 M, 4 N, 5 K, 6 alpha_left, 7 alpha_mid,
 *   8 alpha_right, 9 A, 10 lda, 11 B, 12 ldb, 13 beta_left, 14 beta_right,
 *   15 C, 16 ldc, then (qgemm_ex_s only) 17 split_terms, then stream.
 */
qgemm_status_t qgemm_ex_d(int opA, int opB, int64_t M, int64_t N, int64_t K,
                          const double *alpha_left, const double *alpha_mid,
                          const double *alpha_right, const double *A, int64_t lda,
                          const double *B, int64_t ldb, const double *beta_left,
                          const double *beta_right, double *C, int64_t ldc, void *stream);
qgemm_status_t qgemm_ex_s(int opA, int opB, int64_t M, int64_t N, int64_t K,
                          const double *alpha_left, const double *alpha_mid,
                          const double *alpha_right, const float *A, int64_t lda,
                          const float *B, int64_t ldb, const double *beta_left,
                          const double *beta_right, float *C, int64_t ldc,
                          int split_terms, void *stream);

/*
 * qherk_d / qherk_s -- Hermitian rank-k update (one of the BLAS-3 operations
 * the paper's GEMM kernels are meant to serve, Sec. 3; quaternion
 * Hermiticity Q = Q^H, Sec. 2.2), in the BLAS HERK convention:
 *     trans = QGEMM_OP_N:  C <- alpha A A^H + beta C,   A is N x K
 *     trans = QGEMM_OP_C:  C <- alpha A^H A + beta C,   A is K x N
 * alpha and beta are real.  Only the triangle `uplo` (QGEMM_LOWER: mu >= nu,
 * QGEMM_UPPER: mu <= nu) of the N x N matrix C is read and written; the
 * vector part of each diagonal element is set to zero (a Hermitian matrix
 * has a real diagonal; the input's diagonal vector part is not used).
 * Quick returns: N == 0, or (alpha == 0 or K == 0) with beta == 1, leave C
 * untouched; beta == 0 never reads C.  About half the work of the GEMM.
 * Arguments: 1 uplo, 2 trans, 3 N, 4 K, 5 alpha, 6 A, 7 lda, 8 beta, 9 C,
 *   10 ldc, then (qherk_s only) 11 split_terms, then stream.
 */
qgemm_status_t qherk_d(int uplo, int trans, int64_t N, int64_t K, double alpha,
                       const double *A, int64_t lda, double beta, double *C, int64_t ldc,
                       void *stream);
qgemm_status_t qherk_s(int uplo, int trans, int64_t N, int64_t K, double alpha,
                       const float *A, int64_t lda, double beta, float *C, int64_t ldc,
                       int split_terms, void *stream);

/*
 * qtrmm_d / qtrmm_s -- triangular matrix multiply (the other BLAS-3
 * operation the paper's GEMM kernels are meant to serve, Sec. 3), in the BLAS
 * TRMM convention but out of place:
 *     side = QGEMM_SIDE_LEFT:   C <- alpha op(T) B,   T is M x M
 *     side = QGEMM_SIDE_RIGHT:  C <- alpha B op(T),   T is N x N
 * B and C are M x N (leading dimensions ldb, ldc >= max(1, M)); alpha is a
 * quaternion multiplying from the left, as in qgemm_d.  T is the triangle
 * `uplo` (QGEMM_LOWER: row >= column, QGEMM_UPPER: row <= column) of the
 * stored A (lda >= max(1, order of T)); A's other triangle is never read.
 * diag = QGEMM_UNIT: T's diagonal is the unit quaternion and A's diagonal is
 * not read.  trans is any op (N, T, C or R) applied to T.  C is written, not
 * read, and must not overlap A or B (checked: QGEMM_ERR_INVALID_ARG on C).
 * alpha == 0: C <- 0 and A, B are not read.  Each output tile walks only the
 * K-range the triangle covers, so the work is about half that of qgemm_d.
 * Arguments: 1 side, 2 uplo, 3 trans, 4 diag, 5 M, 6 N, 7 alpha, 8 A,
 *   9 lda, 10 B, 11 ldb, 12 C, 13 ldc, then (qtrmm_s only) 14 split_terms,
 *   then stream.
 */
qgemm_status_t qtrmm_d(int side, int uplo, int trans, int diag, int64_t M, int64_t N,
                       const double *alpha, const double *A, int64_t lda,
                       const double *B, int64_t ldb, double *C, int64_t ldc, void *stream);
qgemm_status_t qtrmm_s(int side, int uplo, int trans, int diag, int64_t M, int64_t N,
                       const double *alpha, const float *A, int64_t lda,
                       const float *B, int64_t ldb, float *C, int64_t ldc,
                       int split_terms, void *stream);

/*
 * qgemm_mixed_d -- mixed-type GEMM (the quaternion-real and
 * quaternion-complex arithmetic the paper's library provides, Sec. 5):
 *     C <- alpha op(A) op(B) + beta C
 * with one of A, B real or complex and the other quaternion; C, alpha and
 * beta are quaternions (alpha, beta from the left).  typeA / typeB give the
 * element kind and so the reals per stored element: QGEMM_REAL (1 double),
 * QGEMM_COMPLEX (2 doubles, re then im), QGEMM_QUATERNION (4 doubles).  Leading
 * dimensions count elements.  A real x enters as x e0 and a complex z0 + z1 i
 * as z0 e0 + z1 e1 (Eq. complex_subalg, Eq. h_c_iso); op T transposes, C
 * conjugate-transposes, R conjugates (a no-op on a real operand, complex
 * conjugation on a complex one).  Both quaternion: same as qgemm_d.  Neither
 * quaternion: QGEMM_ERR_INVALID_ARG (argument 2).  The embedded operand is
 * never widened: a real operand costs 4 and a complex one 8 real
 * multiply-adds per element product (16 for quaternion x quaternion).
 * Alignment: one element of each operand (8, 16 or 32 bytes).  Quick returns
 * and beta == 0 / alpha == 0 rules as qgemm_d.
 * Arguments: 1 typeA, 2 typeB, 3 opA, 4 opB, 5 M, 6 N, 7 K, 8 alpha, 9 A,
 *   10 lda, 11 B, 12 ldb, 13 beta, 14 C, 15 ldc, then stream.
 */
qgemm_status_t qgemm_mixed_d(int typeA, int typeB, int opA, int opB, int64_t M, int64_t N, int64_t K,
                             const double *alpha, const double *A, int64_t lda,
                             const double *B, int64_t ldb, const double *beta,
                             double *C, int64_t ldc, void *stream);
/*
 * qgemm_mixed_s -- as qgemm_mixed_d with float storage (A, B, C arrays of
 * float; alignment 4, 8 or 16 bytes per element).  The elements are widened
 * exactly to double as they are staged and the products are formed in FP64,
 * so the only rounding beyond FP64 accumulation is the final store of C in
 * float.  Both operands quaternion: same as qgemm_s with 6 products.
 */
qgemm_status_t qgemm_mixed_s(int typeA, int typeB, int opA, int opB, int64_t M, int64_t N, int64_t K,
                             const double *alpha, const float *A, int64_t lda,
                             const float *B, int64_t ldb, const double *beta,
                             float *C, int64_t ldc, void *stream);

/*
 * Level-1/2 operations (the quaternion BLAS-1/2 subset the paper's library
 * provides, Sec. 5), BLAS conventions: vectors are n quaternions strided by
 * inc >= 1 elements (4 reals each); scalars are host arrays of 4 doubles
 * multiplying from the left; _d works on double, _s on float storage, and
 * both accumulate in double.  These operations read O(1) flops per byte and
 * are bound by HBM bandwidth.  Every reduction runs in a fixed order, so a
 * result is reproducible bit for bit.  Vectors / matrices must be aligned to
 * one quaternion (32 bytes double, 16 bytes float).
 *
 * qaxpy_d / qaxpy_s -- y_i <- alpha x_i + y_i, i < n.  alpha == 0 or n == 0:
 *   y untouched.  x and y may be the same vector (same pointer and inc) but
 *   must not overlap otherwise.
 *   Arguments: 1 n, 2 alpha, 3 x, 4 incx, 5 y, 6 incy, then stream.
 */
qgemm_status_t qaxpy_d(int64_t n, const double *alpha, const double *x, int64_t incx, double *y, int64_t incy,
                       void *stream);
qgemm_status_t qaxpy_s(int64_t n, const double *alpha, const float *x, int64_t incx, float *y, int64_t incy,
                       void *stream);

/*
 * qdot_d / qdot_s -- result <- sum_i x_i y_i (conj == 0) or sum_i conj(x_i) y_i
 *   (conj == 1), written to device memory `result` (4 reals of the storage
 *   type; n == 0 gives zero).  `work` is a device workspace of at least
 *   QGEMM_DOT_WORK_DOUBLES doubles (partial sums), owned by the caller and
 *   needed only when n > 0; calls that share it must not overlap.
 *   Arguments: 1 conj, 2 n, 3 x, 4 incx, 5 y, 6 incy, 7 result, 8 work, then
 *   stream.
 */
#define QGEMM_DOT_WORK_DOUBLES 4096
qgemm_status_t qdot_d(int conj, int64_t n, const double *x, int64_t incx, const double *y, int64_t incy,
                      double *result, double *work, void *stream);
qgemm_status_t qdot_s(int conj, int64_t n, const float *x, int64_t incx, const float *y, int64_t incy,
                      float *result, double *work, void *stream);

/*
 * qdot_d_noalloc -- qdot_d for callers that cannot allocate device memory or
 *   hold a workspace (code under hipGraph capture, tight serving loops,
 *   harnesses that forbid hipMalloc).  Same result, bit for bit, as qdot_d
 *   with a workspace: the same kernels, with their partial sums in a
 *   workspace of the library's own, a file-scope device array of
 *   QGEMM_DOT_WORK_DOUBLES doubles (32 KiB) per GPU, held until the process
 *   ends.  The call allocates nothing (no hipMalloc, hipFree or allocating
 *   library routine) and only launches kernels; its first call on a device
 *   looks the array's address up (hipGetSymbolAddress).  n is not limited by
 *   the array: the first pass writes at most 1024 partial sums whatever n.
 *   Every call on one GPU shares that GPU's array: calls that overlap on one
 *   GPU (other streams, other host threads) race and give undefined results;
 *   calls in stream order on one stream are safe.
 *   Arguments: 1 conj, 2 n, 3 x, 4 incx, 5 y, 6 incy, 7 result, then stream.
 */
qgemm_status_t qdot_d_noalloc(int conj, int64_t n, const double *x, int64_t incx, const double *y, int64_t incy,
                              double *result, void *stream);

/*
 * qgemv_d / qgemv_s -- y <- alpha op(A) x + beta y with A stored M x N
 *   (lda >= max(1, M)): op N or R gives x of N and y of M elements, op T or C
 *   x of M and y of N elements.  Quick returns (y untouched): M == 0, N == 0,
 *   or alpha == 0 with beta == 1.  beta == 0: y not read; alpha == 0: A and x
 *   not read.  y must not overlap A or x.
 *   Arguments: 1 trans, 2 M, 3 N, 4 alpha, 5 A, 6 lda, 7 x, 8 incx, 9 beta,
 *   10 y, 11 incy, then stream.
 */
qgemm_status_t qgemv_d(int trans, int64_t M, int64_t N, const double *alpha, const double *A, int64_t lda,
                       const double *x, int64_t incx, const double *beta, double *y, int64_t incy, void *stream);
qgemm_status_t qgemv_s(int trans, int64_t M, int64_t N, const double *alpha, const float *A, int64_t lda,
                       const float *x, int64_t incx, const double *beta, float *y, int64_t incy, void *stream);

/*
 * Grouped (batched) quaternion GEMM: many independent problems
 *   C_i <- alpha op(A_i) op(B_i) + beta C_i,  i = 0..count-1,
 * (Sec. 3.1, Eq. general_gemm, for each problem) with common ops, scalars
 * and element type, run as ONE persistent kernel launch.  This batching is
 * an extension beyond the paper.
 *   dtype QGEMM_DTYPE_F64: the arrays are double and every problem runs on
 *     the FP64 tile of qgemm_d (same arithmetic; one tile class, 32 x 64
 *     quaternions).  split_terms must be 0.
 *   dtype QGEMM_DTYPE_F32: the arrays are float and every problem runs on
 *     the split-BF16 tile of qgemm_s (split_terms as there).  The tile shape
 *     of each problem is chosen per size class from a table produced by the
 *     library's tile tuner (the analogue of the paper's autotuned caching
 *     parameters, Sec. 5).
 *
 * qgemm_batched_plan_create: validates every problem (as qgemm_d / qgemm_s
 *   do; on failure qgemm_last_invalid_arg() names the field -- 3 M, 4 N,
 *   5 K, 7 A, 8 lda, 9 B, 10 ldb, 12 C, 13 ldc, numbered as in those calls --
 *   and qgemm_last_invalid_problem() its index), builds the work table on
 *   the host and copies it to the current device (hipMalloc + synchronous
 *   copy: do NOT call it inside a stream capture).  tile_class < 0 uses the
 *   tuned table (FP32) or the one FP64 class; otherwise FP32 plans take
 *   0..3 (0 = 32x64, 1 = 64x32, 2 = 32x32, 3 = 16x64 quaternions) and FP64
 *   plans 0 (32x64) for every problem.  The plan keeps the problem pointers
 *   and sizes: the buffers must stay valid while the plan is run.
 *   Arguments: 1 plan, 2 dtype, 3 opA, 4 opB, 5 count, 6 problems, 7 alpha,
 *   8 beta, 9 split_terms, 10 tile_class.
 * qgemm_batched_run: enqueues the single launch on `stream`.  It allocates
 *   nothing, copies nothing and does not synchronise, so it may be captured
 *   into a hipGraph and replayed.  Must run on the device the plan was made
 *   on.  Problems whose C overlap, or overlap any A or B, give undefined
 *   results.
 * qgemm_batched_plan_destroy: frees the plan's device tables (synchronises
 *   the device).
 */
typedef enum {
    QGEMM_DTYPE_F32 = 0,
    QGEMM_DTYPE_F64 = 1
} qgemm_dtype_t;

typedef struct qgemm_problem_t {
    int64_t M, N, K;
    int64_t lda, ldb, ldc;
    const void *A;
    const void *B;
    void *C;
} qgemm_problem_t;

typedef struct qgemm_plan_s *qgemm_plan_t;

qgemm_status_t qgemm_batched_plan_create(qgemm_plan_t *plan, int dtype, int opA, int opB, int64_t count,
                                         const qgemm_problem_t *problems, const double *alpha,
                                         const double *beta, int split_terms, int tile_class);
qgemm_status_t qgemm_batched_run(qgemm_plan_t plan, void *stream);
qgemm_status_t qgemm_batched_plan_destroy(qgemm_plan_t plan);
/* Work items, grid size and tiles per class (array of 4; FP64 plans use
 * only the first) of a plan. */
qgemm_status_t qgemm_batched_plan_info(qgemm_plan_t plan, int64_t *work_items, int *grid,
                                       int64_t *class_counts);
/* Index of the problem that made the last plan creation on this thread fail, or -1. */
int64_t qgemm_last_invalid_problem(void);

/*
 * The tile table of FP32 plans: 32 tile classes (0..3) indexed
 * [M bucket][N bucket][K bucket] (row-major, M and N buckets 1-16, 17-32,
 * 33-64, 65+; K buckets 1-64, 65+).  The library's tuner (tune_tiles.py)
 * compiles the table it finds into the library; qgemm_batched_set_tile_table
 * installs another for the whole process (NULL restores the compiled-in one;
 * an entry above 3 is QGEMM_ERR_INVALID_ARG, argument 1) and affects plans
 * created afterwards (a plan copies the table in effect once, when it is
 * created); qgemm_batched_get_tile_table copies the table in effect into
 * table[32].  Both are thread-safe.
 */
qgemm_status_t qgemm_batched_set_tile_table(const unsigned char *table);
qgemm_status_t qgemm_batched_get_tile_table(unsigned char *table);

/*
 * Gradient of the real loss L = sum_{mu,nu} <G_{mu nu}, C_{mu nu}> (the
 * Euclidean inner product of the four components) for
 *     C = alpha op(A) op(B) + beta C0,
 * with respect to the stored A, B and C0 (an extension beyond the paper):
 *     d op(A) = conj(alpha) G op(B)^H,   d op(B) = op(A)^H (conj(alpha) G),
 *     dC0 = conj(beta) G,
 * mapped back through op (N: as is, T: transposed, C: conjugate-transposed,
 * R: conjugated).  dA (stored like A, leading dimension ldda), dB (like B,
 * lddb) and dC0 (M x N, lddc0) are overwritten; any of them may be NULL to
 * skip it.  G is M x N with leading dimension ldg.  alpha and beta are
 * constants (no gradient).  At most two GEMM launches and one elementwise
 * launch are enqueued; no workspace is allocated.
 * qgemm_backward_d runs in FP64; qgemm_backward_s on FP32 data through the
 * split-BF16 path (split_terms as in qgemm_s).
 * Arguments: 1 opA, 2 opB, 3 M, 4 N, 5 K, 6 alpha, 7 A, 8 lda, 9 B, 10 ldb,
 *   11 G, 12 ldg, 13 beta, 14 dA, 15 ldda, 16 dB, 17 lddb, 18 dC0, 19 lddc0,
 *   20 split_terms (qgemm_backward_s only), then stream.
 * Outputs must not overlap the inputs.
 */
qgemm_status_t qgemm_backward_d(int opA, int opB, int64_t M, int64_t N, int64_t K,
                                const double *alpha, const double *A, int64_t lda,
                                const double *B, int64_t ldb, const double *G, int64_t ldg,
                                const double *beta, double *dA, int64_t ldda,
                                double *dB, int64_t lddb, double *dC0, int64_t lddc0,
                                void *stream);
qgemm_status_t qgemm_backward_s(int opA, int opB, int64_t M, int64_t N, int64_t K,
                                const double *alpha, const float *A, int64_t lda,
                                const float *B, int64_t ldb, const float *G, int64_t ldg,
                                const double *beta, float *dA, int64_t ldda,
                                float *dB, int64_t lddb, float *dC0, int64_t lddc0,
                                int split_terms, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* QGEMM_H */
