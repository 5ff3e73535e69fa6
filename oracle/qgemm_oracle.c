/*
 * qgemm_oracle.c -- plain, slow, obviously correct CPU reference for quaternion
 * matrix multiplication.  TEST INFRASTRUCTURE ONLY: it is called by the test
 * suite, by the smoke check and by the CPU-baseline leg of the benchmark, and
 * never by the product path.  It shares no code, header, table or constant
 * with the GPU library.
 *
 * Everything is IEEE binary64.  Inputs stored in binary32 are widened exactly
 * by the caller before they reach this file.
 *
 * Notation follows Williams-Young & Li, "On the Efficacy and High-Performance
 * Implementation of Quaternion Matrix Multiplication":
 *   - a quaternion is q = q0 e0 + q1 e1 + q2 e2 + q3 e3, stored as the four
 *     contiguous reals [q0, q1, q2, q3]                     (Sec. 2.1, Eq. quaternion_def;
 *                                                          storage: Sec. 4)
 *   - the product is the Hamilton product                   (Sec. 2.1, Eq. quaternion_prod)
 *   - the conjugate negates the vector part                 (Sec. 2.1, Eq. quaternion_conj)
 *   - (Q^H)_{mu nu} = conj(Q_{nu mu}), Q^T plain transpose  (Sec. 2.2; notation section)
 *   - matrices are column-major                             (Sec. 3.1, Eq. general_gemm)
 *   - left scalar times a product: (qPQ)_{mu nu} = q * sum_k P_{mu k} Q_{k nu}
 *                                                          (Sec. 2.2, left scalar products)
 *   - GEMM: C = alpha A B + beta C, alpha and beta on the left
 *                                                          (Sec. 3.1, Eq. general_gemm; Alg. 1)
 *
 * op codes: 0 = N (as stored), 1 = T (transpose, no conjugation),
 *           2 = C (conjugate transpose), 3 = R (conjugate, no transpose).
 * The T/C reading of op() and the R op used by the gradient are readings
 * chosen here, not the paper's (the paper defines only ^T and ^H on matrices).
 *
 * Parity pins for every function live in tests/test_oracle_pins.py.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of OpenMP threads the oracle uses (<= 0: leave the runtime default). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Threads a parallel region of the oracle would use now. */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Hamilton product out = p q, written out term by term from Eq. quaternion_prod:
 *   scalar part : p0 q0 - sum_{i=1..3} p_i q_i
 *   vector part k: p0 q_k + p_k q0 + sum_{i,j} eps_{ijk} p_i q_j
 * with the Levi-Civita symbol eps_{123} = +1 (so e1 e2 = e3, Eq. quaternion_alg).
 * The eps sum for k = 1 is p2 q3 - p3 q2, for k = 2 is p3 q1 - p1 q3, for k = 3
 * is p1 q2 - p2 q1.  out may alias neither p nor q. */
void oracle_hamilton(const double *p, const double *q, double *out)
{
    out[0] = p[0] * q[0] - (p[1] * q[1] + p[2] * q[2] + p[3] * q[3]);
    out[1] = p[0] * q[1] + p[1] * q[0] + (p[2] * q[3] - p[3] * q[2]);
    out[2] = p[0] * q[2] + p[2] * q[0] + (p[3] * q[1] - p[1] * q[3]);
    out[3] = p[0] * q[3] + p[3] * q[0] + (p[1] * q[2] - p[2] * q[1]);
}

/* Quaternion conjugate, Eq. quaternion_conj. */
static void conj_q(const double *q, double *out)
{
    out[0] = q[0];
    out[1] = -q[1];
    out[2] = -q[2];
    out[3] = -q[3];
}

/* Materialise op(X) as a dense rows x cols column-major quaternion matrix
 * (leading dimension = rows).  X is the stored matrix with leading dimension
 * ldx; for op N/R it is rows x cols, for op T/C it is cols x rows. */
static double *materialise_op(int op, int64_t rows, int64_t cols,
                              const double *X, int64_t ldx)
{
    double *Y = (double *)malloc(sizeof(double) * 4 * (size_t)(rows * cols > 0 ? rows * cols : 1));
    if (!Y) return NULL;
    for (int64_t c = 0; c < cols; ++c) {
        for (int64_t r = 0; r < rows; ++r) {
            const double *src;
            if (op == 0 || op == 3) src = X + 4 * (r + c * ldx);   /* X_{r c}            */
            else                    src = X + 4 * (c + r * ldx);   /* X_{c r} (transpose) */
            double *dst = Y + 4 * (r + c * rows);
            if (op == 2 || op == 3) conj_q(src, dst);
            else memcpy(dst, src, 4 * sizeof(double));
        }
    }
    return Y;
}

/* C <- alpha * op(A) * op(B) + beta * C  over the quaternions.
 * op(A) is M x K, op(B) is K x N, C is M x N (leading dimension ldc).
 * Following the definition of the left scalar product, the sum over kappa is
 * formed first and alpha multiplies it from the left; beta multiplies the old
 * C from the left.  Loop order follows Alg. 1 (reference GEMM): columns nu of C
 * outermost, then kappa, then the rows mu of the column.  Columns are
 * independent, so they are split over OpenMP threads.
 * Semantics chosen here where the paper is silent (the BLAS
 * convention): when beta is exactly zero (all four components) the old C is
 * not read, so NaN/Inf in C do not propagate; when alpha is exactly zero or
 * K == 0 the product is not formed and A, B are not read, giving C <- beta C.
 * Returns 0 on success, -1 on allocation failure, -2 on a bad op code. */
int oracle_qgemm(int opA, int opB, int64_t M, int64_t N, int64_t K,
                 const double *alpha, const double *A, int64_t lda,
                 const double *B, int64_t ldb, const double *beta,
                 double *C, int64_t ldc)
{
    if (opA < 0 || opA > 3 || opB < 0 || opB > 3) return -2;
    if (M <= 0 || N <= 0) return 0;
    const int beta_zero = (beta[0] == 0.0 && beta[1] == 0.0 && beta[2] == 0.0 && beta[3] == 0.0);
    const int alpha_zero = (alpha[0] == 0.0 && alpha[1] == 0.0 && alpha[2] == 0.0 && alpha[3] == 0.0);
    if (alpha_zero) K = 0;
    double *opa = materialise_op(opA, M, K, A, lda);
    double *opb = materialise_op(opB, K, N, B, ldb);
    if (!opa || !opb) { free(opa); free(opb); return -1; }
    int failed = 0;
#pragma omp parallel
    {
        double *acc = (double *)malloc(sizeof(double) * 4 * (size_t)M);
        if (!acc) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t nu = 0; nu < N; ++nu) {
            if (!acc) continue;
            memset(acc, 0, sizeof(double) * 4 * (size_t)M);
            for (int64_t ka = 0; ka < K; ++ka) {
                const double *b = opb + 4 * (ka + nu * K);
                for (int64_t mu = 0; mu < M; ++mu) {
                    double t[4];
                    oracle_hamilton(opa + 4 * (mu + ka * M), b, t);
                    acc[4 * mu + 0] += t[0];
                    acc[4 * mu + 1] += t[1];
                    acc[4 * mu + 2] += t[2];
                    acc[4 * mu + 3] += t[3];
                }
            }
            for (int64_t mu = 0; mu < M; ++mu) {
                double *c = C + 4 * (mu + nu * ldc);
                double s[4], u[4] = {0.0, 0.0, 0.0, 0.0};
                oracle_hamilton(alpha, acc + 4 * mu, s);
                if (!beta_zero) oracle_hamilton(beta, c, u);
                c[0] = s[0] + u[0];
                c[1] = s[1] + u[1];
                c[2] = s[2] + u[2];
                c[3] = s[3] + u[3];
            }
        }
        free(acc);
    }
    free(opa);
    free(opb);
    return failed ? -1 : 0;
}

/* General scalar placement (Sec. 2.2, left, right and middle scalar products
 * (qQ)_{mu nu} = q Q_{mu nu}, (Qq)_{mu nu} = Q_{mu nu} q,
 * (PqQ)_{mu nu} = sum_k P_{mu k} q Q_{k nu}):
 *   C <- aL * ( sum_k op(A)_{mu k} * aM * op(B)_{k nu} ) * aR + bL * C * bR.
 * Each of aL, aM, aR, bR may be NULL, meaning the unit quaternion; bL may be
 * NULL, meaning zero.  Written as plain loops in the order of the formula:
 * for every output element the middle scalar multiplies op(B) from the left,
 * the product op(A) (aM op(B)) is summed over k, and the outer scalars are
 * applied on their sides.  Same quick-return rules as oracle_qgemm (bL zero:
 * C not read; aL or aM or aR zero, or K == 0: the sum is not formed). */
int oracle_qgemm_ex(int opA, int opB, int64_t M, int64_t N, int64_t K,
                    const double *aL, const double *aM, const double *aR,
                    const double *A, int64_t lda, const double *B, int64_t ldb,
                    const double *bL, const double *bR, double *C, int64_t ldc)
{
    static const double one[4] = {1.0, 0.0, 0.0, 0.0};
    static const double zero[4] = {0.0, 0.0, 0.0, 0.0};
    if (opA < 0 || opA > 3 || opB < 0 || opB > 3) return -2;
    if (M <= 0 || N <= 0) return 0;
    if (!aL) aL = one;
    if (!aM) aM = one;
    if (!aR) aR = one;
    if (!bL) bL = zero;
    if (!bR) bR = one;
    const int bz = (bL[0] == 0.0 && bL[1] == 0.0 && bL[2] == 0.0 && bL[3] == 0.0);
    const int az = (aL[0] == 0.0 && aL[1] == 0.0 && aL[2] == 0.0 && aL[3] == 0.0) ||
                   (aM[0] == 0.0 && aM[1] == 0.0 && aM[2] == 0.0 && aM[3] == 0.0) ||
                   (aR[0] == 0.0 && aR[1] == 0.0 && aR[2] == 0.0 && aR[3] == 0.0);
    if (az) K = 0;
    double *opa = materialise_op(opA, M, K, A, lda);
    double *opb = materialise_op(opB, K, N, B, ldb);
    if (!opa || !opb) { free(opa); free(opb); return -1; }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t nu = 0; nu < N; ++nu) {
        for (int64_t mu = 0; mu < M; ++mu) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            for (int64_t ka = 0; ka < K; ++ka) {
                double mb[4], t[4];
                oracle_hamilton(aM, opb + 4 * (ka + nu * K), mb);
                oracle_hamilton(opa + 4 * (mu + ka * M), mb, t);
                acc[0] += t[0]; acc[1] += t[1]; acc[2] += t[2]; acc[3] += t[3];
            }
            double l[4], r[4], u[4] = {0.0, 0.0, 0.0, 0.0}, w[4];
            oracle_hamilton(aL, acc, l);
            oracle_hamilton(l, aR, r);
            double *c = C + 4 * (mu + nu * ldc);
            if (!bz) {
                oracle_hamilton(bL, c, w);
                oracle_hamilton(w, bR, u);
            }
            c[0] = r[0] + u[0];
            c[1] = r[1] + u[1];
            c[2] = r[2] + u[2];
            c[3] = r[3] + u[3];
        }
    }
    free(opa);
    free(opb);
    return 0;
}

/* Hermitian rank-k update (the rank-k update the GEMM kernels serve, Sec. 3;
 * Hermitian: Q = Q^H, Sec. 2.2), a reading in the BLAS HERK convention:
 *   trans = 0 (N): C <- alpha A A^H + beta C,  A is n x k (leading dim lda)
 *   trans = 2 (C): C <- alpha A^H A + beta C,  A is k x n
 * alpha and beta are real.  Only the triangle uplo (0 lower: mu >= nu,
 * 1 upper: mu <= nu) of C is read or written.  The diagonal of a Hermitian
 * matrix is real: its vector part is set to zero in the result (C's diagonal
 * vector part is not read).  beta == 0: C is not read; alpha == 0 or k == 0:
 * the product is not formed, and with beta == 1 as well C is left as it is
 * (the BLAS quick return).  Plain loops over the triangle. */
int oracle_qherk(int uplo, int trans, int64_t n, int64_t k, double alpha, const double *A, int64_t lda,
                 double beta, double *C, int64_t ldc)
{
    if ((uplo != 0 && uplo != 1) || (trans != 0 && trans != 2)) return -2;
    if (n <= 0) return 0;
    if ((alpha == 0.0 || k == 0) && beta == 1.0) return 0;   /* nothing to update (BLAS quick return) */
    if (alpha == 0.0) k = 0;
    double *opa = materialise_op(trans, n, k, A, lda);   /* op(A): n x k */
    if (!opa) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t nu = 0; nu < n; ++nu) {
        const int64_t lo = uplo == 0 ? nu : 0, hi = uplo == 0 ? n : nu + 1;
        for (int64_t mu = lo; mu < hi; ++mu) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            for (int64_t ka = 0; ka < k; ++ka) {
                double cb[4], t[4];
                conj_q(opa + 4 * (nu + ka * n), cb);
                oracle_hamilton(opa + 4 * (mu + ka * n), cb, t);
                acc[0] += t[0]; acc[1] += t[1]; acc[2] += t[2]; acc[3] += t[3];
            }
            double *c = C + 4 * (mu + nu * ldc);
            for (int i = 0; i < 4; ++i) c[i] = alpha * acc[i] + (beta == 0.0 ? 0.0 : beta * c[i]);
            if (mu == nu) c[1] = c[2] = c[3] = 0.0;
        }
    }
    free(opa);
    return 0;
}

/* Triangular matrix multiply (the XTRMM-like operation the GEMM kernels
 * serve, Sec. 3), a reading in the BLAS TRMM convention, written out of
 * place:
 *   side = 0 (left):  C <- alpha op(T) B,  T is M x M
 *   side = 1 (right): C <- alpha B op(T),  T is N x N
 * B and C are M x N; alpha multiplies from the left (as in Eq. general_gemm).
 * T is the triangle uplo (0 lower: r >= c, 1 upper: r <= c) of the stored A;
 * the other triangle of A is not read.  diag = 1 (unit): T's diagonal is the
 * unit quaternion and A's diagonal is not read.  op in {N, T, C, R} as for
 * oracle_qgemm.  C is not read; alpha == 0: C <- 0 and neither A nor B is
 * read.  Steps: form T densely, form op(T), then the plain triple sum.
 * C must not overlap A or B.  Returns 0, -1 (allocation) or -2 (bad code). */
int oracle_qtrmm(int side, int uplo, int trans, int diag, int64_t M, int64_t N,
                 const double *alpha, const double *A, int64_t lda,
                 const double *B, int64_t ldb, double *C, int64_t ldc)
{
    if ((side != 0 && side != 1) || (uplo != 0 && uplo != 1) || trans < 0 || trans > 3 ||
        (diag != 0 && diag != 1))
        return -2;
    if (M <= 0 || N <= 0) return 0;
    const int alpha_zero = (alpha[0] == 0.0 && alpha[1] == 0.0 && alpha[2] == 0.0 && alpha[3] == 0.0);
    if (alpha_zero) {
        for (int64_t nu = 0; nu < N; ++nu)
            memset(C + 4 * nu * ldc, 0, sizeof(double) * 4 * (size_t)M);
        return 0;
    }
    const int64_t n = side == 0 ? M : N;
    double *T = (double *)calloc(4 * (size_t)(n * n), sizeof(double));
    if (!T) return -1;
    for (int64_t c = 0; c < n; ++c)
        for (int64_t r = 0; r < n; ++r) {
            double *t = T + 4 * (r + c * n);
            if (r == c && diag == 1) t[0] = 1.0;
            else if (uplo == 0 ? r >= c : r <= c) memcpy(t, A + 4 * (r + c * lda), 4 * sizeof(double));
        }
    double *opt = materialise_op(trans, n, n, T, n);
    free(T);
    if (!opt) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t nu = 0; nu < N; ++nu) {
        for (int64_t mu = 0; mu < M; ++mu) {
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            const int64_t K = side == 0 ? M : N;
            for (int64_t ka = 0; ka < K; ++ka) {
                double t[4];
                if (side == 0) oracle_hamilton(opt + 4 * (mu + ka * n), B + 4 * (ka + nu * ldb), t);
                else           oracle_hamilton(B + 4 * (mu + ka * ldb), opt + 4 * (ka + nu * n), t);
                acc[0] += t[0]; acc[1] += t[1]; acc[2] += t[2]; acc[3] += t[3];
            }
            oracle_hamilton(alpha, acc, C + 4 * (mu + nu * ldc));
        }
    }
    free(opt);
    return 0;
}

/* Mixed-type GEMM (the quaternion-real and quaternion-complex arithmetic of
 * Sec. 5): one operand is a real or complex matrix, embedded into the
 * quaternions by x -> x e0 and z = z0 + z1 i -> z0 e0 + z1 e1 (the complex
 * subalgebra of Eq. complex_subalg and the map Eq. h_c_iso); then
 * C <- alpha op(A) op(B) + beta C exactly as oracle_qgemm.  typeA, typeB
 * give the reals per stored element: 1 real, 2 complex (re, im
 * interleaved), 4 quaternion; leading dimensions count elements.  op T
 * transposes, C conjugate-transposes (complex conjugate = quaternion
 * conjugate of the embedding), R conjugates.  Returns 0, -1 (allocation) or
 * -2 (bad code). */
static double *embed(int type, int op, int64_t rows, int64_t cols, const double *X, int64_t ldx)
{
    /* stored dimensions of X for this op */
    const int64_t sr = (op == 0 || op == 3) ? rows : cols, sc = (op == 0 || op == 3) ? cols : rows;
    double *Q = (double *)calloc(4 * (size_t)(sr * sc > 0 ? sr * sc : 1), sizeof(double));
    if (!Q) return NULL;
    for (int64_t c = 0; c < sc; ++c)
        for (int64_t r = 0; r < sr; ++r)
            for (int k = 0; k < type; ++k)
                Q[4 * (r + c * sr) + k] = X[type * (r + c * ldx) + k];
    return Q;
}

int oracle_qgemm_mixed(int typeA, int typeB, int opA, int opB, int64_t M, int64_t N, int64_t K,
                       const double *alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                       const double *beta, double *C, int64_t ldc)
{
    const int okA = typeA == 1 || typeA == 2 || typeA == 4, okB = typeB == 1 || typeB == 2 || typeB == 4;
    if (!okA || !okB || opA < 0 || opA > 3 || opB < 0 || opB > 3) return -2;
    if (M <= 0 || N <= 0) return 0;
    double *Aq = embed(typeA, opA, M, K, A, lda);
    double *Bq = embed(typeB, opB, K, N, B, ldb);
    if (!Aq || !Bq) { free(Aq); free(Bq); return -1; }
    const int64_t la = (opA == 0 || opA == 3) ? M : K, lb = (opB == 0 || opB == 3) ? K : N;
    const int rc = oracle_qgemm(opA, opB, M, N, K, alpha, Aq, la > 0 ? la : 1, Bq, lb > 0 ? lb : 1, beta, C, ldc);
    free(Aq);
    free(Bq);
    return rc;
}

/* Level-1/2 operations of the quaternion BLAS (the library scope of Sec. 5),
 * as plain loops in the BLAS conventions; vectors are strided by inc >= 1
 * elements, scalars multiply from the left as in Eq. general_gemm.
 *   qaxpy: y_i <- alpha x_i + y_i
 *   qdot : r = sum_i x_i y_i, or sum_i conj(x_i) y_i when conj != 0
 *   qgemv: y <- alpha op(A) x + beta y, A stored M x N; op(A) is M x N (N, R)
 *          or N x M (T, C); beta == 0: y not read; alpha == 0: A, x not read.
 * Returns 0, or -2 on a bad argument. */
int oracle_qaxpy(int64_t n, const double *alpha, const double *x, int64_t incx, double *y, int64_t incy)
{
    if (incx < 1 || incy < 1) return -2;
    for (int64_t i = 0; i < n; ++i) {
        double t[4];
        oracle_hamilton(alpha, x + 4 * i * incx, t);
        for (int c = 0; c < 4; ++c) y[4 * i * incy + c] += t[c];
    }
    return 0;
}

int oracle_qdot(int conj, int64_t n, const double *x, int64_t incx, const double *y, int64_t incy,
                double *result)
{
    if (incx < 1 || incy < 1) return -2;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) {
        double xi[4], t[4];
        if (conj) conj_q(x + 4 * i * incx, xi);
        else memcpy(xi, x + 4 * i * incx, sizeof xi);
        oracle_hamilton(xi, y + 4 * i * incy, t);
        for (int c = 0; c < 4; ++c) acc[c] += t[c];
    }
    memcpy(result, acc, sizeof acc);
    return 0;
}

int oracle_qgemv(int trans, int64_t M, int64_t N, const double *alpha, const double *A, int64_t lda,
                 const double *x, int64_t incx, const double *beta, double *y, int64_t incy)
{
    if (trans < 0 || trans > 3 || incx < 1 || incy < 1) return -2;
    const int64_t rows = (trans == 0 || trans == 3) ? M : N, cols = (trans == 0 || trans == 3) ? N : M;
    if (rows <= 0) return 0;
    const int alpha_zero = alpha[0] == 0.0 && alpha[1] == 0.0 && alpha[2] == 0.0 && alpha[3] == 0.0;
    const int beta_zero = beta[0] == 0.0 && beta[1] == 0.0 && beta[2] == 0.0 && beta[3] == 0.0;
    double *opa = materialise_op(trans, rows, alpha_zero ? 0 : cols, A, lda);
    if (!opa) return -1;
    for (int64_t r = 0; r < rows; ++r) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t c = 0; c < (alpha_zero ? 0 : cols); ++c) {
            double t[4];
            oracle_hamilton(opa + 4 * (r + c * rows), x + 4 * c * incx, t);
            for (int k = 0; k < 4; ++k) acc[k] += t[k];
        }
        double *yr = y + 4 * r * incy;
        double s[4], u[4] = {0.0, 0.0, 0.0, 0.0};
        oracle_hamilton(alpha, acc, s);
        if (!beta_zero) oracle_hamilton(beta, yr, u);
        for (int k = 0; k < 4; ++k) yr[k] = s[k] + u[k];
    }
    free(opa);
    return 0;
}

/* Gradient of the real loss L = sum_{mu nu} <G_{mu nu}, C_{mu nu}> (the
 * Euclidean inner product of the four components) for
 *   C = alpha op(A) op(B) + beta C0.
 * Derivation (a reading chosen here; the paper has no gradient): for one
 * term, <g, alpha a b> = Re(conj(g) alpha a b) is linear in a and in b, and
 * cycling the real part gives
 *   dL/d op(A)_{mu k} = sum_nu  conj(alpha) G_{mu nu} conj(op(B)_{k nu})
 *   dL/d op(B)_{k nu} = sum_mu  conj(op(A)_{mu k}) conj(alpha) G_{mu nu}
 *   dL/d C0_{mu nu}   = conj(beta) G_{mu nu}.
 * The gradient of the stored operand follows from op: N -> same matrix,
 * T -> its transpose, C -> its conjugate transpose, R -> its conjugate.
 * Any of dA, dB, dC0 may be NULL (not computed).  Written as explicit loops:
 * no blocking, no shared code with oracle_qgemm beyond the scalar product.
 * Returns 0, -1 (allocation) or -2 (bad op). */
int oracle_qgemm_backward(int opA, int opB, int64_t M, int64_t N, int64_t K,
                          const double *alpha, const double *A, int64_t lda,
                          const double *B, int64_t ldb, const double *G, int64_t ldg,
                          const double *beta,
                          double *dA, int64_t ldda, double *dB, int64_t lddb,
                          double *dC0, int64_t lddc0)
{
    if (opA < 0 || opA > 3 || opB < 0 || opB > 3) return -2;
    double ca[4], cb[4];
    conj_q(alpha, ca);
    conj_q(beta, cb);
    double *opa = materialise_op(opA, M, K, A, lda);
    double *opb = materialise_op(opB, K, N, B, ldb);
    if (!opa || !opb) { free(opa); free(opb); return -1; }
    if (dA && M > 0 && K > 0) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t ka = 0; ka < K; ++ka) {
            for (int64_t mu = 0; mu < M; ++mu) {
                double acc[4] = {0.0, 0.0, 0.0, 0.0};
                for (int64_t nu = 0; nu < N; ++nu) {
                    double cbq[4], t[4], u[4];
                    conj_q(opb + 4 * (ka + nu * K), cbq);
                    oracle_hamilton(G + 4 * (mu + nu * ldg), cbq, t);
                    oracle_hamilton(ca, t, u);
                    acc[0] += u[0]; acc[1] += u[1]; acc[2] += u[2]; acc[3] += u[3];
                }
                /* acc is dL/d op(A)_{mu ka}; place it in the stored layout */
                double *dst;
                if (opA == 0 || opA == 3) dst = dA + 4 * (mu + ka * ldda);
                else                      dst = dA + 4 * (ka + mu * ldda);
                if (opA == 2 || opA == 3) conj_q(acc, dst);
                else memcpy(dst, acc, sizeof acc);
            }
        }
    }
    if (dB && K > 0 && N > 0) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t nu = 0; nu < N; ++nu) {
            for (int64_t ka = 0; ka < K; ++ka) {
                double acc[4] = {0.0, 0.0, 0.0, 0.0};
                for (int64_t mu = 0; mu < M; ++mu) {
                    double caq[4], t[4], u[4];
                    conj_q(opa + 4 * (mu + ka * M), caq);
                    oracle_hamilton(ca, G + 4 * (mu + nu * ldg), t);
                    oracle_hamilton(caq, t, u);
                    acc[0] += u[0]; acc[1] += u[1]; acc[2] += u[2]; acc[3] += u[3];
                }
                double *dst;
                if (opB == 0 || opB == 3) dst = dB + 4 * (ka + nu * lddb);
                else                      dst = dB + 4 * (nu + ka * lddb);
                if (opB == 2 || opB == 3) conj_q(acc, dst);
                else memcpy(dst, acc, sizeof acc);
            }
        }
    }
    if (dC0) {
        for (int64_t nu = 0; nu < N; ++nu)
            for (int64_t mu = 0; mu < M; ++mu)
                oracle_hamilton(cb, G + 4 * (mu + nu * ldg), dC0 + 4 * (mu + nu * lddc0));
    }
    free(opa);
    free(opb);
    return 0;
}
