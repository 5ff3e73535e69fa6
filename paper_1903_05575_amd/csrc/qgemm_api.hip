// C-ABI layer of libqgemm.so: argument validation (host only, before any HIP
// call), quick returns, and dispatch to the kernels.  See include/qgemm.h.
#include "qgemm_internal.hpp"

#include "../../include/qgemm.h"

#include <stdint.h>

namespace {

thread_local int g_bad_arg = 0;

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

// Validate a GEMM call.  Argument numbering follows the public signatures:
// 1 opA, 2 opB, 3 M, 4 N, 5 K, 6 alpha, 7 A, 8 lda, 9 B, 10 ldb, 11 beta,
// 12 C, 13 ldc.  `align` is the byte size of one quaternion.
qgemm_status_t validate(int opA, int opB, int64_t M, int64_t N, int64_t K, const double *alpha,
                        const void *A, int64_t lda, const void *B, int64_t ldb, const double *beta,
                        const void *C, int64_t ldc, uintptr_t align)
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
    if (reads_ab && !A) return fail(QGEMM_ERR_INVALID_ARG, 7);
    if (reads_ab && !B) return fail(QGEMM_ERR_INVALID_ARG, 9);
    if (!C) return fail(QGEMM_ERR_INVALID_ARG, 12);
    if (reads_ab && (reinterpret_cast<uintptr_t>(A) % align)) return fail(QGEMM_ERR_MISALIGNED, 7);
    if (reads_ab && (reinterpret_cast<uintptr_t>(B) % align)) return fail(QGEMM_ERR_MISALIGNED, 9);
    if (reinterpret_cast<uintptr_t>(C) % align) return fail(QGEMM_ERR_MISALIGNED, 12);
    // 32-bit tile grid and element offsets computed in 64 bits: nothing more to check.
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
    for (int i = 0; i < 4; ++i) {
        d.alpha[i] = alpha[i];
        d.beta[i] = beta[i];
        d.bscale[i] = i == 0 ? 1.0 : 0.0;
    }
    return d;
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
    qgemm_status_t s = validate(opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, 32);
    if (s != QGEMM_OK || M == 0 || N == 0) return s;
    const auto d = make_desc<double>(opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    if (qg::launch_qgemm_f64(d, static_cast<hipStream_t>(stream)) != hipSuccess) return QGEMM_ERR_HIP;
    return QGEMM_OK;
}

static qgemm_status_t split_common(int opA, int opB, int64_t M, int64_t N, int64_t K, const double *alpha,
                                   const float *A, int64_t lda, const float *B, int64_t ldb, const double *beta,
                                   float *C, double *C64, int64_t ldc, int split_terms, void *stream)
{
    const void *Cv = C64 ? static_cast<const void *>(C64) : static_cast<const void *>(C);
    qgemm_status_t s = validate(opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, Cv, ldc, C64 ? 32 : 16);
    if (s != QGEMM_OK) return s;
    if (split_terms == 0) split_terms = 6;
    if (split_terms != 3 && split_terms != 6 && split_terms != 9) return fail(QGEMM_ERR_INVALID_ARG, 14);
    if (M == 0 || N == 0) return QGEMM_OK;
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

}  // extern "C"
