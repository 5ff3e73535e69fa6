/* Plain C99 user of the library: includes only include/qgemm.h, links
 * libqgemm.so, and drives calls that the host-side validation rejects before
 * any HIP call (so it runs without a GPU).  Prints one line per check. */
#include <stdint.h>
#include <stdio.h>

#include "qgemm.h"

static int failures = 0;

static void expect(const char *what, qgemm_status_t got, qgemm_status_t want, int arg)
{
    const int ok = got == want && (want == QGEMM_OK || qgemm_last_invalid_arg() == arg);
    printf("%s %s: %s arg %d\n", ok ? "ok" : "FAIL", what, qgemm_status_string(got), qgemm_last_invalid_arg());
    failures += !ok;
}

int main(void)
{
    const double one[4] = {1.0, 0.0, 0.0, 0.0};
    double *A = (double *)(uintptr_t)(1ull << 40), *B = (double *)(uintptr_t)(2ull << 40);
    double *C = (double *)(uintptr_t)(3ull << 40);
    expect("qgemm_d bad opA", qgemm_d(9, QGEMM_OP_N, 4, 4, 4, one, A, 4, B, 4, one, C, 4, NULL),
           QGEMM_ERR_INVALID_ARG, 1);
    expect("qgemm_d lda", qgemm_d(QGEMM_OP_T, QGEMM_OP_N, 4, 4, 8, one, A, 4, B, 8, one, C, 4, NULL),
           QGEMM_ERR_INVALID_ARG, 8);
    expect("qgemm_d empty", qgemm_d(QGEMM_OP_N, QGEMM_OP_N, 0, 4, 4, one, NULL, 1, NULL, 4, one, NULL, 1, NULL),
           QGEMM_OK, 0);
    expect("qgemm_s split terms", qgemm_s(QGEMM_OP_N, QGEMM_OP_C, 4, 4, 4, one, (float *)A, 4, (float *)B, 4, one,
                                          (float *)C, 4, 5, NULL), QGEMM_ERR_INVALID_ARG, 14);
    expect("qherk_d uplo", qherk_d(7, QGEMM_OP_N, 4, 4, 1.0, A, 4, 0.0, C, 4, NULL), QGEMM_ERR_INVALID_ARG, 1);
    expect("qtrmm_d side", qtrmm_d(2, QGEMM_LOWER, QGEMM_OP_N, QGEMM_NON_UNIT, 4, 4, one, A, 4, B, 4, C, 4, NULL),
           QGEMM_ERR_INVALID_ARG, 1);
    expect("qgemm_mixed_d types", qgemm_mixed_d(QGEMM_REAL, QGEMM_COMPLEX, QGEMM_OP_N, QGEMM_OP_N, 4, 4, 4, one, A, 4,
                                                B, 4, one, C, 4, NULL), QGEMM_ERR_INVALID_ARG, 2);
    expect("qaxpy_d incx", qaxpy_d(4, one, A, 0, B, 1, NULL), QGEMM_ERR_INVALID_ARG, 4);
    expect("qdot_d work", qdot_d(1, 4, A, 1, B, 1, C, NULL, NULL), QGEMM_ERR_INVALID_ARG, 8);
    expect("qgemv_d misaligned A", qgemv_d(QGEMM_OP_N, 4, 4, one, (double *)((char *)A + 8), 4, B, 1, one, C, 1,
                                           NULL), QGEMM_ERR_MISALIGNED, 5);
    expect("qgemm_backward_d lddc0", qgemm_backward_d(QGEMM_OP_N, QGEMM_OP_N, 4, 4, 4, one, A, 4, B, 4, C, 4, one,
                                                      NULL, 1, NULL, 1, A, 3, NULL), QGEMM_ERR_INVALID_ARG, 19);
    qgemm_plan_t plan = NULL;
    expect("plan count", qgemm_batched_plan_create(&plan, QGEMM_DTYPE_F64, QGEMM_OP_N, QGEMM_OP_N, -1, NULL, one,
                                                   one, 0, -1), QGEMM_ERR_INVALID_ARG, 5);
    expect("tile table NULL", qgemm_batched_get_tile_table(NULL), QGEMM_ERR_INVALID_ARG, 1);
    expect("qdot_d_noalloc incx", qdot_d_noalloc(0, 4, A, 0, B, 1, C, NULL), QGEMM_ERR_INVALID_ARG, 4);
    printf("dot workspace %d doubles\n", QGEMM_DOT_WORK_DOUBLES);
    return failures ? 1 : 0;
}
