// Internal declarations shared by the kernels and the C-ABI layer of
// libqgemm.so.  Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "../../include/qgemm.h"
#include "qgemm_device.hpp"

namespace qg {

// Quaternion-level description of one GEMM launch, already validated.
// Pointers are device pointers to interleaved (q0,q1,q2,q3) elements.
//   opA_t / opB_t : the stored operand is transposed (op T or C)
//   conjA / conjB : op conjugates (op C or R)
//   bscale        : optional left scalar s applied to every element of op(B),
//                   i.e. the product op(A) (s op(B)) (the "middle scalar"
//                   form P q Q of Sec. 2.2)
//   alpha_r, beta_r : scalars multiplying from the right (the Q q form of
//                   Sec. 2.2), applied in the epilogue when has_right
//   store_t / store_conj : write the result transposed and/or conjugated
//                   (used by the gradient to map d op(X) back to dX)
template <typename T>
struct GemmDesc {
    const T *A;
    const T *B;
    T *C;
    int64_t lda, ldb, ldc;
    int M, N, K;
    bool opA_t, conjA, opB_t, conjB;
    bool has_bscale, store_t, store_conj;
    bool has_right;        // alpha_r / beta_r are not both the unit quaternion
    int uplo;              // 0: full C; 1: only mu >= nu (lower); 2: only mu <= nu (upper)
    bool herm_diag;        // zero the vector part of diagonal results (Hermitian output)
    int tri;               // 0: none; 1: op(A) is triangular (K == M); 2: op(B) is triangular (K == N)
    bool tri_lower;        // that triangular operand is zero above its diagonal (after the op)
    bool tri_unit;         // its diagonal is the unit quaternion and is not read
    double alpha[4];
    double beta[4];
    double bscale[4];
    double alpha_r[4];     // right scalars: C <- alpha acc alpha_r + beta C beta_r
    double beta_r[4];
};

// Raise the dynamic LDS limit of kernel `kern` to `bytes` on the current
// device, once per device: the attribute is per device, so a process that
// drives several GPUs sets it on each; `done` holds one bit per device
// ordinal and makes later launches free.  Safe to call from several threads.
inline hipError_t ensure_dynamic_lds(const void *kern, int bytes, std::atomic<uint64_t> &done)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = (dev >= 0 && dev < 64) ? (1ull << dev) : 0ull;
    if (bit && (done.load(std::memory_order_acquire) & bit)) return hipSuccess;
    e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e == hipSuccess && bit) done.fetch_or(bit, std::memory_order_acq_rel);
    return e;
}

// Compute units of the current device, cached per device ordinal (0 if the
// query fails).
inline int device_cus()
{
    static std::atomic<int> cache[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (dev >= 0 && dev < 64) {
        const int c = cache[dev].load(std::memory_order_relaxed);
        if (c > 0) return c;
    }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (dev >= 0 && dev < 64) cache[dev].store(cus, std::memory_order_relaxed);
    return cus;
}

// Launch helpers (return a hipError_t from the launch).
hipError_t launch_qgemm_f64(const GemmDesc<double> &d, hipStream_t stream);
// Split-BF16 path for FP32 operands.  nterms in {3, 6, 9}; panel = kappa
// length of the inner FP32 accumulation.  When c64 is non-null the result
// (and the beta term) is written to that FP64 array instead of d.C.
hipError_t launch_qgemm_bf16x3(const GemmDesc<float> &d, double *c64, int nterms, int panel, hipStream_t stream);
constexpr int kSplitPanel = 64;
// Leading dimensions the FP64 tiles can address with 32-bit in-tile byte
// offsets (64 x 64 x 8 quaternion tiles of 32 bytes; below 2^31 bytes).
inline bool f64_ld_supported(int64_t lda, int64_t ldb, bool ta, bool tb)
{
    const int64_t lim = (int64_t)1 << 31;
    const int64_t fa = 32 * (ta ? (64 * lda + 8) : (8 * lda + 64));
    const int64_t fb = 32 * (tb ? (8 * ldb + 64) : (64 * ldb + 8));
    return fa < lim && fb < lim;
}

// Leading dimensions the split-BF16 tiles can address with 32-bit in-tile
// offsets (64 x 64 x 16 quaternion tiles; below 2^31 bytes).
inline bool split_ld_supported(int64_t lda, int64_t ldb, bool ta, bool tb)
{
    const int64_t lim = (int64_t)1 << 31;
    const int64_t fa = 16 * (ta ? (64 * lda + 16) : (16 * lda + 64));
    const int64_t fb = 16 * (tb ? (16 * ldb + 64) : (64 * ldb + 16));
    return fa < lim && fb < lim;
}
// One mixed-type FP64 launch (qgemm_mixed_f64.hip): out = X . Y with X a
// quaternion operand (P x K after its op) and Y a real (kc = 1) or complex
// (kc = 2, re/im interleaved) operand (K x Q after its op); out is C, or C^T
// when `right` (the quaternion is the right factor of C = op(A) op(B)).
struct MixedDesc {
    const void *X;         // double or float (f32), as all three arrays
    const void *Y;
    void *C;
    bool f32;              // storage is float (arithmetic is FP64 either way)
    int64_t ldx, ldy, ldc;
    int P, Q, K;
    int kc;
    bool right;
    bool xt;               // X stored with kappa contiguous: X[kappa + p ldx], else X[p + kappa ldx]
    bool yt;               // Y stored with q contiguous: Y[q + kappa ldy], else Y[kappa + q ldy]
    bool conjX, conjY;     // conjugate X (quaternion) / Y (complex) as read
    double alpha[4];
    double beta[4];
};
bool mixed_ld_supported(int64_t ldx, int64_t ldy, bool xt, bool yt, int kc, int real_bytes);
hipError_t launch_qgemm_mixed_f64(const MixedDesc &d, hipStream_t stream);

// Level-1/2 launches (qblas_l12.hip).  The dot product uses at most
// kDotParts partial sums of 4 doubles in the caller's workspace.
constexpr int kDotParts = 1024;
template <typename T>
hipError_t launch_qaxpy(int64_t n, const double *alpha, const T *x, int64_t incx, T *y, int64_t incy,
                        hipStream_t stream);
template <typename T>
hipError_t launch_qdot(bool conj, int64_t n, const T *x, int64_t incx, const T *y, int64_t incy, T *result,
                       double *work, hipStream_t stream);
// Device address (on the current device) and size in doubles of the
// library's own dot-product workspace, a file-scope device array.
hipError_t dot_scratch(double **out, int *capacity);
template <typename T>
hipError_t launch_qgemv(int trans, int M, int N, const double *alpha, const T *A, int64_t lda, const T *x,
                        int64_t incx, const double *beta, T *y, int64_t incy, hipStream_t stream);

// Grouped (batched) plans, FP32 (split-BF16 tiles) or FP64; see qgemm_grouped.hip.
struct GroupedPlan;
constexpr int kGroupedClasses = 4;      // tile classes of FP32 plans
constexpr int kGroupedClassesF64 = 1;   // tile classes of FP64 plans
constexpr int kTileTableCells = 32;     // [M bucket 4][N bucket 4][K bucket 2]
void grouped_set_table(const unsigned char *t);   // nullptr: the compiled-in table
void grouped_get_table(unsigned char *t);
int grouped_plan_create(GroupedPlan **out, bool f64, bool ta, bool tb, bool ca, bool cb, int nterms,
                        const double alpha[4], const double beta[4], int64_t count, const ::qgemm_problem_t *probs,
                        int force_class);
int grouped_plan_run(const GroupedPlan *pl, hipStream_t stream);
void grouped_plan_destroy(GroupedPlan *pl);
void grouped_plan_info(const GroupedPlan *pl, int64_t *nitems, int *grid, int64_t *class_count);

// Y <- s X elementwise (left scalar), M x N quaternions.
template <typename T>
hipError_t launch_scale_left(const T *X, int64_t ldx, T *Y, int64_t ldy, int M, int N, const double s[4],
                             hipStream_t stream);

}  // namespace qg
