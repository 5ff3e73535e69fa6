// Elementwise kernel of the gradient: Y <- s X for an M x N quaternion
// matrix (s multiplies from the left, Hamilton product Eq. quaternion_prod).
// HBM-bound: one 16- or 32-byte read and write per element; a grid-stride
// loop over elements with consecutive threads on consecutive rows.
#include "qgemm_internal.hpp"

namespace qg {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void scale_left_kernel(const T *X, int64_t ldx, T *Y, int64_t ldy, int M, int N,
                                                         T s0, T s1, T s2, T s3)
{
    const T s[4] = {s0, s1, s2, s3};
    const int64_t total = (int64_t)M * N;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t nu = t / M;
        const int64_t mu = t - nu * M;
        const T *x = X + 4 * (mu + nu * ldx);
        const T xv[4] = {x[0], x[1], x[2], x[3]};
        T o[4];
        qmul(s, xv, o);
        T *y = Y + 4 * (mu + nu * ldy);
        y[0] = o[0];
        y[1] = o[1];
        y[2] = o[2];
        y[3] = o[3];
    }
}

}  // namespace

template <typename T>
hipError_t launch_scale_left(const T *X, int64_t ldx, T *Y, int64_t ldy, int M, int N, const double s[4],
                             hipStream_t stream)
{
    const int64_t total = (int64_t)M * N;
    if (total <= 0) return hipSuccess;
    const int64_t want = (total + 255) / 256;
    const unsigned blocks = (unsigned)(want < 8192 ? want : 8192);
    hipLaunchKernelGGL(scale_left_kernel<T>, dim3(blocks), dim3(256), 0, stream, X, ldx, Y, ldy, M, N, (T)s[0],
                       (T)s[1], (T)s[2], (T)s[3]);
    return hipGetLastError();
}

template hipError_t launch_scale_left<float>(const float *, int64_t, float *, int64_t, int, int, const double *,
                                             hipStream_t);
template hipError_t launch_scale_left<double>(const double *, int64_t, double *, int64_t, int, int, const double *,
                                              hipStream_t);

}  // namespace qg
