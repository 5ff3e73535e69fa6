// Level-1/2 quaternion BLAS on gfx950: axpy, dot / dotc, gemv.
//
// These operations do O(1) flops per element they read, so they are bound by
// HBM bandwidth, not by the matrix cores: the kernels are written for
// coalesced 16-byte accesses and enough bytes in flight, and accumulate in
// FP64 whatever the storage type (the arithmetic is free at this intensity).
// Scalars multiply from the left (as in Eq. general_gemm); products keep the
// operand order of the definition (Hamilton product, Eq. quaternion_prod).
// Every reduction is done in a fixed order, so results are reproducible run
// to run.
#include "qgemm_internal.hpp"

namespace qg {
namespace {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;

template <typename T>
__device__ __forceinline__ void load_q(const T *p, double q[4])
{
    if constexpr (sizeof(T) == 8) {
        const d2 a = reinterpret_cast<const d2 *>(p)[0], b = reinterpret_cast<const d2 *>(p)[1];
        q[0] = a.x; q[1] = a.y; q[2] = b.x; q[3] = b.y;
    } else {
        const f4 a = *reinterpret_cast<const f4 *>(p);
        q[0] = a.x; q[1] = a.y; q[2] = a.z; q[3] = a.w;
    }
}

template <typename T>
__device__ __forceinline__ void store_q(T *p, const double q[4])
{
    if constexpr (sizeof(T) == 8) {
        reinterpret_cast<d2 *>(p)[0] = (d2){q[0], q[1]};
        reinterpret_cast<d2 *>(p)[1] = (d2){q[2], q[3]};
    } else {
        *reinterpret_cast<f4 *>(p) = (f4){(float)q[0], (float)q[1], (float)q[2], (float)q[3]};
    }
}

__device__ __forceinline__ void conj_inplace(double q[4])
{
    q[1] = -q[1]; q[2] = -q[2]; q[3] = -q[3];
}

struct Scalars {
    double alpha[4];
    double beta[4];
};

// y_i <- alpha x_i + y_i; each thread takes elements i and i + stride per
// iteration, so four loads are in flight before the first store
template <typename T>
__global__ __launch_bounds__(NT) void qaxpy_kernel(int64_t n, Scalars s, const T *x, int64_t incx, T *y, int64_t incy)
{
    const int64_t stride = (int64_t)gridDim.x * NT;
    int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    for (; i + stride < n; i += 2 * stride) {
        double xv[2][4], yv[2][4];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            load_q(x + 4 * (i + u * stride) * incx, xv[u]);
            load_q(y + 4 * (i + u * stride) * incy, yv[u]);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            double t[4];
            qmul(s.alpha, xv[u], t);
            t[0] += yv[u][0]; t[1] += yv[u][1]; t[2] += yv[u][2]; t[3] += yv[u][3];
            store_q(y + 4 * (i + u * stride) * incy, t);
        }
    }
    if (i < n) {
        double xv[4], yv[4], t[4];
        load_q(x + 4 * i * incx, xv);
        load_q(y + 4 * i * incy, yv);
        qmul(s.alpha, xv, t);
        t[0] += yv[0]; t[1] += yv[1]; t[2] += yv[2]; t[3] += yv[3];
        store_q(y + 4 * i * incy, t);
    }
}

// Sum of 4-vectors over the block in a fixed order; thread 0 gets the total.
__device__ __forceinline__ void block_sum4(double v[4], double (*red)[4])
{
    const int t = threadIdx.x;
    red[t][0] = v[0]; red[t][1] = v[1]; red[t][2] = v[2]; red[t][3] = v[3];
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if (t < h) {
            red[t][0] += red[t + h][0]; red[t][1] += red[t + h][1];
            red[t][2] += red[t + h][2]; red[t][3] += red[t + h][3];
        }
        __syncthreads();
    }
    v[0] = red[0][0]; v[1] = red[0][1]; v[2] = red[0][2]; v[3] = red[0][3];
}

// dot pass 1: block b sums x_i y_i (conj(x_i) y_i) over i = b NT + t + k gridDim NT into
// work[4b..4b+3]; the per-thread order is fixed by n and the grid, so the result is reproducible
template <typename T, bool CONJ>
__global__ __launch_bounds__(NT) void qdot_partial_kernel(int64_t n, const T *x, int64_t incx, const T *y,
                                                          int64_t incy, double *work)
{
    __shared__ double red[NT][4];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * NT;
    int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    for (; i + stride < n; i += 2 * stride) {      // two elements, four loads in flight
        double xv[2][4], yv[2][4];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            load_q(x + 4 * (i + u * stride) * incx, xv[u]);
            load_q(y + 4 * (i + u * stride) * incy, yv[u]);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            double t[4];
            if (CONJ) conj_inplace(xv[u]);
            qmul(xv[u], yv[u], t);
            acc[0] += t[0]; acc[1] += t[1]; acc[2] += t[2]; acc[3] += t[3];
        }
    }
    if (i < n) {
        double xv[4], yv[4], t[4];
        load_q(x + 4 * i * incx, xv);
        load_q(y + 4 * i * incy, yv);
        if (CONJ) conj_inplace(xv);
        qmul(xv, yv, t);
        acc[0] += t[0]; acc[1] += t[1]; acc[2] += t[2]; acc[3] += t[3];
    }
    block_sum4(acc, red);
    if (threadIdx.x == 0) {
        double *w = work + 4 * blockIdx.x;
        w[0] = acc[0]; w[1] = acc[1]; w[2] = acc[2]; w[3] = acc[3];
    }
}

// dot pass 2: one block sums the `parts` partials in a fixed order into result
template <typename T>
__global__ __launch_bounds__(NT) void qdot_final_kernel(int parts, const double *work, T *result)
{
    __shared__ double red[NT][4];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < parts; b += NT) {
        acc[0] += work[4 * b]; acc[1] += work[4 * b + 1]; acc[2] += work[4 * b + 2]; acc[3] += work[4 * b + 3];
    }
    block_sum4(acc, red);
    if (threadIdx.x == 0) {
        result[0] = (T)acc[0]; result[1] = (T)acc[1]; result[2] = (T)acc[2]; result[3] = (T)acc[3];
    }
}

// gemv, op N / R: block = GR rows x GC column groups; thread (r, g) sums
// op(A)[mu][nu] x[nu] over nu = g, g + GC, ... of row mu = mu0 + r (GU
// columns in flight), then the column groups are summed in order
// g = 0, 1, ... in LDS.  The GR rows of one column are 512 contiguous bytes
// (FP64, 16 rows) or 128 (FP32, 8 rows).  Measured at 8192 x 8192: 8 columns
// in flight is best for FP64, 4 for FP32; 8-row FP32 blocks beat 16-row ones
// (twice as many blocks in flight) and 4- or 2-row ones (0.213 against 0.239
// and 0.291 ms, even with the blocks of one 128-byte line on one XCD); more
// threads per block were slower for both.
template <typename T>
struct GemvN {
    static constexpr int NTB = NT;
    static constexpr int GR = sizeof(T) == 8 ? 16 : 8;
    static constexpr int GC = NTB / GR;
    static constexpr int GU = sizeof(T) == 8 ? 8 : 4;
};

template <typename T, bool CONJ>
__global__ __launch_bounds__(GemvN<T>::NTB) void qgemv_n_kernel(int M, int ncols, Scalars s, const T *A,
                                                                int64_t lda, const T *x, int64_t incx,
                                                                bool beta_zero, T *y, int64_t incy)
{
    constexpr int GR = GemvN<T>::GR, GC = GemvN<T>::GC, GU = GemvN<T>::GU;
    __shared__ double red[GC][GR][4];
    const int r = threadIdx.x % GR, g = threadIdx.x / GR;
    const int mu = blockIdx.x * GR + r;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (mu < M) {
        const T *Ar = A + 4 * (int64_t)mu;
        int nu = g;
        for (; nu + (GU - 1) * GC < ncols; nu += GU * GC) {     // GU columns in flight per thread
            double a[GU][4], xv[GU][4];
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                load_q(Ar + 4 * (int64_t)(nu + u * GC) * lda, a[u]);
                load_q(x + 4 * (int64_t)(nu + u * GC) * incx, xv[u]);
            }
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                double t[4];
                if (CONJ) conj_inplace(a[u]);
                qmul(a[u], xv[u], t);
                acc[0] += t[0]; acc[1] += t[1]; acc[2] += t[2]; acc[3] += t[3];
            }
        }
        for (; nu < ncols; nu += GC) {
            double a[4], xv[4], t[4];
            load_q(Ar + 4 * (int64_t)nu * lda, a);
            load_q(x + 4 * (int64_t)nu * incx, xv);
            if (CONJ) conj_inplace(a);
            qmul(a, xv, t);
            acc[0] += t[0]; acc[1] += t[1]; acc[2] += t[2]; acc[3] += t[3];
        }
    }
    red[g][r][0] = acc[0]; red[g][r][1] = acc[1]; red[g][r][2] = acc[2]; red[g][r][3] = acc[3];
    __syncthreads();
    if (g == 0 && mu < M) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < GC; ++k) {
            v[0] += red[k][r][0]; v[1] += red[k][r][1]; v[2] += red[k][r][2]; v[3] += red[k][r][3];
        }
        double o[4];
        qmul(s.alpha, v, o);
        T *yr = y + 4 * (int64_t)mu * incy;
        if (!beta_zero) {
            double yv[4], u[4];
            load_q(yr, yv);
            qmul(s.beta, yv, u);
            o[0] += u[0]; o[1] += u[1]; o[2] += u[2]; o[3] += u[3];
        }
        store_q(yr, o);
    }
}

// gemv, op T / C: block b computes the TC outputs nu = TC b + j, j < TC:
// dot products of columns of A (conjugated for op C) with x, sharing each
// load of x.  The four waves take interleaved runs of 64 rows (wave w rows
// 64 w + 256 i + lane), each lane two runs per iteration; lanes are summed by
// a fixed butterfly and the four waves in order through LDS.
constexpr int TC = 4;
constexpr int TW = NT / 64;                     // waves per block

template <typename T, bool CONJ>
__global__ __launch_bounds__(NT) void qgemv_t_kernel(int N, int nrows, Scalars s, const T *A, int64_t lda,
                                                     const T *x, int64_t incx, bool beta_zero, T *y, int64_t incy)
{
    __shared__ double red[TW][TC][4];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nu0 = TC * blockIdx.x;
    int ncol = N - nu0;
    ncol = ncol < TC ? ncol : TC;
    const T *Ac[TC];
#pragma unroll
    for (int j = 0; j < TC; ++j) Ac[j] = A + 4 * (int64_t)(nu0 + (j < ncol ? j : 0)) * lda;   // spare columns repeat the first
    double acc[TC][4] = {};
    constexpr int RUN = 64 * TW;                 // rows covered by the block per run
    int mu = 64 * wave + lane;
    for (; mu + RUN < nrows; mu += 2 * RUN) {
        double a[2][TC][4], xv[2][4];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            load_q(x + 4 * (int64_t)(mu + RUN * u) * incx, xv[u]);
#pragma unroll
            for (int j = 0; j < TC; ++j) load_q(Ac[j] + 4 * (int64_t)(mu + RUN * u), a[u][j]);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int j = 0; j < TC; ++j) {
                double t[4];
                if (CONJ) conj_inplace(a[u][j]);
                qmul(a[u][j], xv[u], t);
                acc[j][0] += t[0]; acc[j][1] += t[1]; acc[j][2] += t[2]; acc[j][3] += t[3];
            }
    }
    if (mu < nrows) {
        double xv[4];
        load_q(x + 4 * (int64_t)mu * incx, xv);
#pragma unroll
        for (int j = 0; j < TC; ++j) {
            double a[4], t[4];
            load_q(Ac[j] + 4 * (int64_t)mu, a);
            if (CONJ) conj_inplace(a);
            qmul(a, xv, t);
            acc[j][0] += t[0]; acc[j][1] += t[1]; acc[j][2] += t[2]; acc[j][3] += t[3];
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int j = 0; j < TC; ++j)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[j][c] += __shfl_xor(acc[j][c], off);
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < TC; ++j)
#pragma unroll
            for (int c = 0; c < 4; ++c) red[wave][j][c] = acc[j][c];
    }
    __syncthreads();
    if (wave == 0 && lane < ncol) {             // lane j writes output nu0 + j
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (int w = 0; w < TW; ++w) {
            v[0] += red[w][lane][0]; v[1] += red[w][lane][1]; v[2] += red[w][lane][2]; v[3] += red[w][lane][3];
        }
        double o[4];
        qmul(s.alpha, v, o);
        T *yr = y + 4 * (int64_t)(nu0 + lane) * incy;
        if (!beta_zero) {
            double yv[4], u[4];
            load_q(yr, yv);
            qmul(s.beta, yv, u);
            o[0] += u[0]; o[1] += u[1]; o[2] += u[2]; o[3] += u[3];
        }
        store_q(yr, o);
    }
}

bool zero4(const double *q) { return q[0] == 0.0 && q[1] == 0.0 && q[2] == 0.0 && q[3] == 0.0; }

Scalars make_scalars(const double *alpha, const double *beta)
{
    Scalars s{};
    for (int i = 0; i < 4; ++i) {
        s.alpha[i] = alpha ? alpha[i] : 0.0;
        s.beta[i] = beta ? beta[i] : 0.0;
    }
    return s;
}

int grid_for(int64_t n, int cap)
{
    const int64_t b = (n + NT - 1) / NT;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace

template <typename T>
hipError_t launch_qaxpy(int64_t n, const double *alpha, const T *x, int64_t incx, T *y, int64_t incy,
                        hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(qaxpy_kernel<T>, dim3(grid_for(n, 8192)), dim3(NT), 0, stream, n,
                       make_scalars(alpha, nullptr), x, incx, y, incy);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_qdot(bool conj, int64_t n, const T *x, int64_t incx, const T *y, int64_t incy, T *result,
                       double *work, hipStream_t stream)
{
    const int parts = n > 0 ? grid_for(n, kDotParts) : 0;
    if (parts > 0) {
        if (conj)
            hipLaunchKernelGGL((qdot_partial_kernel<T, true>), dim3(parts), dim3(NT), 0, stream, n, x, incx, y, incy,
                               work);
        else
            hipLaunchKernelGGL((qdot_partial_kernel<T, false>), dim3(parts), dim3(NT), 0, stream, n, x, incx, y,
                               incy, work);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(qdot_final_kernel<T>, dim3(1), dim3(NT), 0, stream, parts, work, result);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_qgemv(int trans, int M, int N, const double *alpha, const T *A, int64_t lda, const T *x,
                        int64_t incx, const double *beta, T *y, int64_t incy, hipStream_t stream)
{
    const Scalars s = make_scalars(alpha, beta);
    const bool alpha_zero = zero4(s.alpha), beta_zero = zero4(s.beta);
    const bool conj = trans == QGEMM_OP_C || trans == QGEMM_OP_R;
    if (trans == QGEMM_OP_N || trans == QGEMM_OP_R) {
        const int ncols = alpha_zero ? 0 : N;
        const dim3 grid((M + GemvN<T>::GR - 1) / GemvN<T>::GR);
        if (conj)
            hipLaunchKernelGGL((qgemv_n_kernel<T, true>), grid, dim3(GemvN<T>::NTB), 0, stream, M, ncols, s, A,
                               lda, x, incx, beta_zero, y, incy);
        else
            hipLaunchKernelGGL((qgemv_n_kernel<T, false>), grid, dim3(GemvN<T>::NTB), 0, stream, M, ncols, s, A,
                               lda, x, incx, beta_zero, y, incy);
    } else {
        const int nrows = alpha_zero ? 0 : M;
        const dim3 grid((N + TC - 1) / TC);
        if (conj)
            hipLaunchKernelGGL((qgemv_t_kernel<T, true>), grid, dim3(NT), 0, stream, N, nrows, s, A, lda, x, incx,
                               beta_zero, y, incy);
        else
            hipLaunchKernelGGL((qgemv_t_kernel<T, false>), grid, dim3(NT), 0, stream, N, nrows, s, A, lda, x,
                               incx, beta_zero, y, incy);
    }
    return hipGetLastError();
}

// Partial-sum workspace of qdot_d_noalloc: file-scope device memory, one copy
// per GPU that the library runs on, held until the process ends.  In host
// code `scratch` names a host-side stand-in, not the device array: the host
// reaches the array only through the device address hipGetSymbolAddress
// returns with that device current (dot_scratch below), never by the name.
// Every qdot_d_noalloc call on one GPU shares that GPU's copy.  Pass 1 of the
// dot writes the partial sum of every block it launches and pass 2 reads only
// those, so nothing needs clearing between calls; calls that overlap on one
// GPU (two streams, or two host threads) race on it.
namespace {
constexpr int kDotScratchDoubles = 4 * kDotParts;
__device__ __align__(256) double scratch[kDotScratchDoubles];

}  // namespace

// Device address of `scratch` on the current device, looked up once per
// device (ordinals 0..63 are cached; others look it up on every call).  Two
// threads may race the first lookup: both store the same address.
hipError_t dot_scratch(double **out, int *capacity)
{
    static std::atomic<double *> cache[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    *capacity = kDotScratchDoubles;
    if (dev >= 0 && dev < 64) {
        double *p = cache[dev].load(std::memory_order_acquire);
        if (p) {
            *out = p;
            return hipSuccess;
        }
    }
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    if (dev >= 0 && dev < 64) cache[dev].store(static_cast<double *>(ptr), std::memory_order_release);
    *out = static_cast<double *>(ptr);
    return hipSuccess;
}

template hipError_t launch_qaxpy<double>(int64_t, const double *, const double *, int64_t, double *, int64_t,
                                         hipStream_t);
template hipError_t launch_qaxpy<float>(int64_t, const double *, const float *, int64_t, float *, int64_t,
                                        hipStream_t);
template hipError_t launch_qdot<double>(bool, int64_t, const double *, int64_t, const double *, int64_t, double *,
                                        double *, hipStream_t);
template hipError_t launch_qdot<float>(bool, int64_t, const float *, int64_t, const float *, int64_t, float *,
                                       double *, hipStream_t);
template hipError_t launch_qgemv<double>(int, int, int, const double *, const double *, int64_t, const double *,
                                         int64_t, const double *, double *, int64_t, hipStream_t);
template hipError_t launch_qgemv<float>(int, int, int, const double *, const float *, int64_t, const float *,
                                        int64_t, const double *, float *, int64_t, hipStream_t);

}  // namespace qg
