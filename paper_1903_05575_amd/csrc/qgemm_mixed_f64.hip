// FP64 mixed-type quaternion GEMM on the gfx950 FP64 matrix cores: one
// operand real or complex, the other quaternion, C quaternion.  A real x is
// the quaternion x e0 and a complex z0 + z1 i the quaternion z0 e0 + z1 e1
// (the complex subalgebra, Eq. complex_subalg and Eq. h_c_iso).
//
// Method.  The embedded operand is never widened into quaternions: that
// would feed the matrix cores 3 zeros of 4 (real) or 1 of 2 (complex).  The
// product is instead a real contraction over kappa (real operand) or over
// (kappa, s), s = re / im (complex operand), from Eq. quaternion_prod:
//   x y, y real             : (x y)_r = x_r y
//   x z, quaternion on left : x z = z0 x + z1 (x e1),  x e1 = (-x1,  x0,  x3, -x2)
//   z x, quaternion on right: z x = z0 x + z1 (e1 x),  e1 x = (-x1,  x0, -x3,  x2)
// so a real operand costs 4 and a complex one 8 real multiply-adds per
// element product (against 16 for two quaternions).
//
// Roles.  The quaternion operand X (P x K) is the MFMA A operand, expanded
// per lane by a component index and a sign as in the quaternion kernel; the
// real or complex operand Y (K x Q, KC = 1 or 2 reals per element) is the
// MFMA B operand exactly as stored.  out = X . Y is C itself when the
// quaternion is the left factor (P = M, Q = N) and C^T when it is the right
// factor (P = N, Q = M; C = Y X, read as out[nu][mu] = sum X[nu][k] . Y[k][mu]
// with Y the left factor of each product).
//
// MFMA v_mfma_f64_16x16x4_f64 (layout as in qgemm_f64.hip): A row i is
// quaternion row p = i % 4 and component r = i / 4 of the result; A column k
// is kappa = k (KC = 1) or (kappa, s) = (k / 2, k % 2) (KC = 2).  Lane l of
// the result holds all four components of out(p0 + l / 16, q0 + l % 16), so
// the alpha / beta epilogue is lane-local.
//
// Tiling: block = 256 threads = 4 waves, tile BP x BQ = 32 x 64 or 32 x 128
// quaternions of out (see Shape).  Wave w owns rows [8w, 8w + 8) x all BQ
// columns = 2 x BQ/16 MFMA blocks.  A K-tile is 2 or 4 MFMA k-steps, staged
// through two LDS stages; the next K-tile is loaded at the start of a tile and
// written to the other stage after the next-to-last k-step.  Masked elements use the out-of-range buffer offset
// that reads as zero, so the K-loop has no branches.
// LDS layouts (doubles):
//   X stage: [kappa][p][4], row pitch 4 BP + 4
//   Y stage: [kappa * KC + s][q], row pitch BQ + 1
#include "qgemm_internal.hpp"

namespace qg {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int BP = 32, NT = 256;
constexpr int STEPS_MAX = 4;        // K-tile depth (MFMA k-steps) the in-tile offset check allows for
constexpr int BQ_MAX = 128;         // tile width the in-tile offset check allows for
constexpr int XP = 4 * BP + 4;      // doubles per kappa row of the X stage
constexpr unsigned kOob = 0x80000000u;

// Storage type T (double or float): operands are read in T and widened
// exactly to double while staged, so the LDS tiles, the MFMAs and the
// epilogue arithmetic are FP64 for both; C is stored in T.
// Tile: 32 x 64 quaternions of out (2 x 4 MFMA blocks per wave) for a complex
// operand (4 MFMA k-steps = 8 kappa per K-tile, 127 VGPRs, three blocks per
// CU) and for a real operand in float storage (2 k-steps = 8 kappa, 115 VGPRs,
// four blocks per CU); 32 x 128 (2 x 8 blocks, 4 k-steps = 16 kappa, two
// blocks per CU) for a real operand in double storage.  At three or more
// blocks per CU the waves run at raised priority outside their MFMA issue (as
// in the quaternion GEMM's 32-row tiles).  Measured at 8192^3 (interleaved
// runs on one host): complex x quaternion 127.6 -> 123.9 ms with 64 columns
// (from 128) and 125.4 -> 124.4 ms with the priorities; quaternion x real in
// float storage 65.9 -> 64.5 ms on the 32 x 64 shape with the priorities (66.4
// -> 65.0 on another host), but in double storage that shape was 2% faster on
// one host and 4% slower on another (66.0 against 68.8 ms), so double storage
// keeps the wide tile.
template <int KC, typename T>
struct Shape {
    // a real operand in double storage keeps the 32 x 128 tile at two blocks per CU; a real operand in float
    // storage and a complex one take 32 x 64 tiles at four and three blocks per CU
    static constexpr bool WIDE = KC == 1 && sizeof(T) == 8;
    static constexpr int BQ = WIDE ? 128 : 64;                 // quaternion columns of out per tile
    static constexpr int NQ = BQ / 16;                         // MFMA column blocks per wave
    static constexpr int MIN_BLOCKS = WIDE ? 2 : KC == 2 ? 3 : 4;   // resident blocks per CU
    static constexpr int STEPS = KC == 1 && !WIDE ? 2 : 4;     // MFMA k-steps per K-tile
    static constexpr bool PRIO = MIN_BLOCKS >= 3;              // raised wave priority outside the MFMA issue
    static constexpr int YP = BQ + 1;                          // doubles per row of the Y stage
    static constexpr int BK = STEPS * 4 / KC;                  // kappa per K-tile
    static constexpr int X_STAGE = BK * XP;
    static constexpr int Y_STAGE = BK * KC * YP;
    static constexpr int STAGE = X_STAGE + Y_STAGE;
    static constexpr int XPER = sizeof(T) == 8 ? 2 : 1;       // 16-byte loads per quaternion of X
    static constexpr int X_CH = BP * BK * XPER / NT;           // 16-byte loads of X per thread
    static constexpr int Y_EL = BK * BQ / NT;                  // Y elements per thread
    static constexpr int YBYTES = KC * (int)sizeof(T);         // bytes of one Y element
    static constexpr size_t LDS_BYTES = 2 * STAGE * sizeof(double);
    static_assert(X_CH * NT == BP * BK * XPER, "X tile must split evenly");
    static_assert(Y_EL * NT == BK * BQ, "Y tile must split evenly");
    static_assert(BQ <= BQ_MAX && NQ % 4 == 0 && STEPS <= STEPS_MAX && STEPS >= 2, "tile shape");
};

// raw register type of one Y element of `bytes` bytes
template <int bytes>
struct RawY;
template <>
struct RawY<4> { typedef unsigned type; };
template <>
struct RawY<8> { typedef u32x2 type; };
template <>
struct RawY<16> { typedef u32x4 type; };

__device__ __forceinline__ double flip(double v, bool neg)
{
    return __longlong_as_double(__double_as_longlong(v) ^ (neg ? (long long)0x8000000000000000ull : 0ll));
}

template <typename T, int KC, bool RIGHT, bool XT, bool YT>
__global__ __launch_bounds__(NT, (Shape<KC, T>::MIN_BLOCKS)) void qgemm_mixed_f64_kernel(MixedDesc p, int tiles_p, int tiles_q,
                                                                                         int nk)
{
    using S = Shape<KC, T>;
    constexpr int BK = S::BK, BQ = S::BQ, NQ = S::NQ, YP = S::YP;
    constexpr int XPER = S::XPER;
    typedef typename RawY<S::YBYTES>::type YRaw;
    const T *X = static_cast<const T *>(p.X);
    const T *Y = static_cast<const T *>(p.Y);
    T *Cp = static_cast<T *>(p.C);
    extern __shared__ double smem[];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    int tp, tq;
    xcd_tile(blockIdx.x, gridDim.x, tiles_p, tiles_q, 8, tp, tq);
    const int p0 = tp * BP, q0 = tq * BQ;

    // ---- per-lane constants of the A fragment (row i = lane % 16, column k = lane / 16)
    const int fi = lane & 15;
    const int fr = fi >> 2;                       // component of the result
    const int fp = fi & 3;                        // quaternion row within the 4-row block
    const int fk = lane >> 4;
    const int fs = KC == 2 ? (fk & 1) : 0;        // re / im of the complex operand
    const int fcomp = fr ^ fs;                    // component of x feeding this lane
    // sign of the e1 column: x e1 negates rows 0 and 3, e1 x rows 0 and 2
    const bool e1neg = fs == 1 && (fr == 0 || fr == (RIGHT ? 2 : 3));
    const bool neg = e1neg ^ (p.conjX && fcomp != 0) ^ (p.conjY && fs == 1);
    const int x_off = (fk / KC) * XP + (wave * 8 + fp) * 4 + fcomp;   // + step * (4 / KC) * XP + 16 m
    const int y_off = fk * YP + fi;                                     // + step * 4 * YP + 16 n

    d4 acc[2][NQ];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < NQ; ++n) acc[m][n] = (d4){0.0, 0.0, 0.0, 0.0};

    u32x4 rx[S::X_CH];
    YRaw ry[S::Y_EL];

    // X load i: half `half` (double) or all (float) of quaternion (pp, ka)
    auto x_slot = [&](int i, int &pp, int &ka, int &half) {
        const int q = tid + NT * i;
        half = XPER == 2 ? (q & 1) : 0;
        const int e = XPER == 2 ? (q >> 1) : q;
        if (!XT) { pp = e % BP; ka = e / BP; }
        else     { ka = e % BK; pp = e / BK; }
    };
    auto y_slot = [&](int i, int &ka, int &qq) {
        const int e = tid + NT * i;
        if (!YT) { ka = e % BK; qq = e / BK; }
        else     { qq = e % BQ; ka = e / BQ; }
    };

    auto load_tile = [&](int kt) {
        const int k0 = kt * BK;
        const int krem = p.K - k0;
        const T *Xb = X + 4 * (XT ? ((int64_t)p0 * p.ldx + k0) : ((int64_t)k0 * p.ldx + p0));
        const T *Yb = Y + KC * (YT ? ((int64_t)k0 * p.ldy + q0) : ((int64_t)q0 * p.ldy + k0));
        const __amdgpu_buffer_rsrc_t rX = __builtin_amdgcn_make_buffer_rsrc((void *)Xb, (short)0, 0x7fffffff, 0x00020000);
        const __amdgpu_buffer_rsrc_t rY = __builtin_amdgcn_make_buffer_rsrc((void *)Yb, (short)0, 0x7fffffff, 0x00020000);
#pragma unroll
        for (int i = 0; i < S::X_CH; ++i) {
            int pp, ka, half;
            x_slot(i, pp, ka, half);
            const unsigned e = XT ? (unsigned)pp * (unsigned)p.ldx + ka : (unsigned)ka * (unsigned)p.ldx + pp;
            const bool ok = p0 + pp < p.P && ka < krem;
            rx[i] = __builtin_amdgcn_raw_buffer_load_b128(rX, ok ? (unsigned)(4 * sizeof(T)) * e + 16u * half : kOob, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < S::Y_EL; ++i) {
            int ka, qq;
            y_slot(i, ka, qq);
            const unsigned e = YT ? (unsigned)ka * (unsigned)p.ldy + qq : (unsigned)qq * (unsigned)p.ldy + ka;
            const bool ok = q0 + qq < p.Q && ka < krem;
            const unsigned o = ok ? (unsigned)S::YBYTES * e : kOob;
            if constexpr (S::YBYTES == 4) ry[i] = __builtin_amdgcn_raw_buffer_load_b32(rY, o, 0, 0);
            else if constexpr (S::YBYTES == 8) ry[i] = __builtin_amdgcn_raw_buffer_load_b64(rY, o, 0, 0);
            else ry[i] = __builtin_amdgcn_raw_buffer_load_b128(rY, o, 0, 0);
        }
    };

    auto store_tile = [&](double *Xs) {
        double *Ys = Xs + S::X_STAGE;
#pragma unroll
        for (int i = 0; i < S::X_CH; ++i) {
            int pp, ka, half;
            x_slot(i, pp, ka, half);
            if constexpr (XPER == 2) {
                *reinterpret_cast<d2 *>(Xs + ka * XP + pp * 4 + 2 * half) = __builtin_bit_cast(d2, rx[i]);
            } else {
                const f4 v = __builtin_bit_cast(f4, rx[i]);
                *reinterpret_cast<d2 *>(Xs + ka * XP + pp * 4) = (d2){(double)v.x, (double)v.y};
                *reinterpret_cast<d2 *>(Xs + ka * XP + pp * 4 + 2) = (d2){(double)v.z, (double)v.w};
            }
        }
#pragma unroll
        for (int i = 0; i < S::Y_EL; ++i) {
            int ka, qq;
            y_slot(i, ka, qq);
            if constexpr (KC == 1) {
                double v;
                if constexpr (sizeof(T) == 8) v = __builtin_bit_cast(double, ry[i]);
                else v = (double)__builtin_bit_cast(float, ry[i]);
                Ys[ka * YP + qq] = v;
            } else {
                double re, im;
                if constexpr (sizeof(T) == 8) {
                    const d2 z = __builtin_bit_cast(d2, ry[i]);
                    re = z.x; im = z.y;
                } else {
                    const f2 z = __builtin_bit_cast(f2, ry[i]);
                    re = z.x; im = z.y;
                }
                Ys[(2 * ka) * YP + qq] = re;
                Ys[(2 * ka + 1) * YP + qq] = im;
            }
        }
    };

    // Multiply the K-tile in stage `Xs`; the registers of the next K-tile are
    // written to `Nxt` after the third k-step.  Fragments of step kk + 1 are
    // read while step kk's MFMAs run.
    auto step_tile = [&](const double *Xs, double *Nxt) {
        const double *Ys = Xs + S::X_STAGE;
        double a[2][2], b[2][NQ];
#pragma unroll
        for (int m = 0; m < 2; ++m) a[0][m] = Xs[x_off + 16 * m];
#pragma unroll
        for (int n = 0; n < NQ; ++n) b[0][n] = Ys[y_off + 16 * n];
#pragma unroll
        for (int kk = 0; kk < S::STEPS; ++kk) {
            const int cur = kk & 1;
            if (kk + 1 < S::STEPS) {
#pragma unroll
                for (int m = 0; m < 2; ++m) a[cur ^ 1][m] = Xs[(kk + 1) * (4 / KC) * XP + x_off + 16 * m];
#pragma unroll
                for (int n = 0; n < NQ; ++n) b[cur ^ 1][n] = Ys[(kk + 1) * 4 * YP + y_off + 16 * n];
            }
            // raised wave priority outside the MFMA issue (see the tile comment above)
            if constexpr (S::PRIO) __builtin_amdgcn_s_setprio(0);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const double am = flip(a[cur][m], neg);
#pragma unroll
                for (int n = 0; n < NQ; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(am, b[cur][n], acc[m][n], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (S::PRIO) __builtin_amdgcn_s_setprio(1);
            if (kk == S::STEPS - 2) store_tile(Nxt);
        }
    };

    if (nk > 0) {
        load_tile(0);
        store_tile(smem);
        __syncthreads();
    }
    // tiles past the end load as zeros and land in the unused stage
    for (int kt = 0; kt < nk; ++kt) {
        const int st = kt & 1;
        load_tile(kt + 1);
        step_tile(smem + st * S::STAGE, smem + (st ^ 1) * S::STAGE);
        __syncthreads();
    }

    // ---- epilogue: C <- alpha acc + beta C (left scalars), lane-local quaternions.  The old C values of
    // four outputs at a time are all requested before the first of them is written, so their latencies
    // overlap (a read after a write to the same array is not reordered by the compiler).
    const bool beta_zero = p.beta[0] == 0.0 && p.beta[1] == 0.0 && p.beta[2] == 0.0 && p.beta[3] == 0.0;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int pp = p0 + wave * 8 + 4 * m + (lane >> 4);
#pragma unroll
        for (int nh = 0; nh < NQ; nh += 4) {
            double cold[4][4];
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const int qq = q0 + 16 * (nh + n) + (lane & 15);
                cold[n][0] = cold[n][1] = cold[n][2] = cold[n][3] = 0.0;
                if (pp >= p.P || qq >= p.Q || beta_zero) continue;
                const int mu = RIGHT ? qq : pp, nu = RIGHT ? pp : qq;
                const T *src = Cp + 4 * ((int64_t)nu * p.ldc + mu);
                if constexpr (sizeof(T) == 8) {
                    const d2 c0 = reinterpret_cast<const d2 *>(src)[0], c1 = reinterpret_cast<const d2 *>(src)[1];
                    cold[n][0] = c0.x; cold[n][1] = c0.y; cold[n][2] = c1.x; cold[n][3] = c1.y;
                } else {
                    const f4 c = *reinterpret_cast<const f4 *>(src);
                    cold[n][0] = c.x; cold[n][1] = c.y; cold[n][2] = c.z; cold[n][3] = c.w;
                }
            }
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const int qq = q0 + 16 * (nh + n) + (lane & 15);
                if (pp >= p.P || qq >= p.Q) continue;
                const int mu = RIGHT ? qq : pp, nu = RIGHT ? pp : qq;
                const double v[4] = {acc[m][nh + n][0], acc[m][nh + n][1], acc[m][nh + n][2], acc[m][nh + n][3]};
                double o[4];
                qmul(p.alpha, v, o);
                if (!beta_zero) {
                    double u[4];
                    qmul(p.beta, cold[n], u);
                    o[0] += u[0]; o[1] += u[1]; o[2] += u[2]; o[3] += u[3];
                }
                T *dst = Cp + 4 * ((int64_t)nu * p.ldc + mu);
                if constexpr (sizeof(T) == 8) {
                    reinterpret_cast<d2 *>(dst)[0] = (d2){o[0], o[1]};
                    reinterpret_cast<d2 *>(dst)[1] = (d2){o[2], o[3]};
                } else {
                    *reinterpret_cast<f4 *>(dst) = (f4){(float)o[0], (float)o[1], (float)o[2], (float)o[3]};
                }
            }
        }
    }
}

template <typename T, int KC, bool RIGHT, bool XT, bool YT>
hipError_t launch_t(const MixedDesc &d, hipStream_t stream)
{
    using S = Shape<KC, T>;
    auto kern = &qgemm_mixed_f64_kernel<T, KC, RIGHT, XT, YT>;
    static std::atomic<uint64_t> lds_set{0};
    hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void *>(kern), (int)S::LDS_BYTES, lds_set);
    if (e != hipSuccess) return e;
    const int tiles_p = (d.P + BP - 1) / BP;
    const int tiles_q = (d.Q + S::BQ - 1) / S::BQ;
    const bool alpha_zero = d.alpha[0] == 0.0 && d.alpha[1] == 0.0 && d.alpha[2] == 0.0 && d.alpha[3] == 0.0;
    const int nk = alpha_zero ? 0 : (d.K + S::BK - 1) / S::BK;
    const int64_t nblocks = (int64_t)tiles_p * tiles_q;
    if (nblocks <= 0) return hipSuccess;
    if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(kern, dim3((unsigned)nblocks), dim3(NT), S::LDS_BYTES, stream, d, tiles_p, tiles_q, nk);
    return hipGetLastError();
}

template <typename T, int KC, bool RIGHT>
hipError_t launch_layouts(const MixedDesc &d, hipStream_t s)
{
    if (d.xt) return d.yt ? launch_t<T, KC, RIGHT, true, true>(d, s) : launch_t<T, KC, RIGHT, true, false>(d, s);
    return d.yt ? launch_t<T, KC, RIGHT, false, true>(d, s) : launch_t<T, KC, RIGHT, false, false>(d, s);
}

template <typename T>
hipError_t launch_kinds(const MixedDesc &d, hipStream_t s)
{
    if (d.kc == 1) return d.right ? launch_layouts<T, 1, true>(d, s) : launch_layouts<T, 1, false>(d, s);
    if (d.kc == 2) return d.right ? launch_layouts<T, 2, true>(d, s) : launch_layouts<T, 2, false>(d, s);
    return hipErrorInvalidValue;
}

}  // namespace

bool mixed_ld_supported(int64_t ldx, int64_t ldy, bool xt, bool yt, int kc, int real_bytes)
{
    const int64_t lim = (int64_t)1 << 31;
    const int bk = STEPS_MAX * 4 / kc;
    const int64_t fx = 4 * real_bytes * (xt ? ((int64_t)BP * ldx + bk) : ((int64_t)bk * ldx + BP));
    const int64_t fy = kc * real_bytes * (yt ? ((int64_t)bk * ldy + BQ_MAX) : ((int64_t)BQ_MAX * ldy + bk));
    return fx < lim && fy < lim;
}

hipError_t launch_qgemm_mixed_f64(const MixedDesc &d, hipStream_t stream)
{
    if (!mixed_ld_supported(d.ldx, d.ldy, d.xt, d.yt, d.kc, d.f32 ? 4 : 8)) return hipErrorInvalidValue;
    return d.f32 ? launch_kinds<float>(d, stream) : launch_kinds<double>(d, stream);
}

}  // namespace qg
