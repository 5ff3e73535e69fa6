// One output tile of the FP64 quaternion GEMM on the gfx950 FP64 matrix cores.
// Shared by the single-GEMM kernel (qgemm_f64.hip) and the grouped FP64
// kernel (qgemm_grouped.hip).
//
// Method.  Write a quaternion a as the real 4x4 block L(a) with
// vec(a b) = L(a) vec(b) (from Eq. quaternion_prod).  Then, with B and C read
// as real matrices of 4K x N and 4M x N reals (the interleaved column-major
// storage already is that), C_real = L(op A) B_real: a real GEMM of shape
// (4M, N, 4K) doing exactly 16 real multiply-adds per quaternion
// multiply-add, the count of Tab. hc_flops.  L(op A) is never materialised:
// each lane of the MFMA A operand picks one component of one quaternion from
// LDS and flips its sign, so the expansion costs no HBM traffic and no flops.
//
// MFMA.  v_mfma_f64_16x16x4_f64 computes D(16x16) += A(16x4) B(4x16) with
//   A[i][k] in lane i + 16k, B[k][j] in lane j + 16k, and D[i][j] in lane
//   j + 16 (i % 4), register i / 4 (layout measured on gfx950).
// Row i of the A operand is mapped to quaternion row  mu = i % 4  and
// component r = i / 4, column k to component c of op(B).  Then lane l of the
// result holds all four components (registers 0..3) of output quaternion
// (mu0 + l / 16, nu0 + l % 16), so the non-commuting alpha/beta epilogue is
// lane-local.  One MFMA = 4 quaternion rows x 16 quaternion columns x one
// kappa = 64 quaternion multiply-adds.
//
// Tiling (block = 256 threads = 4 waves, BM x BN = 32 x 64, 64 x 64 or
// 32 x 32 quaternions):
//   wave w owns quaternion rows [w BM/4, (w+1) BM/4) x all BN columns = MB x NB
//   MFMA blocks (MB = 2 or 4, NB = BN / 16) of 4 doubles each.  Per kappa a
//   wave reads MB A and NB B fragments (one 8-byte LDS read per lane each) and
//   issues MB NB MFMAs.  32 x 64 tiles: K-tiles of 4, four blocks per CU (123
//   VGPRs, 4.2 + 8.3 KB of LDS per stage); 64 x 64 tiles: K-tiles of 8, two
//   blocks per CU (224 VGPRs, 16.6 + 16.6 KB per stage); 32 x 32 tiles (grids
//   that 32 x 64 tiles fill poorly): K-tiles of 8, four blocks per CU (90
//   VGPRs, 8.3 + 8.3 KB per stage).
//   K is walked in tiles of BK quaternions through two LDS stages: the next
//   tile is fetched from HBM into registers at the start of a tile and
//   written to the other stage in the middle of the current tile's MFMA
//   stream (one barrier per tile).  Fragments of the next kappa step are read
//   from LDS while the current step's MFMAs run.  Operands are read with
//   buffer loads; masked elements use an out-of-range offset that reads as
//   zero, so the K-loop has no branches.
// LDS layouts (doubles):
//   A stage: [kappa][mu][4] with a row pitch of 4*BM + 4 (the pad spreads the
//            transposed-operand writes over the banks); fragment reads of one
//            kappa touch 4 consecutive quaternions = 128 contiguous bytes.
//   B stage: [kappa][component][nu], plane pitch BN + 1; a fragment read is
//            16 consecutive doubles per component.  Staging threads store 4 kappa x 4 nu
//            blocks (op N) or 16 consecutive nu (op T / C), so the component
//            writes of 16 lanes hit 32 distinct banks.  op(B) conjugation and the
//            optional left scale s are applied while writing this stage.
// Triangular operand (TRI = 1: op(A), TRI = 2: op(B); triangular multiply):
//   a tile walks only the K-tiles the triangle reaches from its rows
//   (columns); elements across the diagonal take the zero-reading offset and
//   a unit diagonal is written into LDS in place of the (unread) element, so
//   the other triangle is never read.  Tiles are then ordered by weight, see
//   xcd_chunk_tile.
#pragma once

#include "qgemm_internal.hpp"

namespace qg {
namespace f64 {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int BN = 64;
constexpr int NT = 256;
constexpr int B_PL = BN + 1;                     // doubles per component plane of the B stage

// Tile height: 32 quaternion rows (four blocks per CU), or 64 for triangular
// outputs (two blocks per CU).  Each wave owns BM / 4 rows = MB MFMA row
// blocks.  K-tile: 4 kappa for 32 x 64 tiles, which halves their LDS (25 KB
// per block) and prefetch registers (123 VGPRs) so that four blocks fit per
// CU (measured 8192^3 90.5% -> 91.2% of the FP64 peak, 2048^3 88.9% ->
// 89.8%; an 8192 triangular multiply 127.9 -> 126.7 ms, although its masks
// then spill a few registers); 8 kappa for 64-row tiles, and for 32 x 32
// tiles, whose B tile would not split over the block at 4.  Tile width: 64
// columns, or 32 for general operands on grids that 32 x 64 tiles fill poorly
// (see launch_ops in qgemm_f64.hip).
template <int BMT, int TRI = 0, int BNT = BN>
struct FTile {
    static constexpr int BM = BMT;
    static constexpr int BNW = BNT;              // tile width (quaternion columns)
    static constexpr int NB = BNT / 16;          // MFMA column blocks (16 columns each) per wave
    static constexpr int BPL = BNT + 1;          // doubles per component plane of the B stage
    static constexpr int BK = BMT == 32 && BNT == 64 ? 4 : 8;
    static constexpr int MIN_BLOCKS = BMT == 64 ? 2 : BK == 4 || BNT == 32 ? 4 : 3;   // resident blocks per CU
    static constexpr int STORE_AT = BK == 8 ? 5 : 2;   // k-step after which the next K-tile is staged
    static constexpr int WM = BM / 4;            // quaternion rows per wave
    static constexpr int MB = WM / 4;            // MFMA row blocks (4 rows each) per wave
    static constexpr int A_LD = 4 * BM + 4;      // doubles per kappa row of the A stage
    static constexpr int A_STAGE = BK * A_LD;
    static constexpr int B_STAGE = BK * 4 * BPL;
    static constexpr int STAGE = A_STAGE + B_STAGE;
    static constexpr int A_CHUNKS = BM * BK * 2 / NT;   // 16-byte chunks of A per thread per tile
    static constexpr int B_QUATS = BNT * BK / NT;       // quaternions of B per thread per tile
    static constexpr size_t LDS_BYTES = 2 * STAGE * sizeof(double);
    static_assert(A_CHUNKS * NT == BM * BK * 2, "A tile must split evenly over the block");
    static_assert(B_QUATS * NT == BNT * BK, "B tile must split evenly over the block");
    static_assert(BNT == 64 || (BNT == 32 && BMT == 32 && TRI == 0), "32-column tiles: 32 rows, general operands");
    static_assert(MB * 16 == BM, "whole MFMA row blocks per wave");
    static_assert(BK % 4 == 0 && STORE_AT + 1 < BK, "staging point inside the K-tile");
};

__device__ __forceinline__ double flip(double v, unsigned long long sign)
{
    return __longlong_as_double(__double_as_longlong(v) ^ (long long)sign);
}

constexpr unsigned kOob = 0x80000000u;   // buffer offset read as zero (masked element)

// Compute the BM x 64 output tile at (m0, n0) of the GEMM described by p and
// write it.  nk = number of K-tiles of BK quaternions (0 when alpha == 0).
// smem must hold FTile<BMT, TRI>::LDS_BYTES.  Every thread of the block calls
// this; on return every wave has finished with smem, so the caller may reuse
// it for another tile.
template <int BMT, bool TA, bool TB, bool BS, int TRI, int BNT = BN>
__device__ __forceinline__ void f64_tile(const GemmDesc<double> &p, int m0, int n0, int nk, double *smem)
{
    using FT = FTile<BMT, TRI, BNT>;
    constexpr int BN = FT::BNW, NB = FT::NB, B_PL = FT::BPL;   // shadow the 64-column defaults
    constexpr int BM = FT::BM, BK = FT::BK, WM = FT::WM, MB = FT::MB, A_LD = FT::A_LD, A_STAGE = FT::A_STAGE,
                  STAGE = FT::STAGE, A_CHUNKS = FT::A_CHUNKS, B_QUATS = FT::B_QUATS;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    // K-tiles this tile needs: all, or those a triangular operand reaches
    int kt0 = 0, kt1 = nk;
    if constexpr (TRI == 1) {
        if (p.tri_lower) kt1 = min(nk, (m0 + BM + BK - 1) / BK);   // op(A)[mu][k] = 0 for k > mu
        else kt0 = min(nk, m0 / BK);                                // op(A)[mu][k] = 0 for k < mu
    } else if constexpr (TRI == 2) {
        if (p.tri_lower) kt0 = min(nk, n0 / BK);                    // op(B)[k][nu] = 0 for k < nu
        else kt1 = min(nk, (n0 + BN + BK - 1) / BK);                // op(B)[k][nu] = 0 for k > nu
    }

    // ---- per-lane constants of the A fragment (row i = lane % 16, column c = lane / 16)
    const int fi = lane & 15;
    const int fr = fi >> 2;                      // component of the result row
    const int fmu = fi & 3;                      // quaternion row within the 4-row block
    const int fc = lane >> 4;                    // component of op(B) (k index)
    const int fcomp = fr ^ fc;                   // component of a that L(a)[fr][fc] reads
    const bool neg = l_negative(fr, fc) ^ (p.conjA && fcomp != 0);
    const unsigned long long sgnA = neg ? 0x8000000000000000ull : 0ull;
    const int a_off = (wave * WM + fmu) * 4 + fcomp;      // + kk*A_LD + 16*m
    const int b_off = fc * B_PL + (lane & 15);            // + kk*4*B_PL + 16*n
    const unsigned conjB = p.conjB ? 0x80000000u : 0u;     // sign bit of the high word of q1..q3

    d4 acc[MB][NB];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int n = 0; n < NB; ++n) acc[m][n] = (d4){0.0, 0.0, 0.0, 0.0};

    d2 ra[A_CHUNKS];
    d2 rb[B_QUATS][2];
    unsigned unit_bits = 0;   // slots of the loaded tile on a unit diagonal (triangular operand)

    // Staging coordinates of slot i (recomputed from the thread id where used,
    // which is cheaper than keeping them live in registers): A chunk i holds
    // half `half` of quaternion (mu, ka) of the tile, B slot i quaternion (nu, ka).
    auto a_slot = [&](int i, int &mu, int &ka, int &half) {
        const int q = tid + NT * i;
        half = q & 1;
        if (!TA) { mu = (q >> 1) % BM; ka = (q >> 1) / BM; }
        else     { ka = (q >> 1) % BK; mu = (q >> 1) / BK; }
    };
    // B: each group of 16 lanes stores a 4 x 4 (kappa x nu) block when B is read along kappa, so that
    // its writes into the component planes fall on distinct banks (16 consecutive nu when read along nu).
    auto b_slot = [&](int i, int &nu, int &ka) {
        const int q = tid + NT * i;
        if (!TB) {
            const int lo = q & 15, hi = q >> 4;
            ka = (lo >> 2) + 4 * (hi % (BK / 4));
            nu = (lo & 3) + 4 * (hi / (BK / 4));
        } else {
            nu = q % BN; ka = q / BN;
        }
    };

    // fetch K-tile kt into registers; elements at or past K (and whole tiles past
    // the end) and rows outside the matrix read as zero through the buffer range
    // check (in-tile byte offsets are below 2^31, see f64_ld_supported)
    auto load_tile = [&](int kt) {
        const int k0 = kt * BK;
        // the prefetch past this tile's K-range reads nothing (for a triangular
        // operand that tile lies in the triangle that must not be read)
        const int krem = (kt < kt1 ? p.K : 0) - k0;
        const double *Ab = p.A + 4 * (TA ? ((int64_t)m0 * p.lda + k0) : ((int64_t)k0 * p.lda + m0));
        const double *Bb = p.B + 4 * (TB ? ((int64_t)k0 * p.ldb + n0) : ((int64_t)n0 * p.ldb + k0));
        const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc((void *)Ab, (short)0, 0x7fffffff, 0x00020000);
        const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc((void *)Bb, (short)0, 0x7fffffff, 0x00020000);
        // only K-tiles that cross the diagonal of a triangular operand need its mask (uniform per block)
        const bool diagA = TRI == 1 && k0 < m0 + BM && k0 + BK > m0;
        const bool diagB = TRI == 2 && k0 < n0 + BN && k0 + BK > n0;
        if constexpr (TRI != 0) unit_bits = 0;
#pragma unroll
        for (int i = 0; i < A_CHUNKS; ++i) {
            int mu, ka, half;
            a_slot(i, mu, ka, half);
            const unsigned e = TA ? (unsigned)mu * (unsigned)p.lda + ka : (unsigned)ka * (unsigned)p.lda + mu;
            bool ok = m0 + mu < p.M && ka < krem;
            if constexpr (TRI == 1) {
                if (diagA) {
                    const int gm = m0 + mu, gk = k0 + ka;
                    ok = ok && (p.tri_lower ? gk <= gm : gk >= gm) && !(p.tri_unit && gk == gm);
                    if (p.tri_unit && gk == gm && gm < p.M) unit_bits |= 1u << i;
                }
            }
            ra[i] = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(rA, ok ? 32u * e + 16u * half : kOob, 0, 0));
        }
#pragma unroll
        for (int i = 0; i < B_QUATS; ++i) {
            int nu, ka;
            b_slot(i, nu, ka);
            const unsigned e = TB ? (unsigned)ka * (unsigned)p.ldb + nu : (unsigned)nu * (unsigned)p.ldb + ka;
            bool ok = n0 + nu < p.N && ka < krem;
            if constexpr (TRI == 2) {
                if (diagB) {
                    const int gn = n0 + nu, gk = k0 + ka;
                    ok = ok && (p.tri_lower ? gk >= gn : gk <= gn) && !(p.tri_unit && gk == gn);
                    if (p.tri_unit && gk == gn && gn < p.N) unit_bits |= 1u << i;
                }
            }
            rb[i][0] = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(rB, ok ? 32u * e : kOob, 0, 0));
            rb[i][1] = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(rB, ok ? 32u * e + 16u : kOob, 0, 0));
        }
    };

    auto store_tile = [&](double *As) {
        double *Bs = As + A_STAGE;
#pragma unroll
        for (int i = 0; i < A_CHUNKS; ++i) {
            int mu, ka, half;
            a_slot(i, mu, ka, half);
            d2 v = ra[i];
            if constexpr (TRI == 1) {
                if ((unit_bits >> i) & 1u) v = (d2){half ? 0.0 : 1.0, 0.0};   // unit diagonal, not read
            }
            *reinterpret_cast<d2 *>(As + ka * A_LD + mu * 4 + 2 * half) = v;
        }
#pragma unroll
        for (int i = 0; i < B_QUATS; ++i) {
            int nu, ka;
            b_slot(i, nu, ka);
            double b[4] = {rb[i][0].x, rb[i][0].y, rb[i][1].x, rb[i][1].y};
            if constexpr (TRI == 2) {
                if ((unit_bits >> i) & 1u) { b[0] = 1.0; b[1] = b[2] = b[3] = 0.0; }   // unit diagonal, not read
            }
#pragma unroll
            for (int c = 1; c < 4; ++c)
                b[c] = __longlong_as_double(__double_as_longlong(b[c]) ^ ((long long)conjB << 32));
            if constexpr (BS) {
                double t[4];
                qmul(p.bscale, b, t);
                b[0] = t[0]; b[1] = t[1]; b[2] = t[2]; b[3] = t[3];
            }
            double *dst = Bs + ka * 4 * B_PL + nu;
            dst[0 * B_PL] = b[0];
            dst[1 * B_PL] = b[1];
            dst[2 * B_PL] = b[2];
            dst[3 * B_PL] = b[3];
        }
    };

    // Multiply the K-tile in stage `cur`; the registers holding the next K-tile
    // are written into stage `nxt` half way through, so those LDS writes overlap
    // the MFMAs.  Fragments of step kk + 1 are read while step kk's MFMAs run.
    // 32-row tiles (four blocks per CU): a wave runs at raised priority except
    // while it issues its MFMAs, so that the waves staging a K-tile, reading
    // fragments or heading for the barrier are issued first and the MFMA pipe
    // is fed by whichever waves are in their MFMA phase (measured: 8192^3
    // 0.6-1.1% faster, 1024^3 1.6-1.9%, the FP64 batched launch 1.5%; the
    // opposite priorities were slower, and so was this for 64-row tiles at two
    // blocks per CU, 0.5-0.7%).
    constexpr bool kPrio = BMT == 32;
    auto step_tile = [&](const double *As, double *Nxt) {
        const double *Bs = As + A_STAGE;
        double a[2][MB], b[2][NB];
#pragma unroll
        for (int m = 0; m < MB; ++m) a[0][m] = As[a_off + 16 * m];
#pragma unroll
        for (int n = 0; n < NB; ++n) b[0][n] = Bs[b_off + 16 * n];
#pragma unroll
        for (int kk = 0; kk < BK; ++kk) {
            const int cur = kk & 1;
            if (kk + 1 < BK) {
#pragma unroll
                for (int m = 0; m < MB; ++m) a[cur ^ 1][m] = As[(kk + 1) * A_LD + a_off + 16 * m];
#pragma unroll
                for (int n = 0; n < NB; ++n) b[cur ^ 1][n] = Bs[(kk + 1) * 4 * B_PL + b_off + 16 * n];
            }
            // keep the sign flips of step kk + 1 out of this step: they would wait on the reads above
            if constexpr (kPrio) __builtin_amdgcn_s_setprio(0);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                const double am = flip(a[cur][m], sgnA);
#pragma unroll
                for (int n = 0; n < NB; ++n)
                    acc[m][n] = __builtin_amdgcn_mfma_f64_16x16x4f64(am, b[cur][n], acc[m][n], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (kPrio) __builtin_amdgcn_s_setprio(1);
            if (kk == FT::STORE_AT) store_tile(Nxt);
        }
    };

    if (kt0 < kt1) {
        load_tile(kt0);
        store_tile(smem);
        __syncthreads();
    }
    // the tile after the last is loaded too and lands in the unused stage
    for (int kt = kt0; kt < kt1; ++kt) {
        const int st = (kt - kt0) & 1;
        load_tile(kt + 1);
        step_tile(smem + st * STAGE, smem + (st ^ 1) * STAGE);
        __syncthreads();
    }

    // ---- epilogue: C <- alpha acc + beta C (left scalars), lane-local quaternions.  The old C values of
    // one MFMA row block are all requested before the first of them is written, so their latencies overlap
    // (a read after a write to the same array is not reordered by the compiler).
    const bool beta_zero = p.beta[0] == 0.0 && p.beta[1] == 0.0 && p.beta[2] == 0.0 && p.beta[3] == 0.0;
#pragma unroll
    for (int m = 0; m < MB; ++m) {
        const int mu = m0 + wave * WM + 4 * m + (lane >> 4);
        bool ok[NB];
        int64_t e[NB];
        d2 cold[NB][2];
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            const int nu = n0 + 16 * n + (lane & 15);
            const bool in_tri = p.uplo == 0 || (p.uplo == 1 ? mu >= nu : mu <= nu);
            ok[n] = mu < p.M && nu < p.N && in_tri;
            e[n] = p.store_t ? ((int64_t)mu * p.ldc + nu) : ((int64_t)nu * p.ldc + mu);
            cold[n][0] = cold[n][1] = (d2){0.0, 0.0};
            if (ok[n] && !beta_zero) {
                const d2 *src = reinterpret_cast<const d2 *>(p.C + 4 * e[n]);
                cold[n][0] = src[0];
                cold[n][1] = src[1];
            }
        }
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            if (!ok[n]) continue;
            const int nu = n0 + 16 * n + (lane & 15);
            const double v[4] = {acc[m][n][0], acc[m][n][1], acc[m][n][2], acc[m][n][3]};
            double o[4];
            qmul(p.alpha, v, o);
            if (p.has_right) {
                const double t[4] = {o[0], o[1], o[2], o[3]};
                qmul(t, p.alpha_r, o);
            }
            if (p.store_conj) { o[1] = -o[1]; o[2] = -o[2]; o[3] = -o[3]; }
            if (!beta_zero) {
                const double cq[4] = {cold[n][0].x, cold[n][0].y, cold[n][1].x, cold[n][1].y};
                double u[4];
                qmul(p.beta, cq, u);
                if (p.has_right) {
                    const double t[4] = {u[0], u[1], u[2], u[3]};
                    qmul(t, p.beta_r, u);
                }
                o[0] += u[0]; o[1] += u[1]; o[2] += u[2]; o[3] += u[3];
            }
            if (p.herm_diag && mu == nu) o[1] = o[2] = o[3] = 0.0;
            d2 *dst = reinterpret_cast<d2 *>(p.C + 4 * e[n]);
            dst[0] = (d2){o[0], o[1]};
            dst[1] = (d2){o[2], o[3]};
        }
    }
}


}  // namespace f64
}  // namespace qg
