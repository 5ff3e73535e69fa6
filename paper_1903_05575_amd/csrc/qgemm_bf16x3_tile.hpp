// One output tile of the FP32-stored quaternion GEMM computed as split-BF16
// products on the gfx950 BF16 matrix cores (FP32 accumulation).  Shared by
// the single-GEMM kernel and the grouped (batched) kernel.
//
// Split.  While a tile is staged from HBM into LDS every FP32 component x is
// split into three BF16 pieces with round-to-nearest-even on the successive
// residuals:  h = bf16(x), m = bf16(x - h), l = bf16(x - h - m).  Both
// residuals are exact in FP32, and h + m + l == x for finite |x| below the
// BF16 overflow threshold.  A product a b is the sum of the nine piece
// products; NTERMS selects how many are formed, in order of magnitude:
//   3: hh hm mh      6: + hl mm lh (all terms down to 2^-16 relative)
//   9: + ml lm ll (exact up to accumulation rounding)
//
// Quaternion structure.  As in the FP64 path the product is the real GEMM
// C_real (4M x N) = L(op A) (4M x 4K) B_real (4K x N), where L(a) is the 4x4
// left-multiplication block of a (derived from Eq. quaternion_prod).  The
// BF16 A operand is formed from LDS by a byte permutation and a sign XOR per
// register: no extra HBM traffic, no flops.
//
// MFMA.  v_mfma_f32_32x32x16_bf16: A 32 x 16 (lane l: row l % 32, eight k
// values of group l / 32), B 16 x 32 (lane l: column l % 32, the same eight k
// slots), D 32 x 32 with D[i][j] in lane j + 32 ((i / 4) % 2), register
// 4 (i / 8) + i % 4 (layout measured on gfx950).  Row i of A is quaternion row
// i / 4, component i % 4; the eight k slots of group g are quaternions
// 2g, 2g + 1 of the 4-kappa step, components 0..3.  Then every lane holds
// four complete output quaternions (registers 4j..4j+3), and a B fragment is
// two consecutive quaternions of one column: one 16-byte LDS read.  One MFMA
// block is 8 quaternion rows x 32 quaternion columns x 4 kappa.
//
// Accumulation.  One FP32 MFMA accumulator per output takes all NTERMS
// products; every `panel_tiles` K-tiles it is added into a second FP32
// accumulator and cleared, so rounding errors grow with the panel length
// rather than with K.
//
// Tile.  A block of 256 threads (4 waves, arranged WR x WC) computes BM x BN
// quaternions; a wave owns (BM/WR) x (BN/WC) = MB x NB MFMA blocks.  K
// advances in tiles of BK quaternions through one or two LDS stages.
// LDS (32-bit words): per stage, A as [piece][row][kappa][2 words] and B as
// [piece][column][kappa][2 words], row pitch 2 BK + 4 words.  The 16-byte pad
// spreads the 16-byte fragment reads of consecutive rows over the banks, and
// the staging threads are laid out so that their 8-byte writes do not collide
// either (slot_coords): no LDS bank conflicts for any op pair.
#pragma once

#include "qgemm_internal.hpp"

namespace qg {
namespace split {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;

// f32 pair -> packed bf16 pair (round to nearest even), low half = first
__device__ __forceinline__ unsigned pack_bf16(float x, float y)
{
    const bf16x2 v = __builtin_convertvector((f32x2){x, y}, bf16x2);
    return __builtin_bit_cast(unsigned, v);
}
__device__ __forceinline__ float lo_f32(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float hi_f32(unsigned w) { return __uint_as_float(w & 0xffff0000u); }

// Split two floats into three packed bf16 pairs (h, m, l).
__device__ __forceinline__ void split2(float x, float y, unsigned &h, unsigned &m, unsigned &l)
{
    h = pack_bf16(x, y);
    const float rx = x - lo_f32(h), ry = y - hi_f32(h);
    m = pack_bf16(rx, ry);
    const float sx = rx - lo_f32(m), sy = ry - hi_f32(m);
    l = pack_bf16(sx, sy);
}

// Row r of L(a) for one quaternion a held as two packed bf16 words
// w0 = (a0, a1), w1 = (a2, a3):
//   r = 0: ( a0, -a1, -a2, -a3)     r = 1: ( a1,  a0, -a3,  a2)
//   r = 2: ( a2,  a3,  a0, -a1)     r = 3: ( a3, -a2,  a1,  a0)
// Each output word is one byte permutation of (w1:w0) and one sign XOR.
struct LRow {
    unsigned sel0, sel1, neg0, neg1;
};
__device__ __forceinline__ LRow lrow(int r)
{
    // v_perm selectors over the 8 bytes {w1, w0}: bytes 0-3 = w0, 4-7 = w1
    constexpr unsigned P01 = 0x03020100u, P10 = 0x01000302u, P23 = 0x07060504u, P32 = 0x05040706u;
    LRow x;
    x.sel0 = r == 0 ? P01 : r == 1 ? P10 : r == 2 ? P23 : P32;
    x.sel1 = r == 0 ? P23 : r == 1 ? P32 : r == 2 ? P01 : P10;
    x.neg0 = (r == 0 || r == 3) ? 0x80000000u : 0u;
    x.neg1 = r == 0 ? 0x80008000u : r == 1 ? 0x00008000u : r == 2 ? 0x80000000u : 0u;
    return x;
}

__device__ __forceinline__ bf16x8 expand_a(u32x4 raw, const LRow &L)
{
    u32x4 o;
    o.x = __builtin_amdgcn_perm(raw.y, raw.x, L.sel0) ^ L.neg0;
    o.y = __builtin_amdgcn_perm(raw.y, raw.x, L.sel1) ^ L.neg1;
    o.z = __builtin_amdgcn_perm(raw.w, raw.z, L.sel0) ^ L.neg0;
    o.w = __builtin_amdgcn_perm(raw.w, raw.z, L.sel1) ^ L.neg1;
    return __builtin_bit_cast(bf16x8, o);
}

// (A piece, B piece) of each product, smallest first so that the large term
// lands on an accumulator already holding the corrections.
template <int NTERMS>
struct Terms;
template <>
struct Terms<3> {
    static constexpr int n = 3;
    static constexpr int a[3] = {1, 0, 0};
    static constexpr int b[3] = {0, 1, 0};
};
template <>
struct Terms<6> {
    static constexpr int n = 6;
    static constexpr int a[6] = {2, 1, 0, 1, 0, 0};
    static constexpr int b[6] = {0, 1, 2, 0, 1, 0};
};
template <>
struct Terms<9> {
    static constexpr int n = 9;
    static constexpr int a[9] = {2, 2, 1, 2, 1, 0, 1, 0, 0};
    static constexpr int b[9] = {2, 1, 2, 0, 1, 2, 0, 1, 0};
};

template <int BM_, int BN_, int WR_, int WC_, int BK_>
struct Tile {
    static constexpr int BM = BM_, BN = BN_, WR = WR_, WC = WC_, BK = BK_;
    static constexpr int MB = BM / WR / 8;                     // MFMA blocks per wave along M
    static constexpr int NB = BN / WC / 32;                    // MFMA blocks per wave along N
    static constexpr int RP = 2 * BK + 4;                      // words per LDS row (incl. 16-byte pad)
    static constexpr int A_STAGE = 3 * BM * RP;
    static constexpr int B_STAGE = 3 * BN * RP;
    static constexpr int STAGE = A_STAGE + B_STAGE;
    static constexpr size_t LDS_BYTES = 2 * STAGE * sizeof(unsigned);   // two stages
    static constexpr size_t LDS_BYTES_1 = STAGE * sizeof(unsigned);     // one stage
    static constexpr int A_Q = BM * BK / NT;                   // quaternions of A per thread per K-tile
    static constexpr int B_Q = BN * BK / NT;
    static_assert(WR * WC == 4, "four waves per block");
    static_assert(MB >= 1 && NB >= 1 && MB * WR * 8 == BM && NB * WC * 32 == BN, "wave tiling");
    static_assert(A_Q >= 1 && B_Q >= 1 && A_Q * NT == BM * BK && B_Q * NT == BN * BK, "tile split");
    static_assert(BK % 4 == 0, "BK must be a multiple of the MFMA kappa step");
};

// Staging slot qd of a ROWS x BK tile -> (row, kappa).  Every group of 16
// lanes writes 8-byte words that fall on 32 distinct banks of the row pitch
// 2 BK + 4 words: with the operand contiguous along the row index (ROW_FAST)
// the group takes 8 rows x 2 kappa; contiguous along kappa, one row of 16
// kappa (BK = 16) or two rows 4 apart of 8 kappa (BK = 8, 80 bytes x 4 rows
// = half the banks).  Global reads stay in runs of 8 or 16 quaternions.
template <int ROWS, int BK, bool ROW_FAST>
__device__ __forceinline__ void slot_coords(int qd, int &row, int &ka)
{
    static_assert(ROWS % 8 == 0 && (BK == 8 || BK == 16), "staging slot layout");
    const int lo = qd & 15, hi = qd >> 4;
    if constexpr (ROW_FAST) {
        row = (hi % (ROWS / 8)) * 8 + (lo & 7);
        ka = (hi / (ROWS / 8)) * 2 + (lo >> 3);
    } else if constexpr (BK == 8) {
        ka = lo & 7;
        row = (lo >> 3) * 4 + (hi & 3) + 8 * (hi >> 2);
    } else {
        ka = lo;
        row = hi;
    }
}

// Compute the BM x BN output tile at (m0, n0) of problem p and write it.
// nk = number of K-tiles to walk (0 when alpha == 0).  `lds` must hold
// TL::LDS_BYTES (STAGES = 2) or TL::LDS_BYTES_1 (STAGES = 1).  Every thread of
// the block must call this.  In both variants the next K-tile is fetched into
// registers while the current one is multiplied; with STAGES = 1 the block
// then stages it into the single LDS stage between two barriers and relies on
// a second resident block per CU to keep the matrix cores busy meanwhile.  BS: op(B) is scaled by
// p.bscale from the left at staging.
// Loads are buffer loads from a per-K-tile resource: a masked element gets
// the offset kOob, which the hardware reads as zero, so the K-loop has no
// branches.  In-tile byte offsets are below 2^31 (see split_offsets_fit).
// TRI = 1 (2): op(A) (op(B)) is the triangle of a triangular multiply: the
// tile walks only the K-tiles the triangle reaches, elements across the
// diagonal read as zero and a unit diagonal is staged in place of the
// (unread) element.
constexpr unsigned kOob = 0x80000000u;

template <class TL, bool TA, bool TB, int NTERMS, bool C64, int STAGES, bool BS = false, int TRI = 0>
__device__ __forceinline__ void split_tile(const GemmDesc<float> &p, double *c64, int m0, int n0, int nk,
                                           int panel_tiles, unsigned *lds)
{
    using TT = Terms<NTERMS>;
    constexpr int BM = TL::BM, BN = TL::BN, BK = TL::BK, MB = TL::MB, NB = TL::NB, RP = TL::RP;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave / TL::WC, wc = wave % TL::WC;

    const int fi = lane & 31;                 // A row / B column within the 32-wide MFMA block
    const int fg = lane >> 5;                 // k group: quaternions 2fg, 2fg+1 of the step
    LRow L = lrow(fi & 3);
    if (p.conjA) {
        // conj(a) negates a1..a3: flip the halves of each output word that come from them
        const int r = fi & 3;
        L.neg0 ^= r == 0 ? 0x80000000u : r == 1 ? 0x00008000u : 0x80008000u;
        L.neg1 ^= r == 1 ? 0x80008000u : r == 2 ? 0x80000000u : r == 3 ? 0x00008000u : 0x80008000u;
    }
    const unsigned conjB = p.conjB ? 0x80000000u : 0u;
    const int a_row = wr * (BM / TL::WR) + (fi >> 2);   // + 8 m
    const int b_row = wc * (BN / TL::WC) + fi;          // + 32 n

    f32x16 acc[MB][NB], tot[MB][NB];
#pragma unroll
    for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int n = 0; n < NB; ++n) {
            acc[m][n] = (f32x16){};
            tot[m][n] = (f32x16){};
        }

    // per-slot coordinates, in-tile byte offsets (kOob where the row is outside the matrix)
    int a_r[TL::A_Q], a_k[TL::A_Q], b_c[TL::B_Q], b_k[TL::B_Q];
    unsigned a_off[TL::A_Q], b_off[TL::B_Q];
#pragma unroll
    for (int i = 0; i < TL::A_Q; ++i) {
        const int qd = tid + NT * i;
        slot_coords<BM, BK, !TA>(qd, a_r[i], a_k[i]);
        a_off[i] = m0 + a_r[i] < p.M ? 16u * (TA ? (unsigned)a_r[i] * (unsigned)p.lda + a_k[i]
                                                 : (unsigned)a_k[i] * (unsigned)p.lda + a_r[i])
                                     : kOob;
    }
#pragma unroll
    for (int i = 0; i < TL::B_Q; ++i) {
        const int qd = tid + NT * i;
        slot_coords<BN, BK, TB>(qd, b_c[i], b_k[i]);
        b_off[i] = n0 + b_c[i] < p.N ? 16u * (TB ? (unsigned)b_k[i] * (unsigned)p.ldb + b_c[i]
                                                 : (unsigned)b_c[i] * (unsigned)p.ldb + b_k[i])
                                     : kOob;
    }

    u32x4 ra[TL::A_Q], rb[TL::B_Q];
    unsigned unit_bits = 0;   // slots of the loaded tile on a unit diagonal (triangular operand)

    // K-tiles this tile needs: all, or those a triangular operand reaches
    int kt0 = 0, kt1 = nk;
    if constexpr (TRI == 1) {
        if (p.tri_lower) kt1 = min(nk, (m0 + BM + BK - 1) / BK);   // op(A)[mu][k] = 0 for k > mu
        else kt0 = min(nk, m0 / BK);                                // op(A)[mu][k] = 0 for k < mu
    } else if constexpr (TRI == 2) {
        if (p.tri_lower) kt0 = min(nk, n0 / BK);                    // op(B)[k][nu] = 0 for k < nu
        else kt1 = min(nk, (n0 + BN + BK - 1) / BK);                // op(B)[k][nu] = 0 for k > nu
    }

    // fetch K-tile kt into registers (tiles at or past K read as zeros)
    auto load_tile = [&](int kt) {
        const int k0 = kt * BK;
        // the prefetch past this tile's K-range reads nothing (for a triangular
        // operand that K-tile lies in the triangle that must not be read)
        const int krem = (kt < kt1 ? p.K : 0) - k0;
        const float *Ab = p.A + 4 * (TA ? ((int64_t)m0 * p.lda + k0) : ((int64_t)k0 * p.lda + m0));
        const float *Bb = p.B + 4 * (TB ? ((int64_t)k0 * p.ldb + n0) : ((int64_t)n0 * p.ldb + k0));
        const __amdgpu_buffer_rsrc_t rA = __builtin_amdgcn_make_buffer_rsrc((void *)Ab, (short)0, 0x7fffffff, 0x00020000);
        const __amdgpu_buffer_rsrc_t rB = __builtin_amdgcn_make_buffer_rsrc((void *)Bb, (short)0, 0x7fffffff, 0x00020000);
        // only K-tiles that cross the diagonal of a triangular operand need its mask (uniform per block)
        const bool diagA = TRI == 1 && k0 < m0 + BM && k0 + BK > m0;
        const bool diagB = TRI == 2 && k0 < n0 + BN && k0 + BK > n0;
        if constexpr (TRI != 0) unit_bits = 0;
#pragma unroll
        for (int i = 0; i < TL::A_Q; ++i) {
            bool ok = a_k[i] < krem;
            if constexpr (TRI == 1) {
                if (diagA) {
                    const int gm = m0 + a_r[i], gk = k0 + a_k[i];
                    ok = ok && (p.tri_lower ? gk <= gm : gk >= gm) && !(p.tri_unit && gk == gm);
                    if (p.tri_unit && gk == gm && gm < p.M) unit_bits |= 1u << i;
                }
            }
            ra[i] = __builtin_amdgcn_raw_buffer_load_b128(rA, ok ? a_off[i] : kOob, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < TL::B_Q; ++i) {
            bool ok = b_k[i] < krem;
            if constexpr (TRI == 2) {
                if (diagB) {
                    const int gn = n0 + b_c[i], gk = k0 + b_k[i];
                    ok = ok && (p.tri_lower ? gk >= gn : gk <= gn) && !(p.tri_unit && gk == gn);
                    if (p.tri_unit && gk == gn && gn < p.N) unit_bits |= 1u << i;
                }
            }
            rb[i] = __builtin_amdgcn_raw_buffer_load_b128(rB, ok ? b_off[i] : kOob, 0, 0);
        }
    };

    auto put = [&](unsigned *plane0, int plane_words, int row, int ka, float x, float y, float z, float w) {
        unsigned h0, md0, l0, h1, md1, l1;
        split2(x, y, h0, md0, l0);
        split2(z, w, h1, md1, l1);
        unsigned *d = plane0 + row * RP + 2 * ka;
        *reinterpret_cast<uint2 *>(d) = make_uint2(h0, h1);
        *reinterpret_cast<uint2 *>(d + plane_words) = make_uint2(md0, md1);
        *reinterpret_cast<uint2 *>(d + 2 * plane_words) = make_uint2(l0, l1);
    };

    auto store_tile = [&](unsigned *As) {
        unsigned *Bs = As + TL::A_STAGE;
#pragma unroll
        for (int i = 0; i < TL::A_Q; ++i) {   // conj(A) is applied through L
            u32x4 v = ra[i];
            if constexpr (TRI == 1) {
                if ((unit_bits >> i) & 1u) v = (u32x4){0x3f800000u, 0u, 0u, 0u};   // unit diagonal
            }
            put(As, BM * RP, a_r[i], a_k[i], __uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z),
                __uint_as_float(v.w));
        }
#pragma unroll
        for (int i = 0; i < TL::B_Q; ++i) {
            u32x4 v = rb[i];
            if constexpr (TRI == 2) {
                if ((unit_bits >> i) & 1u) v = (u32x4){0x3f800000u, 0u, 0u, 0u};   // unit diagonal
            }
            float b[4] = {__uint_as_float(v.x), __uint_as_float(v.y ^ conjB),
                          __uint_as_float(v.z ^ conjB), __uint_as_float(v.w ^ conjB)};
            if constexpr (BS) {
                const float sc[4] = {(float)p.bscale[0], (float)p.bscale[1], (float)p.bscale[2], (float)p.bscale[3]};
                float t[4];
                qmul(sc, b, t);
                b[0] = t[0]; b[1] = t[1]; b[2] = t[2]; b[3] = t[3];
            }
            put(Bs, BN * RP, b_c[i], b_k[i], b[0], b[1], b[2], b[3]);
        }
    };

    auto compute = [&](const unsigned *As) {
        const unsigned *Bs = As + TL::A_STAGE;
#pragma unroll
        for (int ks = 0; ks < BK / 4; ++ks) {
            const int kw = (ks * 4 + 2 * fg) * 2;          // word offset of the kappa pair
            bf16x8 af[3][MB], bfr[3][NB];
#pragma unroll
            for (int pc = 0; pc < 3; ++pc) {
#pragma unroll
                for (int m = 0; m < MB; ++m) {
                    const u32x4 raw = *reinterpret_cast<const u32x4 *>(As + (pc * BM + a_row + 8 * m) * RP + kw);
                    af[pc][m] = expand_a(raw, L);
                }
#pragma unroll
                for (int n = 0; n < NB; ++n) {
                    const u32x4 raw = *reinterpret_cast<const u32x4 *>(Bs + (pc * BN + b_row + 32 * n) * RP + kw);
                    bfr[pc][n] = __builtin_bit_cast(bf16x8, raw);
                }
            }
#pragma unroll
            for (int t = 0; t < TT::n; ++t)
#pragma unroll
                for (int m = 0; m < MB; ++m)
#pragma unroll
                    for (int n = 0; n < NB; ++n)
                        acc[m][n] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[TT::a[t]][m], bfr[TT::b[t]][n],
                                                                            acc[m][n], 0, 0, 0);
        }
    };

    auto flush = [&]() {
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                tot[m][n] += acc[m][n];
                acc[m][n] = (f32x16){};
            }
    };

    unsigned *S0 = lds;
    if constexpr (STAGES == 2) {
        unsigned *S1 = lds + TL::STAGE;
        if (kt0 < kt1) {
            load_tile(kt0);
            store_tile(S0);
            __syncthreads();
        }
        // unrolled by two so that both stages are compile-time constants
        int kt = kt0;
        while (kt < kt1) {
            load_tile(kt + 1);
            compute(S0);
            store_tile(S1);
            __syncthreads();
            ++kt;
            if ((kt - kt0) % panel_tiles == 0) flush();
            if (kt >= kt1) break;
            load_tile(kt + 1);
            compute(S1);
            store_tile(S0);
            __syncthreads();
            ++kt;
            if ((kt - kt0) % panel_tiles == 0) flush();
        }
    } else {
        // one stage: the next K-tile's loads are issued before this tile's
        // MFMAs so their latency hides behind the compute
        if (kt0 < kt1) load_tile(kt0);
        for (int kt = kt0; kt < kt1; ++kt) {
            if (kt > kt0) __syncthreads();               // every wave is done reading the stage
            store_tile(S0);
            __syncthreads();
            load_tile(kt + 1);
            compute(S0);
            if ((kt + 1 - kt0) % panel_tiles == 0) flush();
        }
        __syncthreads();                                 // LDS may be reused by the caller
    }
    flush();

    // epilogue: a lane holds quaternions (registers 4j..4j+3) of rows 2j + lane/32 of each 8-row block.
    // The old C values of a group of outputs are all requested before the first of them is written, so
    // their latencies overlap (a read after a write to the same array is not reordered by the compiler).
    const bool beta_zero = p.beta[0] == 0.0 && p.beta[1] == 0.0 && p.beta[2] == 0.0 && p.beta[3] == 0.0;
    auto out_index = [&](int m, int n, int j, int &mu, int &nu, int64_t &e) -> bool {
        mu = m0 + a_row - (fi >> 2) + 8 * m + 2 * j + fg;
        nu = n0 + b_row + 32 * n;
        if (mu >= p.M || nu >= p.N) return false;
        if (p.uplo != 0 && (p.uplo == 1 ? mu < nu : mu > nu)) return false;
        e = p.store_t ? ((int64_t)mu * p.ldc + nu) : ((int64_t)nu * p.ldc + mu);
        return true;
    };
    if constexpr (C64) {
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int n = 0; n < NB; ++n) {
                double cold[4][4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    int mu, nu;
                    int64_t e = 0;
                    cold[j][0] = cold[j][1] = cold[j][2] = cold[j][3] = 0.0;
                    if (!beta_zero && out_index(m, n, j, mu, nu, e)) {
                        const double *src = c64 + 4 * e;
                        cold[j][0] = src[0]; cold[j][1] = src[1]; cold[j][2] = src[2]; cold[j][3] = src[3];
                    }
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    int mu, nu;
                    int64_t e;
                    if (!out_index(m, n, j, mu, nu, e)) continue;
                    const double v[4] = {tot[m][n][4 * j], tot[m][n][4 * j + 1], tot[m][n][4 * j + 2],
                                         tot[m][n][4 * j + 3]};
                    double o[4];
                    qmul(p.alpha, v, o);
                    if (p.has_right) {
                        const double t[4] = {o[0], o[1], o[2], o[3]};
                        qmul(t, p.alpha_r, o);
                    }
                    if (p.store_conj) { o[1] = -o[1]; o[2] = -o[2]; o[3] = -o[3]; }
                    if (!beta_zero) {
                        double u[4];
                        qmul(p.beta, cold[j], u);
                        if (p.has_right) {
                            const double t[4] = {u[0], u[1], u[2], u[3]};
                            qmul(t, p.beta_r, u);
                        }
                        o[0] += u[0]; o[1] += u[1]; o[2] += u[2]; o[3] += u[3];
                    }
                    if (p.herm_diag && mu == nu) o[1] = o[2] = o[3] = 0.0;
                    double *dst = c64 + 4 * e;
                    dst[0] = o[0]; dst[1] = o[1]; dst[2] = o[2]; dst[3] = o[3];
                }
            }
    } else {
        const float al[4] = {(float)p.alpha[0], (float)p.alpha[1], (float)p.alpha[2], (float)p.alpha[3]};
        const float be[4] = {(float)p.beta[0], (float)p.beta[1], (float)p.beta[2], (float)p.beta[3]};
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            f32x4 cold[NB][4];
#pragma unroll
            for (int n = 0; n < NB; ++n)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    int mu, nu;
                    int64_t e = 0;
                    cold[n][j] = (f32x4){};
                    if (!beta_zero && out_index(m, n, j, mu, nu, e))
                        cold[n][j] = *reinterpret_cast<const f32x4 *>(p.C + 4 * e);
                }
#pragma unroll
            for (int n = 0; n < NB; ++n)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    int mu, nu;
                    int64_t e;
                    if (!out_index(m, n, j, mu, nu, e)) continue;
                    const float v[4] = {tot[m][n][4 * j], tot[m][n][4 * j + 1], tot[m][n][4 * j + 2],
                                        tot[m][n][4 * j + 3]};
                    float o[4];
                    qmul(al, v, o);
                    if (p.has_right) {
                        const float ar[4] = {(float)p.alpha_r[0], (float)p.alpha_r[1], (float)p.alpha_r[2],
                                             (float)p.alpha_r[3]};
                        const float t[4] = {o[0], o[1], o[2], o[3]};
                        qmul(t, ar, o);
                    }
                    if (p.store_conj) { o[1] = -o[1]; o[2] = -o[2]; o[3] = -o[3]; }
                    if (!beta_zero) {
                        const float cq[4] = {cold[n][j].x, cold[n][j].y, cold[n][j].z, cold[n][j].w};
                        float u[4];
                        qmul(be, cq, u);
                        if (p.has_right) {
                            const float br[4] = {(float)p.beta_r[0], (float)p.beta_r[1], (float)p.beta_r[2],
                                                 (float)p.beta_r[3]};
                            const float t[4] = {u[0], u[1], u[2], u[3]};
                            qmul(t, br, u);
                        }
                        o[0] += u[0]; o[1] += u[1]; o[2] += u[2]; o[3] += u[3];
                    }
                    if (p.herm_diag && mu == nu) o[1] = o[2] = o[3] = 0.f;
                    *reinterpret_cast<f32x4 *>(p.C + 4 * e) = (f32x4){o[0], o[1], o[2], o[3]};
                }
        }
    }
}

// In-tile byte offsets of the largest tile must stay below 2^31 (the masked
// offset kOob): the farthest element read is ((BM-1) lda + BK) for a
// transposed A and (BK lda + BM) otherwise (likewise for B), 16 bytes each.
inline bool split_offsets_fit(int64_t lda, int64_t ldb, bool ta, bool tb, int BM, int BN, int BK)
{
    const int64_t lim = (int64_t)1 << 31;
    const int64_t fa = 16 * (ta ? (BM * lda + BK) : (BK * lda + BM));
    const int64_t fb = 16 * (tb ? (BK * ldb + BN) : (BN * ldb + BK));
    return fa < lim && fb < lim;
}

}  // namespace split
}  // namespace qg
