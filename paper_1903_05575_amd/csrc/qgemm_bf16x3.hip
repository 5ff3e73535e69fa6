// Single FP32-stored quaternion GEMM on the split-BF16 tile of
// qgemm_bf16x3_tile.hpp: one 64 x 64-quaternion tile per block, four waves
// stacked along M (each 16 rows x 64 columns = 2 x 2 MFMA blocks), two blocks
// per CU, blocks ordered XCD-aware.  Two K pipelines:
//   TL2: K-tiles of 8 quaternions through two LDS stages (31 KB each, one
//        barrier per K-tile) -- used when the grid fills two blocks per CU,
//        where the other block covers each block's staging; measured 2-4%
//        faster than TL1 there, and its op N/N instantiation does not spill;
//   TL3: 32 x 64 tiles on the TL2 pipeline -- for full outputs whose 64-row
//        grid fills the block slots clearly worse (e.g. 1024 x 1024 outputs:
//        256 tiles of 64 x 64 for 512 slots);
//   TL1: K-tiles of 16 quaternions through one LDS stage (two barriers per
//        K-tile, half as many K-tiles) -- for the remaining grids of fewer
//        tiles than slots, where each CU holds one block and the per-K-tile
//        overhead is exposed.
#include "qgemm_bf16x3_tile.hpp"

namespace qg {
namespace {

using TL1 = split::Tile<64, 64, 4, 1, 16>;
using TL2 = split::Tile<64, 64, 4, 1, 8>;
using TL3 = split::Tile<32, 64, 4, 1, 8>;   // 32-row tiles for grids that 64-row tiles fill poorly

template <class TL, bool TA, bool TB, int NTERMS, bool C64, int STAGES, int TRI>
__global__ __launch_bounds__(split::NT, 2) void qgemm_bf16x3_kernel(GemmDesc<float> p, double *c64, int tiles_m,
                                                                    int tiles_n, int nk, int panel_tiles)
{
    extern __shared__ unsigned lds[];
    int tm, tn;
    if constexpr (TRI != 0) {   // triangular operand: work depends on the tile row (1) or column (2) only
        xcd_chunk_tile(blockIdx.x, gridDim.x, tiles_m, tiles_n, TRI == 1, (TRI == 1) == p.tri_lower, tm, tn);
        split::split_tile<TL, TA, TB, NTERMS, C64, STAGES, false, TRI>(p, c64, tm * TL::BM, tn * TL::BN, nk,
                                                                       panel_tiles, lds);
    } else {
        if (p.uplo == 0) xcd_tile(blockIdx.x, gridDim.x, tiles_m, tiles_n, 8, tm, tn);
        else xcd_tri_tile(blockIdx.x, gridDim.x, p.uplo == 1, tm, tn);   // triangular output: its tiles only
        if (p.has_bscale)
            split::split_tile<TL, TA, TB, NTERMS, C64, STAGES, true>(p, c64, tm * TL::BM, tn * TL::BN, nk,
                                                                     panel_tiles, lds);
        else
            split::split_tile<TL, TA, TB, NTERMS, C64, STAGES, false>(p, c64, tm * TL::BM, tn * TL::BN, nk,
                                                                      panel_tiles, lds);
    }
}

template <class TL, bool TA, bool TB, int NTERMS, bool C64, int STAGES, int TRI>
hipError_t launch_s(const GemmDesc<float> &d, double *c64, int panel, int64_t nblocks, hipStream_t stream)
{
    auto kern = &qgemm_bf16x3_kernel<TL, TA, TB, NTERMS, C64, STAGES, TRI>;
    constexpr size_t lds_bytes = STAGES == 1 ? TL::LDS_BYTES_1 : TL::LDS_BYTES;
    static std::atomic<uint64_t> lds_set{0};
    hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void *>(kern), (int)lds_bytes, lds_set);
    if (e != hipSuccess) return e;
    const int tiles_m = (d.M + TL::BM - 1) / TL::BM;
    const int tiles_n = (d.N + TL::BN - 1) / TL::BN;
    const bool alpha_zero = d.alpha[0] == 0.0 && d.alpha[1] == 0.0 && d.alpha[2] == 0.0 && d.alpha[3] == 0.0;
    const int nk = alpha_zero ? 0 : (d.K + TL::BK - 1) / TL::BK;
    const int panel_tiles = panel / TL::BK > 0 ? panel / TL::BK : 1;
    hipLaunchKernelGGL(kern, dim3((unsigned)nblocks), dim3(split::NT), lds_bytes, stream, d, c64, tiles_m, tiles_n,
                       nk, panel_tiles);
    return hipGetLastError();
}

// Fraction of the block slots (two per CU) that a grid of `tiles` equal tiles
// keeps busy over its rounds.
double slot_fill(int64_t tiles, int64_t slots)
{
    const int64_t rounds = (tiles + slots - 1) / slots;
    return rounds > 0 ? (double)tiles / (double)(rounds * slots) : 1.0;
}

template <bool TA, bool TB, int NTERMS, bool C64, int TRI>
hipError_t launch_t(const GemmDesc<float> &d, double *c64, int panel, hipStream_t stream)
{
    static_assert(TL1::BM == TL2::BM && TL1::BN == TL2::BN && TL3::BN == TL2::BN, "same tile widths");
    static_assert(TL1::BM == TL1::BN, "triangular launches need square tiles");
    const int tiles_m = (d.M + TL1::BM - 1) / TL1::BM;
    const int tiles_n = (d.N + TL1::BN - 1) / TL1::BN;
    const int64_t nblocks = d.uplo == 0 ? (int64_t)tiles_m * tiles_n : (int64_t)tiles_m * (tiles_m + 1) / 2;
    if (nblocks <= 0) return hipSuccess;
    if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
    if constexpr (TRI == 0) {
        const int64_t slots = 2 * (int64_t)device_cus();
        if (d.uplo == 0 && slots > 0) {
            const int64_t tiles32 = (int64_t)((d.M + TL3::BM - 1) / TL3::BM) * tiles_n;
            if (slot_fill(tiles32, slots) > 1.1 * slot_fill(nblocks, slots))
                return launch_s<TL3, TA, TB, NTERMS, C64, 2, TRI>(d, c64, panel, tiles32, stream);
        }
        if (nblocks < slots) return launch_s<TL1, TA, TB, NTERMS, C64, 1, TRI>(d, c64, panel, nblocks, stream);
    }
    return launch_s<TL2, TA, TB, NTERMS, C64, 2, TRI>(d, c64, panel, nblocks, stream);
}

template <int NTERMS, bool C64, int TRI = 0>
hipError_t dispatch_ops(const GemmDesc<float> &d, double *c64, int panel, hipStream_t s)
{
    if (d.opA_t) return d.opB_t ? launch_t<true, true, NTERMS, C64, TRI>(d, c64, panel, s)
                                : launch_t<true, false, NTERMS, C64, TRI>(d, c64, panel, s);
    return d.opB_t ? launch_t<false, true, NTERMS, C64, TRI>(d, c64, panel, s)
                   : launch_t<false, false, NTERMS, C64, TRI>(d, c64, panel, s);
}

template <int TRI>
hipError_t dispatch_tri(const GemmDesc<float> &d, int nterms, int panel, hipStream_t s)
{
    switch (nterms) {
    case 3: return dispatch_ops<3, false, TRI>(d, nullptr, panel, s);
    case 9: return dispatch_ops<9, false, TRI>(d, nullptr, panel, s);
    default: return dispatch_ops<6, false, TRI>(d, nullptr, panel, s);
    }
}

}  // namespace

hipError_t launch_qgemm_bf16x3(const GemmDesc<float> &d, double *c64, int nterms, int panel, hipStream_t stream)
{
    // every pipeline must address its K-tiles with 32-bit offsets
    if (!split::split_offsets_fit(d.lda, d.ldb, d.opA_t, d.opB_t, TL1::BM, TL1::BN, TL1::BK) ||
        !split::split_offsets_fit(d.lda, d.ldb, d.opA_t, d.opB_t, TL2::BM, TL2::BN, TL2::BK) ||
        !split::split_offsets_fit(d.lda, d.ldb, d.opA_t, d.opB_t, TL3::BM, TL3::BN, TL3::BK))
        return hipErrorInvalidValue;
    if (d.tri != 0) {
        // a triangular operand is square and comes without a scale, a triangular output or an FP64 result
        if (c64 || d.has_bscale || d.uplo != 0 || (d.tri == 1 ? d.K != d.M : d.K != d.N)) return hipErrorInvalidValue;
        return d.tri == 1 ? dispatch_tri<1>(d, nterms, panel, stream) : dispatch_tri<2>(d, nterms, panel, stream);
    }
    if (c64) {
        switch (nterms) {
        case 3: return dispatch_ops<3, true>(d, c64, panel, stream);
        case 9: return dispatch_ops<9, true>(d, c64, panel, stream);
        default: return dispatch_ops<6, true>(d, c64, panel, stream);
        }
    }
    switch (nterms) {
    case 3: return dispatch_ops<3, false>(d, c64, panel, stream);
    case 9: return dispatch_ops<9, false>(d, c64, panel, stream);
    default: return dispatch_ops<6, false>(d, c64, panel, stream);
    }
}

}  // namespace qg
