// FP64 quaternion GEMM on the gfx950 FP64 matrix cores: one launch of
// f64_tile (qgemm_f64_tile.hpp, which describes the method, the MFMA
// mapping, the tiling and the LDS layouts) per output tile, ordered
// XCD-aware.
#include "qgemm_f64_tile.hpp"

namespace qg {
namespace {

using namespace f64;

template <int BMT, bool TA, bool TB, bool BS, int TRI, int BNT = BN>
__global__ __launch_bounds__(NT, (FTile<BMT, TRI, BNT>::MIN_BLOCKS)) void qgemm_f64_kernel(GemmDesc<double> p,
                                                                                          int tiles_m, int tiles_n,
                                                                                          int nk)
{
    extern __shared__ double smem[];
    int tm, tn;
    if constexpr (TRI != 0)   // work depends on the tile row (TRI 1) or column (TRI 2) only
        xcd_chunk_tile(blockIdx.x, gridDim.x, tiles_m, tiles_n, TRI == 1, (TRI == 1) == p.tri_lower, tm, tn);
    else if (p.uplo == 0) xcd_tile(blockIdx.x, gridDim.x, tiles_m, tiles_n, 8, tm, tn);
    else xcd_tri_tile(blockIdx.x, gridDim.x, p.uplo == 1, tm, tn);   // triangular output: its tiles only
    f64_tile<BMT, TA, TB, BS, TRI, BNT>(p, tm * FTile<BMT, TRI, BNT>::BM, tn * BNT, nk, smem);
}

template <int BMT, bool TA, bool TB, bool BS, int TRI, int BNT = BN>
hipError_t launch_t(const GemmDesc<double> &d, hipStream_t stream)
{
    using FT = FTile<BMT, TRI, BNT>;
    if (d.uplo != 0 && FT::BM != BNT) return hipErrorInvalidValue;   // the triangular grid needs square tiles
    static std::atomic<uint64_t> lds_set{0};
    hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void *>(&qgemm_f64_kernel<BMT, TA, TB, BS, TRI, BNT>),
                                      (int)FT::LDS_BYTES, lds_set);
    if (e != hipSuccess) return e;
    const int tiles_m = (d.M + FT::BM - 1) / FT::BM;
    const int tiles_n = (d.N + BNT - 1) / BNT;
    const bool alpha_zero = d.alpha[0] == 0.0 && d.alpha[1] == 0.0 && d.alpha[2] == 0.0 && d.alpha[3] == 0.0;
    const int nk = alpha_zero ? 0 : (d.K + FT::BK - 1) / FT::BK;
    const int64_t nblocks = d.uplo == 0 ? (int64_t)tiles_m * tiles_n : (int64_t)tiles_m * (tiles_m + 1) / 2;
    if (nblocks <= 0) return hipSuccess;
    if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((qgemm_f64_kernel<BMT, TA, TB, BS, TRI, BNT>), dim3((unsigned)nblocks), dim3(NT), FT::LDS_BYTES,
                       stream, d, tiles_m, tiles_n, nk);
    return hipGetLastError();
}

template <int BMT, bool BS, int TRI, int BNT = BN>
hipError_t launch_ops_t(const GemmDesc<double> &d, hipStream_t stream)
{
    if (d.opA_t)
        return d.opB_t ? launch_t<BMT, true, true, BS, TRI, BNT>(d, stream)
                       : launch_t<BMT, true, false, BS, TRI, BNT>(d, stream);
    return d.opB_t ? launch_t<BMT, false, true, BS, TRI, BNT>(d, stream)
                   : launch_t<BMT, false, false, BS, TRI, BNT>(d, stream);
}

// Fraction of the block slots that a grid of `tiles` equal tiles keeps busy over its rounds.
double slot_fill(int64_t tiles, int64_t slots)
{
    const int64_t rounds = (tiles + slots - 1) / slots;
    return rounds > 0 ? (double)tiles / (double)(rounds * slots) : 1.0;
}

// Full outputs and triangular operands use 32 x 64 tiles with 4-kappa K-tiles
// (FTile<32>): four blocks per CU (123 VGPRs, 25 KB of LDS each, so 16 waves)
// keep the matrix pipes busier than two blocks of 64-row tiles (224 VGPRs,
// 8 waves), and twice as many tiles fill small grids better.  Measured on op
// N/N against the 64-row tiles: 2048^3 88.3% -> 89.8-90.0% of the FP64 peak,
// 4096^3 89.5% -> 90.8-91.2%, 8192^3 89.9% -> 91.1-91.6%; an 8192 left lower
// triangular multiply 131.7 -> 126.7 ms.
// Triangular outputs (herk) keep square 64 x 64 tiles: a grid of the 32 x 64
// tiles that meet the triangle measured 129 -> 138 ms at N = K = 8192 (more
// of each tile on the diagonal is computed and then masked).
template <bool BS, int TRI>
hipError_t launch_ops(const GemmDesc<double> &d, hipStream_t stream)
{
    if constexpr (TRI != 0) {
        return launch_ops_t<32, BS, TRI>(d, stream);
    } else {
        if (d.uplo == 0) {
            // Grids that 32 x 64 tiles fill poorly (1024 x 1024 outputs: 512 tiles for 1024 block slots) take
            // 32 x 32 tiles with 8-kappa K-tiles, also four blocks per CU, when those fill the slots more than
            // 10% better over their rounds.  Measured: 1024^3 66.0 -> 67.5 TFLOP/s, 1536^3 62.0 -> 68.3;
            // 2048^3 and larger keep 32 x 64 tiles (their grids fill the slots).
            const int64_t slots = (int64_t)FTile<32, 0>::MIN_BLOCKS * device_cus();
            const int64_t tm = (d.M + 31) / 32, t64 = tm * ((d.N + 63) / 64), t32 = tm * ((d.N + 31) / 32);
            if (slots > 0 && slot_fill(t32, slots) > 1.1 * slot_fill(t64, slots))
                return launch_ops_t<32, BS, 0, 32>(d, stream);
            return launch_ops_t<32, BS, 0>(d, stream);
        }
        if constexpr (BS) return hipErrorInvalidValue;   // no scaled operand with a triangular output
        else return launch_ops_t<64, false, 0>(d, stream);
    }
}

}  // namespace

hipError_t launch_qgemm_f64(const GemmDesc<double> &d, hipStream_t stream)
{
    if (!f64_ld_supported(d.lda, d.ldb, d.opA_t, d.opB_t)) return hipErrorInvalidValue;
    if (d.tri != 0) {
        // a triangular operand is square and comes without a scale or a triangular output
        if (d.has_bscale || d.uplo != 0 || (d.tri == 1 ? d.K != d.M : d.K != d.N)) return hipErrorInvalidValue;
        return d.tri == 1 ? launch_ops<false, 1>(d, stream) : launch_ops<false, 2>(d, stream);
    }
    return d.has_bscale ? launch_ops<true, 0>(d, stream) : launch_ops<false, 0>(d, stream);
}

}  // namespace qg
