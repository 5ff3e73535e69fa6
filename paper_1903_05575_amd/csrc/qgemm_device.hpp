// Device helpers shared by the GEMM kernels of libqgemm.so (internal).
#pragma once

#include <hip/hip_runtime.h>

namespace qg {

// 32-bit lane-constant sign mask of row r / column c of the real 4x4
// left-multiplication block L(a) with vec(a b) = L(a) vec(b):
//   L(a) = [[a0,-a1,-a2,-a3],[a1,a0,-a3,a2],[a2,a3,a0,-a1],[a3,-a2,a1,a0]]
// derived from Eq. quaternion_prod.  Entry (r, c) equals
// sign(r, c) * a[r ^ c]; bit 4r+c of kLNegMask is set where sign is -1.
constexpr unsigned kLNegMask = (1u << 1) | (1u << 2) | (1u << 3) | (1u << 6) | (1u << 11) | (1u << 13);

__host__ __device__ inline bool l_negative(int r, int c) { return (kLNegMask >> (4 * r + c)) & 1u; }

// Hamilton product p q on the device (Eq. quaternion_prod), used by the
// epilogue for the left scalars.  Kept separate from any CPU reference.
template <typename T>
__device__ __forceinline__ void qmul(const T p[4], const T q[4], T out[4])
{
    out[0] = p[0] * q[0] - p[1] * q[1] - p[2] * q[2] - p[3] * q[3];
    out[1] = p[0] * q[1] + p[1] * q[0] + p[2] * q[3] - p[3] * q[2];
    out[2] = p[0] * q[2] - p[1] * q[3] + p[2] * q[0] + p[3] * q[1];
    out[3] = p[0] * q[3] + p[1] * q[2] - p[2] * q[1] + p[3] * q[0];
}

// Blocks are dispatched round-robin over the 8 XCDs of the MI355X (block b
// runs on XCD b % 8, each XCD with its own L2).  Renumber so that every XCD
// owns one contiguous range of work ids.
__device__ __forceinline__ int xcd_id(int bid, int nblocks)
{
    const int xcd = bid & 7;
    const int local = bid >> 3;
    const int per = nblocks >> 3;
    const int rem = nblocks & 7;
    return (xcd < rem) ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// Tile of a tiles_m x tiles_n grid for block bid: XCD-contiguous ids rastered
// in groups of `group` tile rows, so neighbouring tiles on one XCD share A and
// B panels.
__device__ __forceinline__ void xcd_tile(int bid, int nblocks, int tiles_m, int tiles_n,
                                         int group, int &tm, int &tn)
{
    const int id = xcd_id(bid, nblocks);
    const int gsz = group * tiles_n;
    const int g = id / gsz;
    const int first_m = g * group;
    const int gm = min(tiles_m - first_m, group);
    const int within = id - g * gsz;
    tm = first_m + within % gm;
    tn = within / gm;
}

// Tile of the lower (tm >= tn) or upper (tm <= tn) triangle of a square tile
// grid for block bid; the grid has exactly T (T + 1) / 2 blocks, enumerated
// row by row of the lower triangle, so every XCD gets an equal share.
__device__ __forceinline__ void xcd_tri_tile(int bid, int nblocks, bool lower, int &tm, int &tn)
{
    const int id = xcd_id(bid, nblocks);
    int r = (int)((sqrt(8.0 * (double)id + 1.0) - 1.0) * 0.5);
    while ((int64_t)r * (r + 1) / 2 > id) --r;
    while ((int64_t)(r + 1) * (r + 2) / 2 <= id) ++r;
    const int c = id - r * (r + 1) / 2;
    tm = lower ? r : c;
    tn = lower ? c : r;
}

// Tile for block bid when the work of a tile depends only on its tile row
// (by_rows) or only on its tile column, as in a triangular multiply.  Tiles
// are listed heaviest first (reverse: the heaviest row or column is the last
// one) in groups of 8 rows (columns), each group rastered across the other
// axis, so 64 consecutive list entries form an 8 x 8 patch.  In every full run
// of 512 blocks (64 per XCD) XCD x takes the x-th patch of the run: the XCDs
// always work on neighbouring patches of nearly equal weight, each patch
// sharing its operand panels in one L2.  The last partial run is taken in
// list order.  The map is a bijection from [0, tiles_m * tiles_n).
__device__ __forceinline__ void xcd_chunk_tile(int bid, int nblocks, int tiles_m, int tiles_n, bool by_rows,
                                               bool reverse, int &tm, int &tn)
{
    int pos = bid;
    if (bid < (nblocks & ~511)) pos = (bid & ~511) + 64 * (bid & 7) + ((bid & 511) >> 3);
    const int nw = by_rows ? tiles_m : tiles_n;
    const int no = by_rows ? tiles_n : tiles_m;
    const int gsz = 8 * no;
    const int g = pos / gsz;
    const int first = g * 8;
    const int gw = min(nw - first, 8);
    const int within = pos - g * gsz;
    int w = first + within % gw;
    const int o = within / gw;
    if (reverse) w = nw - 1 - w;
    tm = by_rows ? w : o;
    tn = by_rows ? o : w;
}

}  // namespace qg
