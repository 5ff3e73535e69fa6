// Grouped (batched) quaternion GEMM: thousands of independent problems of
// uneven size in one persistent launch, of the split-BF16 tile for FP32
// problems or of the FP64 tile (qgemm_f64_tile.hpp) for FP64 problems.
//
// Plan (host, outside any capture): every problem is cut into output tiles
// whose shape is looked up per size class in the tuned tile table
// (tile_table.inc; FP64 problems all take the 32 x 64 FP64 tile); the
// (problem, tile) work items are sorted by cost
// (padded MFMA work + a fixed per-tile overhead) and dealt to the persistent
// blocks longest-processing-time first, each block receiving a contiguous
// run of the item array.  The block slots of the assignment are numbered so
// that consecutive slots run on one XCD: the equal-cost tiles of a problem,
// dealt one after another, then mostly share one L2 for its A and B panels
// (2.08 -> 2.01 ms on 4096 problems of sizes log-uniform in [8, 512]).
// Problem descriptors, items and per-block offsets go to device memory once.
// Run (capture-safe): a single launch of three (FP32) or four (FP64) blocks
// per CU; block b walks items [start[b], start[b+1]).  No allocation, copy,
// memset or atomic.
#include "qgemm_bf16x3_tile.hpp"
#include "qgemm_f64_tile.hpp"

#include "../../include/qgemm.h"

#include <algorithm>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <queue>
#include <vector>

namespace qg {
namespace {

#include "tile_table.inc"

// One problem as the kernels read it; the arrays are float (FP32 plans) or
// double (FP64 plans).
struct DevProblem {
    const void *A;
    const void *B;
    void *C;
    int64_t lda, ldb, ldc;
    int M, N, K, pad;
};

// Tile classes.  No 64 x 64 class: without it the kernel fits three blocks
// per CU (at most 41.5 KB of LDS and 168 VGPRs each), which hides more of the
// per-item latency than the larger tile saved (measured on the 4096-problem
// workload: 2.33 -> 2.13 ms); the tuner had picked 64 x 64 for only three
// size classes, by at most 20%.
using T0 = split::Tile<32, 64, 4, 1, 16>;
using T1 = split::Tile<64, 32, 4, 1, 16>;
using T2 = split::Tile<32, 32, 4, 1, 16>;
using T3 = split::Tile<16, 64, 2, 2, 16>;
constexpr int kClasses = 4;
constexpr int kBM[kClasses] = {32, 64, 32, 16};
constexpr int kBN[kClasses] = {64, 32, 32, 64};
constexpr int kBK = 16;
constexpr size_t kLds = T0::LDS_BYTES_1 > T1::LDS_BYTES_1 ? T0::LDS_BYTES_1 : T1::LDS_BYTES_1;
static_assert(T2::LDS_BYTES_1 <= kLds && T3::LDS_BYTES_1 <= kLds, "LDS sized for the largest tile");
constexpr int kBlocksPerCU = 3;
static_assert(kBlocksPerCU * kLds <= 160 * 1024, "resident blocks fit the LDS of a CU");

struct Scalars {
    double alpha[4];
    double beta[4];
    int conjA, conjB;
};

template <bool TA, bool TB, int NTERMS>
__global__ __launch_bounds__(split::NT, kBlocksPerCU) void grouped_kernel(const DevProblem *__restrict__ probs,
                                                             const int4 *__restrict__ items,
                                                             const int *__restrict__ starts, Scalars s,
                                                             int panel_tiles)
{
    extern __shared__ unsigned lds[];
    const bool alpha_zero = s.alpha[0] == 0.0 && s.alpha[1] == 0.0 && s.alpha[2] == 0.0 && s.alpha[3] == 0.0;
    const int end = starts[blockIdx.x + 1];
    for (int w = starts[blockIdx.x]; w < end; ++w) {
        const int4 it = items[w];                       // (problem, tile row, tile column, class)
        const DevProblem pr = probs[it.x];
        GemmDesc<float> d;
        d.A = static_cast<const float *>(pr.A);
        d.B = static_cast<const float *>(pr.B);
        d.C = static_cast<float *>(pr.C);
        d.lda = pr.lda;
        d.ldb = pr.ldb;
        d.ldc = pr.ldc;
        d.M = pr.M;
        d.N = pr.N;
        d.K = pr.K;
        d.opA_t = TA;
        d.opB_t = TB;
        d.conjA = s.conjA != 0;
        d.conjB = s.conjB != 0;
        d.has_bscale = false;
        d.store_t = false;
        d.store_conj = false;
        d.has_right = false;
        d.uplo = 0;
        d.herm_diag = false;
        d.tri = 0;
        d.tri_lower = false;
        d.tri_unit = false;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            d.alpha[i] = s.alpha[i];
            d.beta[i] = s.beta[i];
            d.bscale[i] = 0.0;
            d.alpha_r[i] = 0.0;
            d.beta_r[i] = 0.0;
        }
        const int nk = alpha_zero ? 0 : (pr.K + kBK - 1) / kBK;
        switch (it.w) {
        case 0: split::split_tile<T0, TA, TB, NTERMS, false, 1>(d, nullptr, it.y * 32, it.z * 64, nk, panel_tiles, lds); break;
        case 1: split::split_tile<T1, TA, TB, NTERMS, false, 1>(d, nullptr, it.y * 64, it.z * 32, nk, panel_tiles, lds); break;
        case 2: split::split_tile<T2, TA, TB, NTERMS, false, 1>(d, nullptr, it.y * 32, it.z * 32, nk, panel_tiles, lds); break;
        default: split::split_tile<T3, TA, TB, NTERMS, false, 1>(d, nullptr, it.y * 16, it.z * 64, nk, panel_tiles, lds); break;
        }
        // no barrier here: the one-stage tile ends its K-loop on one, so every wave is done with LDS
    }
}

// FP64 problems: one tile class, the 32 x 64 tile of the single FP64 GEMM
// (K-tiles of 4, 25 KB of LDS, four blocks per CU).
using F64T = f64::FTile<32, 0>;
constexpr int kF64BM = F64T::BM, kF64BN = f64::BN, kF64BK = F64T::BK;
constexpr int kF64BlocksPerCU = F64T::MIN_BLOCKS;
static_assert(kF64BlocksPerCU * F64T::LDS_BYTES <= 160 * 1024, "resident FP64 blocks fit the LDS of a CU");

template <bool TA, bool TB>
__global__ __launch_bounds__(f64::NT, kF64BlocksPerCU) void grouped_f64_kernel(const DevProblem *__restrict__ probs,
                                                                            const int4 *__restrict__ items,
                                                                            const int *__restrict__ starts, Scalars s)
{
    extern __shared__ double smem64[];
    const bool alpha_zero = s.alpha[0] == 0.0 && s.alpha[1] == 0.0 && s.alpha[2] == 0.0 && s.alpha[3] == 0.0;
    const int end = starts[blockIdx.x + 1];
    for (int w = starts[blockIdx.x]; w < end; ++w) {
        const int4 it = items[w];                       // (problem, tile row, tile column, class)
        const DevProblem pr = probs[it.x];
        GemmDesc<double> d;
        d.A = static_cast<const double *>(pr.A);
        d.B = static_cast<const double *>(pr.B);
        d.C = static_cast<double *>(pr.C);
        d.lda = pr.lda;
        d.ldb = pr.ldb;
        d.ldc = pr.ldc;
        d.M = pr.M;
        d.N = pr.N;
        d.K = pr.K;
        d.opA_t = TA;
        d.opB_t = TB;
        d.conjA = s.conjA != 0;
        d.conjB = s.conjB != 0;
        d.has_bscale = false;
        d.store_t = false;
        d.store_conj = false;
        d.has_right = false;
        d.uplo = 0;
        d.herm_diag = false;
        d.tri = 0;
        d.tri_lower = false;
        d.tri_unit = false;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            d.alpha[i] = s.alpha[i];
            d.beta[i] = s.beta[i];
            d.bscale[i] = 0.0;
            d.alpha_r[i] = 0.0;
            d.beta_r[i] = 0.0;
        }
        const int nk = alpha_zero ? 0 : (pr.K + kF64BK - 1) / kF64BK;
        // f64_tile leaves smem free for the next item (its K-loop ends on a barrier)
        f64::f64_tile<32, TA, TB, false, 0>(d, it.y * kF64BM, it.z * kF64BN, nk, smem64);
    }
}

int bucket_mn(int64_t x) { return x <= 16 ? 0 : x <= 32 ? 1 : x <= 64 ? 2 : 3; }
int bucket_k(int64_t x) { return x <= 64 ? 0 : 1; }

template <bool TA, bool TB, int NTERMS>
hipError_t set_attr()
{
    static std::atomic<uint64_t> lds_set{0};
    return ensure_dynamic_lds(reinterpret_cast<const void *>(&grouped_kernel<TA, TB, NTERMS>), (int)kLds, lds_set);
}

template <int NTERMS>
hipError_t launch_n(bool ta, bool tb, dim3 grid, hipStream_t st, const DevProblem *p, const int4 *it,
                    const int *starts, Scalars s, int panel_tiles)
{
#define QG_GROUPED_CASE(A_, B_)                                                                         \
    if (ta == A_ && tb == B_) {                                                                         \
        hipError_t e = set_attr<A_, B_, NTERMS>();                                                      \
        if (e != hipSuccess) return e;                                                                  \
        hipLaunchKernelGGL((grouped_kernel<A_, B_, NTERMS>), grid, dim3(split::NT), kLds, st, p, it, starts, s, \
                           panel_tiles);                                                                \
        return hipGetLastError();                                                                       \
    }
    QG_GROUPED_CASE(false, false)
    QG_GROUPED_CASE(false, true)
    QG_GROUPED_CASE(true, false)
    QG_GROUPED_CASE(true, true)
#undef QG_GROUPED_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_f64(bool ta, bool tb, dim3 grid, hipStream_t st, const DevProblem *p, const int4 *it,
                      const int *starts, Scalars s)
{
#define QG_GROUPED_F64_CASE(A_, B_)                                                                     \
    if (ta == A_ && tb == B_) {                                                                         \
        static std::atomic<uint64_t> lds_set{0};                                                        \
        hipError_t e = ensure_dynamic_lds(reinterpret_cast<const void *>(&grouped_f64_kernel<A_, B_>),  \
                                          (int)F64T::LDS_BYTES, lds_set);                               \
        if (e != hipSuccess) return e;                                                                  \
        hipLaunchKernelGGL((grouped_f64_kernel<A_, B_>), grid, dim3(f64::NT), F64T::LDS_BYTES, st, p, it, starts, s); \
        return hipGetLastError();                                                                       \
    }
    QG_GROUPED_F64_CASE(false, false)
    QG_GROUPED_F64_CASE(false, true)
    QG_GROUPED_F64_CASE(true, false)
    QG_GROUPED_F64_CASE(true, true)
#undef QG_GROUPED_F64_CASE
    return hipErrorInvalidValue;
}

}  // namespace

struct GroupedPlan {
    int device = 0;
    bool f64 = false;                            // FP64 problems (else FP32 on the split path)
    bool ta = false, tb = false;
    int nterms = 6;
    Scalars s{};
    DevProblem *d_probs = nullptr;
    int4 *d_items = nullptr;
    int *d_starts = nullptr;
    int64_t nitems = 0;
    int grid = 0;
    int64_t class_count[kClasses] = {};
};

// The table in effect: the tuned one compiled in, or one installed at run
// time (qgemm_batched_set_tile_table, the tuner's hook).  Guarded by a mutex;
// a plan takes one copy of it when it is created.
namespace {
std::mutex g_table_mutex;
unsigned char g_table[4][4][2];
bool g_table_custom = false;
}  // namespace

void grouped_set_table(const unsigned char *t)
{
    std::lock_guard<std::mutex> lk(g_table_mutex);
    g_table_custom = t != nullptr;
    if (t) memcpy(g_table, t, sizeof(g_table));
}

void grouped_get_table(unsigned char *t)
{
    std::lock_guard<std::mutex> lk(g_table_mutex);
    memcpy(t, g_table_custom ? &g_table[0][0][0] : &kTileTable[0][0][0], sizeof(g_table));
}

// Tile geometry of class cls: FP64 plans have one class (32 x 64, K-tiles of
// 4), FP32 plans the four split-BF16 classes.
struct TileDims {
    int bm, bn, bk;
};
TileDims tile_dims(bool f64, int cls)
{
    if (f64) return {kF64BM, kF64BN, kF64BK};
    return {kBM[cls], kBN[cls], kBK};
}

// Build a plan.  `probs` have been validated by the caller.  force_class < 0
// selects the tile class from the table (FP32) or the single FP64 class,
// otherwise it is used for every problem.  Returns QGEMM_OK, QGEMM_ERR_ALLOC,
// QGEMM_ERR_HIP, QGEMM_ERR_UNSUPPORTED (more than 2^31 - 1 tiles), or
// -(i + 1) when the leading dimensions of problem i are beyond the tile
// addressing.  Host containers may throw std::bad_alloc; the C-ABI caller
// turns that into QGEMM_ERR_ALLOC.
int grouped_plan_create(GroupedPlan **out, bool f64, bool ta, bool tb, bool ca, bool cb, int nterms,
                        const double alpha[4], const double beta[4], int64_t count, const ::qgemm_problem_t *probs,
                        int force_class)
{
    std::unique_ptr<GroupedPlan> owner(new (std::nothrow) GroupedPlan());
    if (!owner) return QGEMM_ERR_ALLOC;
    GroupedPlan *pl = owner.get();
    pl->f64 = f64;
    pl->ta = ta;
    pl->tb = tb;
    pl->s.conjA = ca ? 1 : 0;
    pl->s.conjB = cb ? 1 : 0;
    pl->nterms = nterms;
    for (int i = 0; i < 4; ++i) {
        pl->s.alpha[i] = alpha[i];
        pl->s.beta[i] = beta[i];
    }
    unsigned char table[4][4][2];                // one consistent table for the whole plan
    grouped_get_table(&table[0][0][0]);
    auto class_of = [&](const ::qgemm_problem_t &q) {
        if (f64) return 0;
        return force_class >= 0 ? force_class : (int)table[bucket_mn(q.M)][bucket_mn(q.N)][bucket_k(q.K)];
    };
    // count the tiles first: item indices and block starts are 32-bit on the device
    int64_t total_tiles = 0;
    for (int64_t i = 0; i < count; ++i) {
        const ::qgemm_problem_t &q = probs[i];
        if (q.M == 0 || q.N == 0) continue;
        const TileDims t = tile_dims(f64, class_of(q));
        total_tiles += ((q.M + t.bm - 1) / t.bm) * ((q.N + t.bn - 1) / t.bn);
        if (total_tiles > 0x7fffffff) return QGEMM_ERR_UNSUPPORTED;
    }
    std::vector<DevProblem> hp((size_t)count);
    std::vector<int4> items;
    std::vector<double> cost;
    items.reserve((size_t)total_tiles);
    cost.reserve((size_t)total_tiles);
    for (int64_t i = 0; i < count; ++i) {
        const ::qgemm_problem_t &q = probs[i];
        DevProblem &d = hp[(size_t)i];
        d.A = q.A;
        d.B = q.B;
        d.C = q.C;
        d.lda = q.lda;
        d.ldb = q.ldb;
        d.ldc = q.ldc;
        d.M = (int)q.M;
        d.N = (int)q.N;
        d.K = (int)q.K;
        d.pad = 0;
        if (q.M == 0 || q.N == 0) continue;
        const int cls = class_of(q);
        const TileDims t = tile_dims(f64, cls);
        const bool fits = f64 ? f64_ld_supported(q.lda, q.ldb, ta, tb)
                              : split::split_offsets_fit(q.lda, q.ldb, ta, tb, t.bm, t.bn, t.bk);
        if (!fits) return -(int)(i + 1);           // caller reports QGEMM_ERR_UNSUPPORTED for problem i
        const int tm = (int)((q.M + t.bm - 1) / t.bm);
        const int tn = (int)((q.N + t.bn - 1) / t.bn);
        const int64_t kp = ((q.K + t.bk - 1) / t.bk) * t.bk;
        for (int a = 0; a < tm; ++a)
            for (int b = 0; b < tn; ++b) {
                items.push_back(make_int4((int)i, a, b, cls));
                // padded MFMA work of the tile plus a fixed cost of one tile start/epilogue
                cost.push_back((double)t.bm * t.bn * (double)(kp + 48));
            }
        pl->class_count[cls] += (int64_t)tm * tn;
    }
    pl->nitems = (int64_t)items.size();
    if (pl->nitems > 0x7fffffff) return QGEMM_ERR_UNSUPPORTED;   // item indices and block starts are 32-bit
    if (hipGetDevice(&pl->device) != hipSuccess) return QGEMM_ERR_HIP;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, pl->device) != hipSuccess)
        return QGEMM_ERR_HIP;
    const int64_t per_cu = f64 ? kF64BlocksPerCU : kBlocksPerCU;
    const int64_t G = std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * per_cu, pl->nitems));
    pl->grid = (int)G;
    // longest processing time first: each item to the least loaded block
    std::vector<int64_t> order(items.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return cost[a] > cost[b]; });
    using Slot = std::pair<double, int>;
    std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> heap;
    for (int b = 0; b < G; ++b) heap.push({0.0, b});
    std::vector<std::vector<int4>> per((size_t)G);
    for (int64_t k : order) {
        Slot s = heap.top();
        heap.pop();
        per[(size_t)s.second].push_back(items[(size_t)k]);
        heap.push({s.first + cost[(size_t)k], s.second});
    }
    std::vector<int4> flat;
    flat.reserve(items.size());
    std::vector<int> starts((size_t)G + 1, 0);
    for (int b = 0; b < G; ++b) {
        // block b runs on XCD b % 8; consecutive slots go to the same XCD
        const int x = b & 7, per_x = (int)(G >> 3), rem = (int)(G & 7);
        const int slot = (x < rem ? x * (per_x + 1) : rem * (per_x + 1) + (x - rem) * per_x) + (b >> 3);
        starts[(size_t)b] = (int)flat.size();
        flat.insert(flat.end(), per[(size_t)slot].begin(), per[(size_t)slot].end());
    }
    starts[(size_t)G] = (int)flat.size();

    auto fail = [&](int code) {
        (void)hipFree(pl->d_probs);
        (void)hipFree(pl->d_items);
        (void)hipFree(pl->d_starts);
        return code;                               // `owner` deletes the plan
    };
    if (hipMalloc(&pl->d_probs, sizeof(DevProblem) * std::max<size_t>(1, hp.size())) != hipSuccess)
        return fail(QGEMM_ERR_ALLOC);
    if (hipMalloc(&pl->d_items, sizeof(int4) * std::max<size_t>(1, flat.size())) != hipSuccess)
        return fail(QGEMM_ERR_ALLOC);
    if (hipMalloc(&pl->d_starts, sizeof(int) * starts.size()) != hipSuccess) return fail(QGEMM_ERR_ALLOC);
    if (!hp.empty() &&
        hipMemcpy(pl->d_probs, hp.data(), sizeof(DevProblem) * hp.size(), hipMemcpyHostToDevice) != hipSuccess)
        return fail(QGEMM_ERR_HIP);
    if (!flat.empty() &&
        hipMemcpy(pl->d_items, flat.data(), sizeof(int4) * flat.size(), hipMemcpyHostToDevice) != hipSuccess)
        return fail(QGEMM_ERR_HIP);
    if (hipMemcpy(pl->d_starts, starts.data(), sizeof(int) * starts.size(), hipMemcpyHostToDevice) != hipSuccess)
        return fail(QGEMM_ERR_HIP);
    *out = owner.release();
    return QGEMM_OK;
}

int grouped_plan_run(const GroupedPlan *pl, hipStream_t stream)
{
    if (pl->nitems == 0) return QGEMM_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev != pl->device) return QGEMM_ERR_INVALID_ARG;
    const dim3 grid((unsigned)pl->grid);
    if (pl->f64) {
        const hipError_t e = launch_f64(pl->ta, pl->tb, grid, stream, pl->d_probs, pl->d_items, pl->d_starts, pl->s);
        return e == hipSuccess ? QGEMM_OK : QGEMM_ERR_HIP;
    }
    const int panel_tiles = kSplitPanel / kBK;
    hipError_t e;
    switch (pl->nterms) {
    case 3: e = launch_n<3>(pl->ta, pl->tb, grid, stream, pl->d_probs, pl->d_items, pl->d_starts, pl->s, panel_tiles); break;
    case 9: e = launch_n<9>(pl->ta, pl->tb, grid, stream, pl->d_probs, pl->d_items, pl->d_starts, pl->s, panel_tiles); break;
    default: e = launch_n<6>(pl->ta, pl->tb, grid, stream, pl->d_probs, pl->d_items, pl->d_starts, pl->s, panel_tiles); break;
    }
    return e == hipSuccess ? QGEMM_OK : QGEMM_ERR_HIP;
}

void grouped_plan_destroy(GroupedPlan *pl)
{
    if (!pl) return;
    (void)hipFree(pl->d_probs);
    (void)hipFree(pl->d_items);
    (void)hipFree(pl->d_starts);
    delete pl;
}

void grouped_plan_info(const GroupedPlan *pl, int64_t *nitems, int *grid, int64_t *class_count)
{
    if (nitems) *nitems = pl->nitems;
    if (grid) *grid = pl->grid;
    if (class_count)
        for (int c = 0; c < kClasses; ++c) class_count[c] = pl->class_count[c];
}

}  // namespace qg
