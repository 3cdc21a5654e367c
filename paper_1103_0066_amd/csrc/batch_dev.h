// Heterogeneous batches on the device: one persistent kernel integrates the
// 256-element tiles of many meshes and forms, taking tiles from a work
// counter (the paper's element batches, Sec. 4, extended across meshes).
//
// Every workgroup loops: pop `tiles_per_pop` tiles with one atomic, find the
// item each tile belongs to (binary search over the items' first tiles),
// run that form's tile function on LDS carved from one dynamic buffer, and
// stop when the counter passes the last tile.  Items are ordered heaviest
// first on the host, so the tail of the queue holds the cheapest tiles.
#pragma once

#include "adjoint.h"
#include "fwd_mfma.h"

namespace fei {

// Staging rows per form for the two batch variants.  Forward: 0 stages whole
// matrices (the single-mesh default, at most 76 KB of LDS per workgroup), 1
// two rows at a time (near 28 KB).  Adjoint: 0 keeps LDS at or below 92 KB,
// 1 near 28 KB.
template <int F, int D, int VAR>
constexpr int batch_rows()
{
    constexpr int N = Traits<F, D>::N;
    if constexpr (VAR == 0 || N == 3) return N;
    else return 2;
}

template <int F, int D, int VAR>
constexpr int batch_adj_rows()
{
    constexpr int N = Traits<F, D>::N;
    if constexpr (N == 3) return 0;
    else if constexpr (VAR == 0) return (N == 12) ? 4 : N;
    else return 2;
}

template <int F, int D, int PREC, int VAR>
struct BatchFwdTile {
    // FP32: staged FMA tile; MFMA: staged (VAR 0) or direct (VAR 1) stores
    using Fma = FwdFmaTile<F, D, float, batch_rows<F, D, VAR>()>;
    using Mfma = MfmaTile<F, D, float, (PREC == P_FP32 ? P_FP16X2 : PREC), VAR == 1>;
    static constexpr int LDS_BYTES = (PREC == P_FP32) ? Fma::LDS_BYTES : Mfma::LDS_BYTES;
    __device__ __forceinline__ static void run(const FwdParams &p, int64_t blk, unsigned char *smem)
    {
        if constexpr (PREC == P_FP32) Fma::run(p, blk, smem);
        else Mfma::run(p, blk, smem);
    }
};

template <int F, int D, int VAR, bool GATHER = false>
struct BatchAdjTile {
    using Tile = AdjTile<F, D, float, batch_adj_rows<F, D, VAR>(), GATHER>;
    static constexpr int LDS_BYTES = Tile::LDS_BYTES;
};

constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <int PREC, int VAR>
constexpr int batch_fwd_lds()
{
    return cmax(cmax(cmax(BatchFwdTile<LAP1, 2, PREC, VAR>::LDS_BYTES,
                          BatchFwdTile<LAP1, 3, PREC, VAR>::LDS_BYTES),
                     cmax(BatchFwdTile<ELA1, 2, PREC, VAR>::LDS_BYTES,
                          BatchFwdTile<ELA1, 3, PREC, VAR>::LDS_BYTES)),
                cmax(cmax(BatchFwdTile<LAP2, 2, PREC, VAR>::LDS_BYTES,
                          BatchFwdTile<LAP2, 3, PREC, VAR>::LDS_BYTES), 16));
}

template <int VAR>
constexpr int batch_adj_lds()
{
    return cmax(cmax(cmax(BatchAdjTile<LAP1, 2, VAR>::LDS_BYTES, BatchAdjTile<LAP1, 3, VAR>::LDS_BYTES),
                     cmax(BatchAdjTile<ELA1, 2, VAR>::LDS_BYTES, BatchAdjTile<ELA1, 3, VAR>::LDS_BYTES)),
                cmax(BatchAdjTile<LAP2, 2, VAR>::LDS_BYTES, BatchAdjTile<LAP2, 3, VAR>::LDS_BYTES));
}

// Item owning global tile t (items sorted by tile_begin; uniform per workgroup).
__device__ __forceinline__ int batch_find_item(const BatchLaunch &b, int64_t t)
{
    int lo = 0, hi = b.n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.items[mid].tile_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int PREC, int VAR>
__device__ __forceinline__ void batch_fwd_dispatch(const BatchItemDev &d, int64_t blk,
                                                   unsigned char *smem)
{
    const int key = d.form * 4 + d.dim;
    switch (key) {
    case LAP1 * 4 + 2: BatchFwdTile<LAP1, 2, PREC, VAR>::run(d.fp, blk, smem); break;
    case LAP1 * 4 + 3: BatchFwdTile<LAP1, 3, PREC, VAR>::run(d.fp, blk, smem); break;
    case ELA1 * 4 + 2: BatchFwdTile<ELA1, 2, PREC, VAR>::run(d.fp, blk, smem); break;
    case ELA1 * 4 + 3: BatchFwdTile<ELA1, 3, PREC, VAR>::run(d.fp, blk, smem); break;
    case LAP2 * 4 + 2: BatchFwdTile<LAP2, 2, PREC, VAR>::run(d.fp, blk, smem); break;
    case LAP2 * 4 + 3: BatchFwdTile<LAP2, 3, PREC, VAR>::run(d.fp, blk, smem); break;
    default: break;
    }
}

template <int VAR>
__device__ __forceinline__ void batch_adj_dispatch(const BatchItemDev &d, int64_t blk,
                                                   unsigned char *smem)
{
    const int key = d.form * 4 + d.dim;
    switch (key) {
    case LAP1 * 4 + 2: BatchAdjTile<LAP1, 2, VAR>::Tile::run(d.ap, blk, smem); break;
    case LAP1 * 4 + 3: BatchAdjTile<LAP1, 3, VAR>::Tile::run(d.ap, blk, smem); break;
    case ELA1 * 4 + 2: BatchAdjTile<ELA1, 2, VAR>::Tile::run(d.ap, blk, smem); break;
    case ELA1 * 4 + 3: BatchAdjTile<ELA1, 3, VAR>::Tile::run(d.ap, blk, smem); break;
    case LAP2 * 4 + 2: BatchAdjTile<LAP2, 2, VAR>::Tile::run(d.ap, blk, smem); break;
    case LAP2 * 4 + 3: BatchAdjTile<LAP2, 3, VAR>::Tile::run(d.ap, blk, smem); break;
    default: break;
    }
}

// Persistent loop shared by the forward and adjoint kernels.  The tiles are
// split into kBatchCounters contiguous ranges, each with its own work counter
// (one device-wide counter serialized every pop at the memory side).  A
// workgroup starts on the range of its XCD (workgroups are dispatched
// round-robin over the 8 XCDs, blockIdx mod 8) and, once that range is
// drained, takes tiles from the following ranges in turn; every tile is taken
// exactly once (one atomic per pop), and every workgroup exits after finding
// all ranges drained -- also when fewer than 8 workgroups run.
template <bool ADJ, int PREC, int VAR>
__device__ __forceinline__ void batch_loop(const BatchLaunch &b, unsigned char *smem)
{
    __shared__ long long s_tile;
    const int x0 = int(blockIdx.x % kBatchCounters);
    for (int hop = 0; hop < kBatchCounters; ++hop) {
        const int x = (x0 + hop) % kBatchCounters;
        const int64_t r0 = x * b.n_tiles / kBatchCounters;
        const int64_t r1 = (x + 1) * b.n_tiles / kBatchCounters;
        for (;;) {
            if (threadIdx.x == 0) s_tile = r0 + atomicAdd(b.counter + x, b.tiles_per_pop);
            __syncthreads();
            const int64_t t0 = s_tile;
            __syncthreads();
            if (t0 >= r1) break;
            const int64_t t1 = (t0 + b.tiles_per_pop < r1) ? t0 + b.tiles_per_pop : r1;
            for (int64_t t = t0; t < t1; ++t) {
                const int it = batch_find_item(b, t);
                const BatchItemDev &d = b.items[it];
                if constexpr (ADJ) batch_adj_dispatch<VAR>(d, t - d.tile_begin, smem);
                else batch_fwd_dispatch<PREC, VAR>(d, t - d.tile_begin, smem);
                __syncthreads();  // LDS is reused by the next tile
            }
        }
    }
}

template <int PREC, int VAR>
__global__ __launch_bounds__(256) void batch_fwd_kernel(BatchLaunch b)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    batch_loop<false, PREC, VAR>(b, smem);
}

template <int VAR>
__global__ __launch_bounds__(256) void batch_adj_kernel(BatchLaunch b)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    batch_loop<true, P_FP32, VAR>(b, smem);
}

// One (form, dim) group of a batch as an ordinary grid: workgroup b takes
// the group's tile b.  Specialized per form, so registers and LDS are those
// of that form alone; the plan captures the groups as concurrent branches of
// one graph.  GATHER: the adjoint writes J-bar and has no vertex table.
template <int F, int D, int PREC, int VAR, bool ADJ, bool GATHER = false>
__global__ __launch_bounds__(256) void batch_group_kernel(BatchLaunch b)
{
    using FT = BatchFwdTile<F, D, PREC, VAR>;
    using AT = typename BatchAdjTile<F, D, VAR, GATHER>::Tile;
    constexpr int LDS = ADJ ? AT::LDS_BYTES : FT::LDS_BYTES;
    __shared__ __attribute__((aligned(16))) unsigned char smem[LDS > 16 ? LDS : 16];
    const int64_t t = xcd_block(blockIdx.x, gridDim.x);
    const int it = batch_find_item(b, t);
    const BatchItemDev &d = b.items[it];
    if constexpr (ADJ) AT::run(d.ap, t - d.tile_begin, smem);
    else FT::run(d.fp, t - d.tile_begin, smem);
}

// Work-counter reset as a kernel node (graphs get no memset nodes).
__global__ void batch_reset_kernel(int32_t *counter)
{
    if (threadIdx.x < kBatchCounters) counter[threadIdx.x] = 0;
}

}  // namespace fei
