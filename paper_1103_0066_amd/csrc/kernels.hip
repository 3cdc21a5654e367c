// All device code of libfei: kernel instantiations and the launcher tables
// the host layer dispatches through.  One translation unit, so the
// device-global reference tables (K fragments, sparse K) exist once per
// device module.
#include <algorithm>
#include <type_traits>

#include "adjoint.h"
#include "assemble.h"
#include "batch_dev.h"
#include "gather.h"
#include "fwd_coef.h"
#include "fwd_form.h"
#include "fwd_iso.h"
#include "fwd_fma.h"
#include "fwd_mfma.h"

// K tables (block tensor and MFMA fragments), emitted by gen_tables.cpp.
#include "_gen/tables.inc"

namespace fei {

namespace {

constexpr int kBlock = 256;

// Persistent grid: as many workgroups as fit on the device at once (queried
// once per kernel instantiation), at most one per tile.
template <auto KERNEL>
int persistent_grid(int64_t n_tiles)
{
    static const int64_t resident = []() -> int64_t {
        int dev = 0, blocks = 0, n_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, KERNEL, kBlock, 0) != hipSuccess ||
            blocks < 1 || n_cu < 1)
            return 256;
        return int64_t(blocks) * n_cu;
    }();
    return int(resident < n_tiles ? resident : n_tiles);
}

// A persistent kernel over the 256-element workgroup tiles.
template <auto KERNEL, typename P>
hipError_t launch_persistent(const P &p, hipStream_t s)
{
    const int64_t n_tiles = (p.m.n_elements + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(KERNEL, dim3(persistent_grid<KERNEL>(n_tiles)), dim3(kBlock), 0, s, p,
                       n_tiles);
    return hipGetLastError();
}

template <int F, int D, typename CT, int R, int WAVES = 4>
hipError_t launch_fwd_fma(const FwdParams &p, hipStream_t s)
{
    const int64_t per = 64 * WAVES;
    const int64_t n_groups = (p.m.n_elements + per - 1) / per;
    hipLaunchKernelGGL((fwd_fma_kernel<F, D, CT, R, WAVES>), dim3(unsigned(n_groups)),
                       dim3(unsigned(per)), 0, s, p);
    return hipGetLastError();
}

// MFMA forward: one workgroup per tile, except for fragment sets above 32
// per lane (3D elasticity in BF16x3: 45), which a persistent grid loads once
// per workgroup instead of once per tile (each measured the faster for its
// form on MI355X).
template <int F, int D, typename CT, int PREC, bool DIRECT>
hipError_t launch_fwd_mfma(const FwdParams &p, hipStream_t s)
{
    if constexpr (MfmaShape<F, D, PREC>::MT * MfmaShape<F, D, PREC>::KS > 32) {
        return launch_persistent<fwd_mfma_kernel<F, D, CT, PREC, DIRECT, true>>(p, s);
    } else {
        const int64_t n_groups = (p.m.n_elements + kBlock - 1) / kBlock;
        hipLaunchKernelGGL((fwd_mfma_kernel<F, D, CT, PREC, DIRECT, false>), dim3(unsigned(n_groups)),
                           dim3(kBlock), 0, s, p, n_groups);
        return hipGetLastError();
    }
}

template <int F, int D, typename CT, int R, bool GATHER = false>
hipError_t launch_adj_fma(const AdjParams &p, hipStream_t s)
{
    if constexpr (GATHER || AdjTile<F, D, CT, R, false>::WHOLE) {
        const int64_t n_tiles = (p.m.n_elements + kBlock - 1) / kBlock;
        if (n_tiles == 0) return hipSuccess;
        hipLaunchKernelGGL((adj_tile_kernel<F, D, CT, R, GATHER>), dim3(unsigned(n_tiles)),
                           dim3(kBlock), 0, s, p);
        return hipGetLastError();
    } else {
        return launch_persistent<adj_fma_kernel<F, D, CT, R>>(p, s);
    }
}

template <int F, int D, int PREC, bool GATHER>
hipError_t launch_adj_mfma(const AdjParams &p, hipStream_t s)
{
    return launch_persistent<adj_mfma_kernel<F, D, PREC, GATHER>>(p, s);
}

// Split-precision adjoint: the MFMA fold over whole staged matrices (n*n a
// multiple of 4: every form but the 3 x 3 matrices of the 2D P1 Laplacian),
// FP32 coordinates.
template <int F, int D>
AdjLauncher adj_mfma_for(const Variant &v)
{
    constexpr int N = Traits<F, D>::N;
    if constexpr ((N * N) % 4 != 0) {
        return nullptr;
    } else {
        if (v.coord_f64 || (v.rows != 0 && v.rows != N)) return nullptr;
        const bool g = v.gather != 0;
        switch (v.precision) {
        case P_FP16X2: return g ? &launch_adj_mfma<F, D, P_FP16X2, true> : &launch_adj_mfma<F, D, P_FP16X2, false>;
        case P_BF16X2: return g ? &launch_adj_mfma<F, D, P_BF16X2, true> : &launch_adj_mfma<F, D, P_BF16X2, false>;
        case P_BF16X3: return g ? &launch_adj_mfma<F, D, P_BF16X3, true> : &launch_adj_mfma<F, D, P_BF16X3, false>;
        default: return nullptr;
        }
    }
}

// Staging rows R that fit: R divides n, R*n floats is a whole number of
// 16-byte pieces, and four waves' staging buffers fit in the 160 KB LDS.
template <int F, int D, int R>
constexpr bool rows_ok()
{
    constexpr int N = Traits<F, D>::N;
    return R == 0 || (N % R == 0 && (R * N) % 4 == 0 && 4 * 64 * (R * N + 4) * 4 <= 160 * 1024);
}

// The forward also stages whole matrices of any size (packed when n*n is not
// a multiple of 4).
template <int F, int D, int R>
constexpr bool fwd_rows_ok()
{
    return rows_ok<F, D, R>() || R == Traits<F, D>::N;
}

// Tuned defaults of the staging rows (measured on MI355X).  Forward: whole
// matrices (each staged chunk leaves as one contiguous run; row chunks leave
// strided runs and measured up to 2.5x slower); adjoint: small chunks (two
// rows of the 12 x 12 matrices), so that two workgroups with their
// vertex-merge tables fit in a CU's LDS and registers (3D elasticity: 250 us
// at R = 2 against 268-280 us at R = 3, 4).
template <int F, int D>
constexpr int default_rows()
{
    return Traits<F, D>::N;
}

// Adjoint staging defaults (measured on MI355X).  Whole matrices (R = n,
// staged 64 or 32 elements at a time, line-aligned) for the 4 x 4 and
// 10 x 10 matrices: 3D P1 Laplacian 144 -> 132 us, 3D P2 Laplacian 204 ->
// 178 us (direct per-lane reads before).  The 12 x 12 elasticity matrices
// keep 2-row chunks in the persistent, software-pipelined kernel: whole
// 32-matrix chunks leave no registers for an in-flight chunk next to the
// 45 folded sums and measured 388 against 265 us.
template <int F, int D>
constexpr int default_adj_rows()
{
    constexpr int N = Traits<F, D>::N;
    if constexpr (N == 4 || N == 10) return N;
    else if constexpr (N == 12 || N == 6) return 2;
    else return 0;
}

// The gather form (no vertex table, one workgroup per tile): R = 4 for 3D
// elasticity (measured against R = 2, 3 and whole matrices: 260 vs 395 us),
// whole matrices for the 10 x 10 ones (183 vs 206 us at R = 2).
template <int F, int D>
constexpr int default_gather_rows()
{
    constexpr int N = Traits<F, D>::N;
    return N == 12 ? 4 : default_adj_rows<F, D>();
}

template <int F, int D, typename CT, int R>
FwdLauncher fwd_fma_if_ok()
{
    if constexpr (fwd_rows_ok<F, D, R>()) return &launch_fwd_fma<F, D, CT, R>;
    else return nullptr;
}

// The adjoint also holds two R-row chunks of dA per lane in registers (the
// one being folded and the next one in flight): R*n <= 48 floats each.  The
// larger chunks spill (3D elasticity with R = 6: 14x slower, measured), so
// they are not offered.
template <int F, int D, typename CT, int R>
AdjLauncher adj_fma_if_ok()
{
    if constexpr (rows_ok<F, D, R>() && (R * Traits<F, D>::N <= 48 || R == Traits<F, D>::N))
        return &launch_adj_fma<F, D, CT, R>;
    else return nullptr;
}

inline int resolve_rows(int rows, int def) { return rows == 0 ? def : (rows < 0 ? 0 : rows); }

template <int F, int D, typename CT>
FwdLauncher fwd_fma_rows(int rows)
{
    switch (resolve_rows(rows, default_rows<F, D>())) {
    case 0: return fwd_fma_if_ok<F, D, CT, 0>();
    case 2: return fwd_fma_if_ok<F, D, CT, 2>();
    case 3: return fwd_fma_if_ok<F, D, CT, 3>();
    case 4: return fwd_fma_if_ok<F, D, CT, 4>();
    case 6: return fwd_fma_if_ok<F, D, CT, 6>();
    case 10: return fwd_fma_if_ok<F, D, CT, 10>();
    case 12: return fwd_fma_if_ok<F, D, CT, 12>();
    default: return nullptr;
    }
}

template <int F, int D, typename CT>
AdjLauncher adj_fma_rows(int rows)
{
    switch (resolve_rows(rows, default_adj_rows<F, D>())) {
    case 0: return adj_fma_if_ok<F, D, CT, 0>();
    case 2: return adj_fma_if_ok<F, D, CT, 2>();
    case 3: return adj_fma_if_ok<F, D, CT, 3>();
    case 4: return adj_fma_if_ok<F, D, CT, 4>();
    case 6: return adj_fma_if_ok<F, D, CT, 6>();
    case 10: return adj_fma_if_ok<F, D, CT, 10>();
    case 12: return adj_fma_if_ok<F, D, CT, 12>();
    default: return nullptr;
    }
}

// Elements per workgroup other than 256 (FP32 coordinates, default staging).
template <int F, int D>
FwdLauncher fwd_fma_block(int block)
{
    constexpr int R = default_rows<F, D>();
    switch (block) {
    case 64: return &launch_fwd_fma<F, D, float, R, 1>;
    case 128: return &launch_fwd_fma<F, D, float, R, 2>;
    case 512: return &launch_fwd_fma<F, D, float, R, 8>;
    default: return nullptr;
    }
}

template <int F, int D, typename CT>
FwdLauncher fwd_for_prec(const Variant &v)
{
    if (v.block != 0 && v.block != 256) {
        if (v.precision != P_FP32 || v.rows != 0 || !std::is_same<CT, float>::value) return nullptr;
        return fwd_fma_block<F, D>(v.block);
    }
    if (v.precision == P_FP32) return fwd_fma_rows<F, D, CT>(v.rows);
    // MFMA form: staged stores of whole matrices (0, or rows = n), or direct (-1)
    const bool direct = v.rows < 0;
    if (v.rows > 0 && v.rows != Traits<F, D>::N) return nullptr;
    switch (v.precision) {
    case P_FP16X2:
        return direct ? &launch_fwd_mfma<F, D, CT, P_FP16X2, true>
                      : &launch_fwd_mfma<F, D, CT, P_FP16X2, false>;
    case P_BF16X2:
        return direct ? &launch_fwd_mfma<F, D, CT, P_BF16X2, true>
                      : &launch_fwd_mfma<F, D, CT, P_BF16X2, false>;
    case P_BF16X3:
        return direct ? &launch_fwd_mfma<F, D, CT, P_BF16X3, true>
                      : &launch_fwd_mfma<F, D, CT, P_BF16X3, false>;
    default: return nullptr;
    }
}

template <int F, int D>
FwdLauncher fwd_for_coords(const Variant &v)
{
    return v.coord_f64 ? fwd_for_prec<F, D, double>(v) : fwd_for_prec<F, D, float>(v);
}

template <int F, int D>
AdjLauncher adj_for_coords(const Variant &v)
{
    if (v.precision != P_FP32) return adj_mfma_for<F, D>(v);
    if (v.gather) {   // plans' vertex gather: FP32 coordinates, default staging
        if (v.coord_f64 || v.rows != 0) return nullptr;
        return &launch_adj_fma<F, D, float, default_gather_rows<F, D>(), true>;
    }
    return v.coord_f64 ? adj_fma_rows<F, D, double>(v.rows) : adj_fma_rows<F, D, float>(v.rows);
}

__global__ void validate_kernel(MeshView m, int nv_per, unsigned long long *n_bad)
{
    const int64_t total = m.n_elements * nv_per;
    unsigned long long bad = 0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int32_t v = m.conn[i];
        bad += (v < 0 || int64_t(v) >= m.n_vertices) ? 1ull : 0ull;
    }
    if (bad) atomicAdd(n_bad, bad);
}

}  // namespace

FwdLauncher find_forward(const Variant &v)
{
    if (v.dim == 2) {
        switch (v.form) {
        case LAP1: return fwd_for_coords<LAP1, 2>(v);
        case ELA1: return fwd_for_coords<ELA1, 2>(v);
        case LAP2: return fwd_for_coords<LAP2, 2>(v);
        }
    } else if (v.dim == 3) {
        switch (v.form) {
        case LAP1: return fwd_for_coords<LAP1, 3>(v);
        case ELA1: return fwd_for_coords<ELA1, 3>(v);
        case LAP2: return fwd_for_coords<LAP2, 3>(v);
        }
    }
    return nullptr;
}

namespace {

template <int F, int D, typename CT, int R>
hipError_t launch_fwd_coef(const FwdParams &p, hipStream_t s)
{
    const int64_t n_groups = (p.m.n_elements + kBlock - 1) / kBlock;
    hipLaunchKernelGGL((fwd_coef_kernel<F, D, CT, R>), dim3(unsigned(n_groups)), dim3(kBlock), 0,
                       s, p);
    return hipGetLastError();
}

template <int F, int D, typename CT>
FwdLauncher fwd_coef_rows(int rows)
{
    constexpr int N = Traits<F, D>::N;
    const int r = resolve_rows(rows, N);
    if (r == N) return &launch_fwd_coef<F, D, CT, N>;
    if (r == 0) return &launch_fwd_coef<F, D, CT, 0>;
    if constexpr (N % 2 == 0 && (2 * N) % 4 == 0)
        if (r == 2) return &launch_fwd_coef<F, D, CT, 2>;
    return nullptr;
}

template <int F, int D>
FwdLauncher fwd_coef_for(const Variant &v)
{
    if (v.precision != P_FP32) return nullptr;
    return v.coord_f64 ? fwd_coef_rows<F, D, double>(v.rows) : fwd_coef_rows<F, D, float>(v.rows);
}

}  // namespace

FwdLauncher find_forward_coefficient(const Variant &v)
{
    switch (v.form * 4 + v.dim) {
    case WLAP1 * 4 + 2: return fwd_coef_for<WLAP1, 2>(v);
    case WLAP1 * 4 + 3: return fwd_coef_for<WLAP1, 3>(v);
    case WLAP2 * 4 + 2: return fwd_coef_for<WLAP2, 2>(v);
    case WLAP2 * 4 + 3: return fwd_coef_for<WLAP2, 3>(v);
    default: return nullptr;
    }
}

AdjLauncher find_adjoint(const Variant &v)
{
    if (v.dim == 2) {
        switch (v.form) {
        case LAP1: return adj_for_coords<LAP1, 2>(v);
        case ELA1: return adj_for_coords<ELA1, 2>(v);
        case LAP2: return adj_for_coords<LAP2, 2>(v);
        }
    } else if (v.dim == 3) {
        switch (v.form) {
        case LAP1: return adj_for_coords<LAP1, 3>(v);
        case ELA1: return adj_for_coords<ELA1, 3>(v);
        case LAP2: return adj_for_coords<LAP2, 3>(v);
        }
    }
    return nullptr;
}

namespace {

template <int PREC, int VAR>
hipError_t launch_batch_fwd(const BatchLaunch &b, int grid, hipStream_t s)
{
    constexpr int lds = batch_fwd_lds<PREC, VAR>();
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&batch_fwd_kernel<PREC, VAR>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((batch_fwd_kernel<PREC, VAR>), dim3(grid), dim3(kBlock), lds, s, b);
    return hipGetLastError();
}

template <int VAR>
hipError_t launch_batch_adj(const BatchLaunch &b, int grid, hipStream_t s)
{
    constexpr int lds = batch_adj_lds<VAR>();
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&batch_adj_kernel<VAR>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((batch_adj_kernel<VAR>), dim3(grid), dim3(kBlock), lds, s, b);
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_batch_fwd_var(const BatchLaunch &b, int variant, int grid, hipStream_t s)
{
    return variant == 0 ? launch_batch_fwd<PREC, 0>(b, grid, s) : launch_batch_fwd<PREC, 1>(b, grid, s);
}

}  // namespace

size_t batch_lds_bytes(bool adjoint, int precision, int variant)
{
    if (variant != 0 && variant != 1) return 0;
    if (adjoint) return precision == P_FP32 ? (variant ? batch_adj_lds<1>() : batch_adj_lds<0>()) : 0;
    switch (precision) {
    case P_FP32: return variant ? batch_fwd_lds<P_FP32, 1>() : batch_fwd_lds<P_FP32, 0>();
    case P_FP16X2: return variant ? batch_fwd_lds<P_FP16X2, 1>() : batch_fwd_lds<P_FP16X2, 0>();
    case P_BF16X2: return variant ? batch_fwd_lds<P_BF16X2, 1>() : batch_fwd_lds<P_BF16X2, 0>();
    case P_BF16X3: return variant ? batch_fwd_lds<P_BF16X3, 1>() : batch_fwd_lds<P_BF16X3, 0>();
    default: return 0;
    }
}

hipError_t launch_batch(bool adjoint, int precision, int variant, const BatchLaunch &b, int grid,
                        hipStream_t s)
{
    if (adjoint) return variant ? launch_batch_adj<1>(b, grid, s) : launch_batch_adj<0>(b, grid, s);
    switch (precision) {
    case P_FP32: return launch_batch_fwd_var<P_FP32>(b, variant, grid, s);
    case P_FP16X2: return launch_batch_fwd_var<P_FP16X2>(b, variant, grid, s);
    case P_BF16X2: return launch_batch_fwd_var<P_BF16X2>(b, variant, grid, s);
    case P_BF16X3: return launch_batch_fwd_var<P_BF16X3>(b, variant, grid, s);
    default: return hipErrorInvalidValue;
    }
}

namespace {

template <int F, int D, int PREC, int VAR, bool ADJ, bool GATHER = false>
hipError_t launch_group(const BatchLaunch &b, hipStream_t s)
{
    hipLaunchKernelGGL((batch_group_kernel<F, D, PREC, VAR, ADJ, GATHER>), dim3(unsigned(b.n_tiles)),
                       dim3(kBlock), 0, s, b);
    return hipGetLastError();
}

template <int F, int D, int PREC>
hipError_t launch_group_pv(bool adj, bool gather, int variant, const BatchLaunch &b, hipStream_t s)
{
    if (adj) {
        if constexpr (PREC == P_FP32) {
            if (gather)
                return variant ? launch_group<F, D, P_FP32, 1, true, true>(b, s)
                               : launch_group<F, D, P_FP32, 0, true, true>(b, s);
            return variant ? launch_group<F, D, P_FP32, 1, true>(b, s)
                           : launch_group<F, D, P_FP32, 0, true>(b, s);
        } else {
            return hipErrorInvalidValue;
        }
    }
    return variant ? launch_group<F, D, PREC, 1, false>(b, s) : launch_group<F, D, PREC, 0, false>(b, s);
}

template <int F, int D>
hipError_t launch_group_fd(bool adj, bool gather, int precision, int variant, const BatchLaunch &b,
                           hipStream_t s)
{
    switch (precision) {
    case P_FP32: return launch_group_pv<F, D, P_FP32>(adj, gather, variant, b, s);
    case P_FP16X2: return launch_group_pv<F, D, P_FP16X2>(adj, gather, variant, b, s);
    case P_BF16X2: return launch_group_pv<F, D, P_BF16X2>(adj, gather, variant, b, s);
    case P_BF16X3: return launch_group_pv<F, D, P_BF16X3>(adj, gather, variant, b, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_batch_group(bool adjoint, bool gather, int form, int dim, int precision,
                              int variant, const BatchLaunch &b, hipStream_t s)
{
    if (b.n_tiles <= 0) return hipSuccess;
    switch (form * 4 + dim) {
    case LAP1 * 4 + 2: return launch_group_fd<LAP1, 2>(adjoint, gather, precision, variant, b, s);
    case LAP1 * 4 + 3: return launch_group_fd<LAP1, 3>(adjoint, gather, precision, variant, b, s);
    case ELA1 * 4 + 2: return launch_group_fd<ELA1, 2>(adjoint, gather, precision, variant, b, s);
    case ELA1 * 4 + 3: return launch_group_fd<ELA1, 3>(adjoint, gather, precision, variant, b, s);
    case LAP2 * 4 + 2: return launch_group_fd<LAP2, 2>(adjoint, gather, precision, variant, b, s);
    case LAP2 * 4 + 3: return launch_group_fd<LAP2, 3>(adjoint, gather, precision, variant, b, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_reset(int32_t *counter, hipStream_t s)
{
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, s, counter);
    return hipGetLastError();
}

hipError_t launch_incidence_build(const Incidence &g, hipStream_t s)
{
    auto grid = [](int64_t n) { return unsigned(std::min<int64_t>((n + 255) / 256, 8192)); };
    const int64_t total = g.n_elements * g.nv;
    hipLaunchKernelGGL(incidence_zero_kernel, dim3(grid(g.n_vertices + 1)), dim3(256), 0, s, g.ptr,
                       g.n_vertices + 1);
    hipLaunchKernelGGL(incidence_zero_kernel, dim3(grid(g.n_vertices)), dim3(256), 0, s, g.cursor,
                       g.n_vertices);
    // count and fill: one batch of kIncBatch references per workgroup step
    const unsigned gb = unsigned(std::min<int64_t>((total + kIncBatch - 1) / kIncBatch, 4096));
    if (gb > 0) hipLaunchKernelGGL(incidence_count_kernel, dim3(gb), dim3(256), 0, s, g);
    // scan of ptr[0 .. n_vertices]: one workgroup for a single block, else
    // block scans, a scan of their totals (kept in cursor, which is zeroed
    // again before the fill) and the offsets added back
    const int64_t n = g.n_vertices + 1;
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    if (nb <= 1) {
        hipLaunchKernelGGL(incidence_scan_kernel, dim3(1), dim3(1024), 0, s, g.ptr, n);
    } else {
        // nb <= n_vertices here: cursor [n_vertices] holds the block totals
        hipLaunchKernelGGL(incidence_scan_blocks_kernel, dim3(unsigned(nb)), dim3(256), 0, s, g.ptr,
                           n, g.cursor);
        hipLaunchKernelGGL(incidence_scan_kernel, dim3(1), dim3(1024), 0, s, g.cursor, nb);
        hipLaunchKernelGGL(incidence_add_kernel, dim3(unsigned(nb - 1)), dim3(256), 0, s, g.ptr, n,
                           g.cursor);
        hipLaunchKernelGGL(incidence_zero_kernel, dim3(grid(nb)), dim3(256), 0, s, g.cursor, nb);
    }
    if (gb > 0) hipLaunchKernelGGL(incidence_fill_kernel, dim3(gb), dim3(256), 0, s, g);
    const int64_t sw = (g.n_vertices + kSortVerts - 1) / kSortVerts;     // waves of the sort
    if (sw > 0)
        hipLaunchKernelGGL(incidence_sort_kernel, dim3(unsigned(std::min<int64_t>((sw + 3) / 4, 8192))),
                           dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_vertex_gather(const GatherItem *items, int n_items, const int32_t *xoff,
                                int64_t blocks_per_xcd, hipStream_t s)
{
    if (n_items == 0 || blocks_per_xcd == 0) return hipSuccess;
    hipLaunchKernelGGL(vertex_gather_kernel, dim3(unsigned(8 * blocks_per_xcd)), dim3(256), 0, s,
                       items, n_items, xoff);
    return hipGetLastError();
}

hipError_t launch_vertex_gather_one(const GatherItem &it, hipStream_t s)
{
    if (it.n_vertices <= 0) return hipSuccess;
    int64_t most = 0;
    for (int x = 0; x < 8; ++x) {
        const int64_t n = gather_slice_begin(it.n_vertices, x + 1) - gather_slice_begin(it.n_vertices, x);
        most = n > most ? n : most;
    }
    if (most == 0) return hipSuccess;
    hipLaunchKernelGGL(vertex_gather_one_kernel, dim3(unsigned(8 * most)), dim3(256), 0, s, it);
    return hipGetLastError();
}

int assemble_chunk_rows() { return kAsmRows; }
int assemble_chunk_slots() { return kAsmSlots; }
int assemble_lanes() { return kAsmLanes; }

hipError_t launch_assemble(int form, int dim, const AsmParams &p, hipStream_t s)
{
    if (p.n_chunks <= 0) return hipSuccess;
    const unsigned grid = unsigned((p.n_chunks + 3) / 4);
    switch (form * 4 + dim) {
    case LAP1 * 4 + 2: hipLaunchKernelGGL((assemble_kernel<LAP1, 2>), dim3(grid), dim3(256), 0, s, p); break;
    case LAP1 * 4 + 3: hipLaunchKernelGGL((assemble_kernel<LAP1, 3>), dim3(grid), dim3(256), 0, s, p); break;
    case ELA1 * 4 + 2: hipLaunchKernelGGL((assemble_kernel<ELA1, 2>), dim3(grid), dim3(256), 0, s, p); break;
    case ELA1 * 4 + 3: hipLaunchKernelGGL((assemble_kernel<ELA1, 3>), dim3(grid), dim3(256), 0, s, p); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_validate(const MeshView &m, int dim, unsigned long long *n_bad_dev,
                           hipStream_t s)
{
    const int64_t total = m.n_elements * (dim + 1);
    const int64_t want = (total + kBlock - 1) / kBlock;
    const unsigned grid = unsigned(want < 4096 ? (want > 0 ? want : 1) : 4096);
    hipLaunchKernelGGL(validate_kernel, dim3(grid), dim3(kBlock), 0, s, m, dim + 1, n_bad_dev);
    return hipGetLastError();
}

template <int D, int DEG, int NC, bool SYM, bool NOVAL>
hipError_t launch_form_t(const FormParams &p, hipStream_t s)
{
    const int64_t n_groups = (p.m.n_elements + kBlock - 1) / kBlock;
    if (n_groups == 0) return hipSuccess;
    hipLaunchKernelGGL((form_kernel<D, DEG, NC, SYM, NOVAL>), dim3(unsigned(n_groups)), dim3(kBlock),
                       0, s, p);
    return hipGetLastError();
}

template <int D, int DEG, int NC>
hipError_t launch_form_sym(bool sym, bool noval, const FormParams &p, hipStream_t s)
{
    if (noval)
        return sym ? launch_form_t<D, DEG, NC, true, true>(p, s)
                   : launch_form_t<D, DEG, NC, false, true>(p, s);
    return sym ? launch_form_t<D, DEG, NC, true, false>(p, s)
               : launch_form_t<D, DEG, NC, false, false>(p, s);
}

hipError_t launch_form(int dim, int degree, int ncomp, bool sym, bool noval, const FormParams &p,
                       hipStream_t s)
{
    const bool vec = ncomp == dim;
    if (ncomp != 1 && !vec) return hipErrorInvalidValue;
    if (dim == 2) {
        if (degree == 1) return vec ? launch_form_sym<2, 1, 2>(sym, noval, p, s) : launch_form_sym<2, 1, 1>(sym, noval, p, s);
        if (degree == 2) return vec ? launch_form_sym<2, 2, 2>(sym, noval, p, s) : launch_form_sym<2, 2, 1>(sym, noval, p, s);
    } else if (dim == 3) {
        if (degree == 1) return vec ? launch_form_sym<3, 1, 3>(sym, noval, p, s) : launch_form_sym<3, 1, 1>(sym, noval, p, s);
        if (degree == 2) return vec ? launch_form_sym<3, 2, 3>(sym, noval, p, s) : launch_form_sym<3, 2, 1>(sym, noval, p, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_iso(int dim, const FwdParams &p, hipStream_t s)
{
    const int64_t n_groups = (p.m.n_elements + kBlock - 1) / kBlock;
    if (n_groups == 0) return hipSuccess;
    if (dim == 3)
        hipLaunchKernelGGL(iso_kernel<3>, dim3(unsigned(n_groups)), dim3(kBlock), 0, s, p);
    else if (dim == 2)
        hipLaunchKernelGGL(iso_kernel<2>, dim3(unsigned(n_groups)), dim3(kBlock), 0, s, p);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace fei
