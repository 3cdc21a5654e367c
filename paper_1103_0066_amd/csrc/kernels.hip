// All device code of libfei: kernel instantiations and the launcher tables
// the host layer dispatches through.  One translation unit, so the
// __constant__ reference tables exist once per device module.
#include "adjoint.h"
#include "fwd_fma.h"
#include "fwd_mfma.h"

// K tables (block tensor and MFMA fragments), emitted by gen_tables.cpp.
#include "_gen/tables.inc"

namespace fei {

namespace {

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t E) { return unsigned((E + kBlock - 1) / kBlock); }

template <int F, int D, typename CT>
hipError_t launch_fwd_fma(const FwdParams &p, hipStream_t s)
{
    hipLaunchKernelGGL((fwd_fma_kernel<F, D, CT>), dim3(grid_for(p.m.n_elements)), dim3(kBlock),
                       0, s, p);
    return hipGetLastError();
}

template <int F, int D, typename CT, int PREC>
hipError_t launch_fwd_mfma(const FwdParams &p, hipStream_t s)
{
    hipLaunchKernelGGL((fwd_mfma_kernel<F, D, CT, PREC>), dim3(grid_for(p.m.n_elements)),
                       dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

template <int F, int D, typename CT>
hipError_t launch_adj_fma(const AdjParams &p, hipStream_t s)
{
    hipLaunchKernelGGL((adj_fma_kernel<F, D, CT>), dim3(grid_for(p.m.n_elements)), dim3(kBlock),
                       0, s, p);
    return hipGetLastError();
}

template <int F, int D, typename CT>
FwdLauncher fwd_for_prec(int prec)
{
    switch (prec) {
    case P_FP32: return &launch_fwd_fma<F, D, CT>;
    case P_FP16X2: return &launch_fwd_mfma<F, D, CT, P_FP16X2>;
    case P_BF16X2: return &launch_fwd_mfma<F, D, CT, P_BF16X2>;
    case P_BF16X3: return &launch_fwd_mfma<F, D, CT, P_BF16X3>;
    default: return nullptr;
    }
}

template <int F, int D>
FwdLauncher fwd_for_coords(const Variant &v)
{
    return v.coord_f64 ? fwd_for_prec<F, D, double>(v.precision)
                       : fwd_for_prec<F, D, float>(v.precision);
}

template <int F, int D>
AdjLauncher adj_for_coords(const Variant &v)
{
    if (v.precision != P_FP32) return nullptr;
    return v.coord_f64 ? &launch_adj_fma<F, D, double> : &launch_adj_fma<F, D, float>;
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

hipError_t launch_validate(const MeshView &m, int dim, unsigned long long *n_bad_dev,
                           hipStream_t s)
{
    const int64_t total = m.n_elements * (dim + 1);
    const int64_t want = (total + kBlock - 1) / kBlock;
    const unsigned grid = unsigned(want < 4096 ? (want > 0 ? want : 1) : 4096);
    hipLaunchKernelGGL(validate_kernel, dim3(grid), dim3(kBlock), 0, s, m, dim + 1, n_bad_dev);
    return hipGetLastError();
}

}  // namespace fei
