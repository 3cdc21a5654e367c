// Forward element integration, FP32 fused multiply-add form.
//
// One lane per element (a wave integrates 64 elements).  The lane gathers its
// vertices, forms J, adj J, det J and the folded geometric tensor Gf in
// registers (Sec. 3, eq. 8), then produces the element matrix row by row:
//
//   A_{(a,c),(b,d)} = sum_{mu,nu} K^{ab}_{mu nu} G^{(mu c),(nu d)}     (eq. 6; eq. 14 block form)
//
// which is the paper's per-entry contraction of a d x d block of G with a
// d x d block of K (Sec. 4.3), here executed sequentially by the lane for all
// n^2 entries of its element.  K is the same for every lane of the grid, so
// it lives in a __constant__ table and reaches the lanes through the scalar
// data cache as SGPR operands of v_fma_f32 -- the wave-uniform broadcast is
// what the scalar unit exists for, and it leaves LDS free.  Each finished row
// is stored at once with the widest aligned vector store, so only one row of
// A is live in registers (the paper's interleaved stores, Sec. 4.3).
#pragma once

#include "geometry.h"
#include "shapes.h"

namespace fei {

// Block reference tensors, one per (form, dim), in mutable __constant__
// memory, so the kernels read K at run time rather than folding it into code.
// The specializations holding the values are generated at build time.
template <int FORM, int DIM>
__constant__ KBlockTable<FORM, DIM> c_kblock;

template <int FORM, int DIM>
__device__ __forceinline__ float kval(int i, int j, int mu, int nu)
{
    using T = Traits<FORM, DIM>;
    return c_kblock<FORM, DIM>.v[((i * T::NB + j) * DIM + mu) * DIM + nu];
}

// One entry of A from the folded geometric tensor (all indices compile-time
// after unrolling).
template <int FORM, int DIM>
__device__ __forceinline__ float contract_entry(const float (&Gf)[Traits<FORM, DIM>::G], int I,
                                                int J)
{
    using T = Traits<FORM, DIM>;
    const int a = I / T::NC, c = I % T::NC, b = J / T::NC, d = J % T::NC;
    float acc = 0.f;
#pragma unroll
    for (int mu = 0; mu < DIM; ++mu)
#pragma unroll
        for (int nu = 0; nu < DIM; ++nu)
            acc = fmaf(kval<FORM, DIM>(a, b, mu, nu),
                       Gf[sym_index(T::GD, mu * T::NC + c, nu * T::NC + d)], acc);
    return acc;
}

template <int VEC>
struct VecT;
template <> struct VecT<4> { using type = f32x4_t; };
template <> struct VecT<2> { using type = f32x2_t; };
template <> struct VecT<1> { using type = float; };

template <int FORM, int DIM>
__device__ __forceinline__ void contract_store(const float (&Gf)[Traits<FORM, DIM>::G],
                                               float *__restrict__ Ae)
{
    using T = Traits<FORM, DIM>;
    constexpr int N = T::N;
    constexpr int VEC = (N % 4 == 0) ? 4 : (N % 2 == 0) ? 2 : 1;
    using V = typename VecT<VEC>::type;
#pragma unroll
    for (int I = 0; I < N; ++I) {
#pragma unroll
        for (int J0 = 0; J0 < N; J0 += VEC) {
            float r[VEC];
#pragma unroll
            for (int k = 0; k < VEC; ++k) r[k] = contract_entry<FORM, DIM>(Gf, I, J0 + k);
            V out;
            __builtin_memcpy(&out, r, sizeof(V));
            *reinterpret_cast<V *>(Ae + I * N + J0) = out;
        }
    }
}

template <int FORM, int DIM, typename CT>
__global__ __launch_bounds__(256) void fwd_fma_kernel(FwdParams p)
{
    using T = Traits<FORM, DIM>;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t e = blk * 256 + threadIdx.x;
    if (e >= p.m.n_elements) return;
    int v[DIM + 1];
    load_conn<DIM>(p.m.conn, e, v);
    CT xv[DIM + 1][DIM];
    gather<DIM>(p.m, v, xv);
    float mu = 0.f, lam = 0.f;
    if constexpr (FORM == ELA1) {
        mu = __builtin_nontemporal_load(p.mu + e);
        lam = __builtin_nontemporal_load(p.lam + e);
    }
    float Gf[T::G];
    bool singular;
    const bool flag = geometry<FORM, DIM>(xv, mu, lam, p.tau2, Gf, singular);
    count_flags(p.counters, flag, singular);
    contract_store<FORM, DIM>(Gf, p.A + e * (int64_t)(T::N * T::N));
}

}  // namespace fei
