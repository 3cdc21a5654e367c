// Forward integration of the Laplacian with a P1 coefficient w (Sec. 3.1,
// eqs. 20-23), FP32 fused multiply-adds:
//
//   A_ij = sum_k w_k G^{mu nu} K^{ijk}_{mu nu},
//
// G the Laplacian's geometric tensor (eq. 8), w_k the coefficient's values at
// the element's vertices, and K^{ijk}_{mu nu} = int_ref dphi_i/dxi_mu phi_k
// dphi_j/dxi_nu the arity-3 reference tensor, computed a priori in exact
// integers (the coefficient's index k folds into the geometric tensor as
// G_k = w_k G, eq. 23).  One lane per element; K is compiled into the
// instruction stream as in the constant-coefficient forward (zero terms
// skipped at compile time), and loads, output staging and stores are that
// forward's (FwdFmaTile).
#pragma once

#include "fwd_fma.h"

namespace fei {

template <int FORM, int DIM>
struct KWFold;

template <int FORM, int DIM>
__device__ __forceinline__ float kwval(int i, int j, int m, int mu, int nu)
{
    using T = Traits<FORM, DIM>;
    return KWFold<FORM, DIM>::t.v[(((i * T::NB + j) * (DIM + 1) + m) * DIM + mu) * DIM + nu];
}

template <int FORM, int DIM, typename CT, int R>
struct FwdCoefTile : FwdFmaTile<FORM, DIM, CT, R> {
    using Base = FwdFmaTile<FORM, DIM, CT, R>;
    using T = Traits<FORM, DIM>;
    using U = Unique<FORM, DIM>;
    static_assert(has_coefficient(FORM), "forms with a P1 coefficient");

    struct Xw {
        CT x[DIM + 1][DIM];
        float w[DIM + 1];
    };

    __device__ static Xw gather_w(const FwdParams &p, const typename Base::In &in)
    {
        Xw g;
        gather<DIM>(p.m, in.v, g.x);
#pragma unroll
        for (int a = 0; a <= DIM; ++a) g.w[a] = p.w[in.v[a]];
        return g;
    }

    __device__ static void compute(const FwdParams &p, int64_t e0, const Xw &g, float (&Au)[U::NU])
    {
        float Gf[T::G];
        bool flag = false, singular = false;
        if (e0 + (threadIdx.x & 63) < p.m.n_elements) {
            flag = geometry<FORM, DIM>(g.x, 0.f, 0.f, p.tau2, Gf, singular);
        } else {
#pragma unroll
            for (int k = 0; k < T::G; ++k) Gf[k] = 0.f;
        }
        count_flags(p.counters, flag, singular);
        // G_k = w_k G (eq. 23), then A_ij = sum_{k, mu, nu} K^{ijk}_{mu nu} G_k^{mu nu}
        float Gk[DIM + 1][T::G];
#pragma unroll
        for (int m = 0; m <= DIM; ++m)
#pragma unroll
            for (int q = 0; q < T::G; ++q) Gk[m][q] = g.w[m] * Gf[q];
#pragma unroll
        for (int I = 0; I < T::N; ++I)
#pragma unroll
            for (int J = I; J < T::N; ++J) {
                float acc = 0.f;
#pragma unroll
                for (int m = 0; m <= DIM; ++m)
#pragma unroll
                    for (int mu = 0; mu < DIM; ++mu)
#pragma unroll
                        for (int nu = 0; nu < DIM; ++nu) {
                            const float k = kwval<FORM, DIM>(I, J, m, mu, nu);
                            if (k != 0.f) acc = fmaf(k, Gk[m][sym_index(DIM, mu, nu)], acc);
                        }
                Au[sym_index(T::N, I, J)] = acc;
            }
    }

    __device__ __forceinline__ static void run(const FwdParams &p, int64_t blk, unsigned char *smem)
    {
        const int64_t e0 = blk * 256 + wave_id() * 64;
        const Xw g = gather_w(p, Base::load(p, e0));
        float Au[U::NU];
        compute(p, e0, g, Au);
        Base::store(p, e0, Au, smem);
    }
};

template <int FORM, int DIM, typename CT, int R>
__global__ __launch_bounds__(256) void fwd_coef_kernel(FwdParams p)
{
    using Tile = FwdCoefTile<FORM, DIM, CT, R>;
    __shared__ __attribute__((aligned(16))) unsigned char smem[Tile::LDS_BYTES > 0 ? Tile::LDS_BYTES : 16];
    Tile::run(p, xcd_block(blockIdx.x, gridDim.x), smem);
}

}  // namespace fei
