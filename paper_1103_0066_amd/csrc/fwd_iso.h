// Isoparametric P2 Laplacian on elements with quadratic geometry (Sec. 3.1,
// eqs. 16-19), FP32 forward.
//
// The geometry map x(xi) = sum_n x_n psi_n(xi) uses the element's NB nodes
// (vertices, then edge nodes; psi the P2 basis, which is also the solution
// basis).  Following the paper, the inverse Jacobian is projected into a
// finite element space -- here the vertex functions lambda_k, by its values
// B_k = J(xi_k)^-1 at the vertices -- and |J| is taken out of the integral as
// one constant, |det J| at the barycenter (eq. 17).  Then
//
//   A_ij = G^{(k mu),(l nu)} K^{ijkl}_{mu nu},                       (eq. 19)
//   G^{(k mu),(l nu)} = sum_alpha B_k[mu][alpha] B_l[nu][alpha] |J_c|  (eq. 18)
//
// with the arity-4 reference tensor K integrated exactly at build time
// (KIsoFold: folded over the symmetric pairs of G, integers times a scale).
// One lane per element; the 55 (2D: 21) unique entries of the symmetric
// matrix are 78 x 55 (21 x 21) dot products with K compiled into the code
// (zero entries skipped); the matrices leave through the same whole-matrix
// LDS staging as the P2 Laplacian forward.  Elements whose Jacobian at a
// vertex or at the barycenter fails the quality test build G in FP64.
#pragma once

#include <utility>

#include "fwd_fma.h"

namespace fei {

template <int DIM>
struct KIsoFold;

// d psi_n / d xi_mu of the P2 basis at vertex k (point < NV) or at the
// barycenter (point == NV); compile-time after unrolling.
template <int DIM>
__host__ __device__ constexpr float iso_dpsi(int n, int mu, int point)
{
    constexpr int NV = DIM + 1;
    auto bc = [&](int a) -> float { return point < NV ? (a == point ? 1.f : 0.f) : 1.f / NV; };
    auto gl = [&](int a) -> float { return a == 0 ? -1.f : (a - 1 == mu ? 1.f : 0.f); };
    if (n < NV) return (4.f * bc(n) - 1.f) * gl(n);
    int e = NV;
    for (int a = 0; a < NV; ++a)
        for (int b = a + 1; b < NV; ++b, ++e)
            if (e == n) return 4.f * (bc(a) * gl(b) + bc(b) * gl(a));
    return 0.f;
}

// J at a point, adjugate and determinant, in precision R, from the node
// offsets d_n = x_n - x_0 (d_0 = 0): the coefficients of every derivative sum
// to zero, so J = sum_n c_n d_n, and the offsets of nearby FP32 coordinates
// are exact (Sterbenz), while a sum of c_n x_n over absolute coordinates
// would lose |x| / h of the accuracy.
template <int DIM, typename R>
__device__ __forceinline__ R iso_adj(const float (&dn)[IsoShape<DIM>::NB][DIM], int point,
                                     R (&J)[DIM][DIM], R (&adj)[DIM][DIM])
{
#pragma unroll
    for (int al = 0; al < DIM; ++al)
#pragma unroll
        for (int mu = 0; mu < DIM; ++mu) {
            R s = R(0);
#pragma unroll
            for (int n = 1; n < IsoShape<DIM>::NB; ++n) {
                const float c = iso_dpsi<DIM>(n, mu, point);
                if (c != 0.f) s += R(c) * R(dn[n][al]);
            }
            J[al][mu] = s;
        }
    return adjugate(J, adj);
}

// Unique pairs of G from the vertex inverses (computed in R) and |J_c|.
template <int DIM, typename R>
__device__ __forceinline__ void iso_g(const float (&xn)[IsoShape<DIM>::NB][DIM], R scale,
                                      float (&G)[IsoShape<DIM>::G], bool &singular)
{
    using S = IsoShape<DIM>;
    R B[S::NV][DIM][DIM];
#pragma unroll
    for (int k = 0; k < S::NV; ++k) {
        R J[DIM][DIM], adj[DIM][DIM];
        const R det = iso_adj<DIM, R>(xn, k, J, adj);
        singular = singular || det == R(0);
        const R inv = R(1) / det;
#pragma unroll
        for (int mu = 0; mu < DIM; ++mu)
#pragma unroll
            for (int al = 0; al < DIM; ++al) B[k][mu][al] = adj[mu][al] * inv;
    }
    R Jc[DIM][DIM], adjc[DIM][DIM];
    const R detc = iso_adj<DIM, R>(xn, S::NV, Jc, adjc);
    singular = singular || detc == R(0);
    const R s = (detc < R(0) ? -detc : detc) * scale;
#pragma unroll
    for (int p = 0; p < S::GD; ++p)
#pragma unroll
        for (int q = p; q < S::GD; ++q) {
            const int k = p / DIM, mu = p % DIM, l = q / DIM, nu = q % DIM;
            R acc = R(0);
#pragma unroll
            for (int al = 0; al < DIM; ++al) acc += B[k][mu][al] * B[l][nu][al];
            G[sym_index(S::GD, p, q)] = float(s * acc);
        }
}

// Unique entry U of A: a dot product of the 78 (2D: 21) pairs of G with row
// U of the folded K, zero terms dropped at compile time.  One instantiation
// per entry (an index sequence), so every index is a constant and the loop
// over the pairs unrolls.
template <int DIM, int U>
__device__ __forceinline__ float iso_entry(const float (&G)[IsoShape<DIM>::G])
{
    float acc = 0.f;
#pragma unroll
    for (int g = 0; g < IsoShape<DIM>::G; ++g) {
        const float k = KIsoFold<DIM>::t.v[U * IsoShape<DIM>::G + g];
        if (k != 0.f) acc = fmaf(k, G[g], acc);
    }
    return acc;
}

template <int DIM, int... U>
__device__ __forceinline__ void iso_entries(const float (&G)[IsoShape<DIM>::G],
                                            float (&Au)[IsoShape<DIM>::NU],
                                            std::integer_sequence<int, U...>)
{
    ((Au[U] = iso_entry<DIM, U>(G)), ...);
}

template <int DIM>
__global__ __launch_bounds__(256) void iso_kernel(FwdParams p)
{
    using S = IsoShape<DIM>;
    using Store = FwdFmaTile<LAP2, DIM, float, Traits<LAP2, DIM>::N>;
    static_assert(Traits<LAP2, DIM>::N == S::NB && Unique<LAP2, DIM>::NU == S::NU, "shapes");
    __shared__ __attribute__((aligned(16))) unsigned char smem[Store::LDS_BYTES];

    const int64_t e0 = xcd_block(blockIdx.x, gridDim.x) * 256 + wave_id() * 64;
    const int64_t E = p.m.n_elements;
    const int64_t e = e0 + (threadIdx.x & 63);
    const bool live = e < E;
    const int64_t ec = live ? e : E - 1;

    float xn[S::NB][DIM];
    {
        const int32_t *__restrict__ c = p.m.conn + ec * S::NB;
        const float *__restrict__ X = static_cast<const float *>(p.m.x);
        const float *__restrict__ Y = static_cast<const float *>(p.m.y);
        const float *__restrict__ Z = static_cast<const float *>(p.m.z);
        int v[S::NB];
#pragma unroll
        for (int n = 0; n < S::NB; ++n) v[n] = __builtin_nontemporal_load(c + n);
#pragma unroll
        for (int n = 0; n < S::NB; ++n) {
            xn[n][0] = X[v[n]];
            xn[n][1] = Y[v[n]];
            if constexpr (DIM == 3) xn[n][2] = Z[v[n]];
        }
        // offsets from node 0 (xn[0] becomes 0)
#pragma unroll
        for (int n = S::NB - 1; n >= 0; --n)
#pragma unroll
            for (int al = 0; al < DIM; ++al) xn[n][al] -= xn[0][al];
    }
    // quality test on the Jacobians at the vertices and the barycenter
    bool flag = false, singular = false;
    if (live) {
#pragma unroll
        for (int pt = 0; pt <= S::NV; ++pt) {
            float J[DIM][DIM], adj[DIM][DIM];
            const float det = iso_adj<DIM, float>(xn, pt, J, adj);
            flag = flag || needs_fp64<DIM>(J, adj, det, p.tau2);
        }
    }
    float G[S::G];
    constexpr double KS = KIsoFold<DIM>::t.scale;
    if (!flag) {
        iso_g<DIM, float>(xn, float(KS), G, singular);
    } else {
        iso_g<DIM, double>(xn, KS, G, singular);
    }
    if (!live) singular = false;
    count_flags(p.counters, flag, singular);

    float Au[S::NU];
    iso_entries<DIM>(G, Au, std::make_integer_sequence<int, S::NU>{});
    Store::store(p, e0, Au, smem);
}

}  // namespace fei
