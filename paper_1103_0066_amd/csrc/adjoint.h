// Adjoint of the element integration for L = sum_e <dA_e, A_e>.
//
// The forward chain is A = Gf : K (eq. 1), Gf from (B = J^-1, s = |det J|,
// mu, lambda) (eq. 8 and its Lame analogue), J from the vertex coordinates.
// Reverse, per element, one lane per element, recomputing the geometry:
//
//   U_g   = sum_IJ dA_IJ Kf[g][IJ]             (the folded K^T applied to dA)
//   S     = symmetric tensor with S_pp = U_pp, S_pq = S_qp = U_pq / 2
//   Laplacian forms, Gf = c s B B^T:
//     sbar = c <S, BB^T>,  Bbar = 2 c s S B
//   Elasticity, Gf = c s [mu P1(B) + lambda P2(B)]:
//     H_mn = sum_c S_(mc),(nc);  Z_kg = sum_cn S_(kc),(ng) B_nc;
//     Y_kg = sum_nd S_(kg),(nd) B_nd;
//     F1 = <H, BB^T> + sum_md B_md Z_md;  F2 = sum_mc B_mc Y_mc
//     mubar = c s F1,  lambar = c s F2,  sbar = c (mu F1 + lambda F2)
//     Bbar = c s (2 mu (H B + Z) + 2 lambda Y)
//   Jbar = sbar s B^T - B^T Bbar B^T        (d|det J| = s J^-T : dJ, dB = -B dJ B)
//   xbar_{m+1} += Jbar[:, m],  xbar_0 -= sum_m Jbar[:, m]   (FP32 atomics)
//
// Flagged elements (quality test) and FP64 coordinates run the geometry
// reverse in FP64.
#pragma once

#include "fwd_fma.h"

namespace fei {

template <int FORM, int DIM, typename R>
__device__ __forceinline__ void adjoint_chain(const R (&adj)[DIM][DIM], R det, float mu_f,
                                              float lam_f, const float (&U)[Traits<FORM, DIM>::G],
                                              float (&Jbar)[DIM][DIM], float &mubar,
                                              float &lambar)
{
    using T = Traits<FORM, DIM>;
    const R s = det < R(0) ? -det : det;
    const R c = R(T::SCALE);
    const R inv = R(1) / det;
    R B[DIM][DIM];
#pragma unroll
    for (int m = 0; m < DIM; ++m)
#pragma unroll
        for (int a = 0; a < DIM; ++a) B[m][a] = adj[m][a] * inv;
    R M[DIM][DIM];
#pragma unroll
    for (int m = 0; m < DIM; ++m)
#pragma unroll
        for (int n = 0; n < DIM; ++n) {
            R acc = R(0);
#pragma unroll
            for (int a = 0; a < DIM; ++a) acc += B[m][a] * B[n][a];
            M[m][n] = acc;
        }
    auto Sv = [&](int p, int q) -> R {
        const R u = R(U[sym_index(T::GD, p, q)]);
        return p == q ? u : R(0.5) * u;
    };
    R sbar;
    R Bbar[DIM][DIM];
    if constexpr (FORM != ELA1) {
        R F = R(0);
#pragma unroll
        for (int m = 0; m < DIM; ++m)
#pragma unroll
            for (int n = 0; n < DIM; ++n) F += Sv(m, n) * M[m][n];
        sbar = c * F;
#pragma unroll
        for (int k = 0; k < DIM; ++k)
#pragma unroll
            for (int g = 0; g < DIM; ++g) {
                R acc = R(0);
#pragma unroll
                for (int n = 0; n < DIM; ++n) acc += Sv(k, n) * B[n][g];
                Bbar[k][g] = R(2) * c * s * acc;
            }
        mubar = 0.f;
        lambar = 0.f;
    } else {
        const R mu = R(mu_f), lam = R(lam_f);
        R H[DIM][DIM], Z[DIM][DIM], Y[DIM][DIM];
#pragma unroll
        for (int m = 0; m < DIM; ++m)
#pragma unroll
            for (int n = 0; n < DIM; ++n) {
                R h = R(0);
#pragma unroll
                for (int cc = 0; cc < DIM; ++cc) h += Sv(m * DIM + cc, n * DIM + cc);
                H[m][n] = h;
            }
#pragma unroll
        for (int k = 0; k < DIM; ++k)
#pragma unroll
            for (int g = 0; g < DIM; ++g) {
                R z = R(0), y = R(0);
#pragma unroll
                for (int cc = 0; cc < DIM; ++cc)
#pragma unroll
                    for (int n = 0; n < DIM; ++n) {
                        z += Sv(k * DIM + cc, n * DIM + g) * B[n][cc];
                        y += Sv(k * DIM + g, n * DIM + cc) * B[n][cc];
                    }
                Z[k][g] = z;
                Y[k][g] = y;
            }
        R F1 = R(0), F2 = R(0);
#pragma unroll
        for (int m = 0; m < DIM; ++m)
#pragma unroll
            for (int n = 0; n < DIM; ++n) {
                F1 += H[m][n] * M[m][n] + B[m][n] * Z[m][n];
                F2 += B[m][n] * Y[m][n];
            }
        mubar = float(c * s * F1);
        lambar = float(c * s * F2);
        sbar = c * (mu * F1 + lam * F2);
#pragma unroll
        for (int k = 0; k < DIM; ++k)
#pragma unroll
            for (int g = 0; g < DIM; ++g) {
                R hb = R(0);
#pragma unroll
                for (int n = 0; n < DIM; ++n) hb += H[k][n] * B[n][g];
                Bbar[k][g] = c * s * (R(2) * mu * (hb + Z[k][g]) + R(2) * lam * Y[k][g]);
            }
    }
    // Jbar[a][m] = sbar s B[m][a] - sum_kl B[k][a] Bbar[k][l] B[m][l]
    R W[DIM][DIM];  // W = Bbar B^T : W[k][m] = sum_l Bbar[k][l] B[m][l]
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
            R acc = R(0);
#pragma unroll
            for (int l = 0; l < DIM; ++l) acc += Bbar[k][l] * B[m][l];
            W[k][m] = acc;
        }
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
            R acc = sbar * s * B[m][a];
#pragma unroll
            for (int k = 0; k < DIM; ++k) acc -= B[k][a] * W[k][m];
            Jbar[a][m] = float(acc);
        }
}

template <int FORM, int DIM, typename CT>
__global__ __launch_bounds__(256) void adj_fma_kernel(AdjParams p)
{
    using T = Traits<FORM, DIM>;
    constexpr int N = T::N;
    constexpr int VEC = (N % 4 == 0) ? 4 : (N % 2 == 0) ? 2 : 1;
    using V = typename VecT<VEC>::type;
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

    // U = Kf applied to dA (streamed row by row)
    float U[T::G];
#pragma unroll
    for (int g = 0; g < T::G; ++g) U[g] = 0.f;
    const float *__restrict__ dAe = p.dA + e * (int64_t)(N * N);
#pragma unroll
    for (int I = 0; I < N; ++I) {
#pragma unroll
        for (int J0 = 0; J0 < N; J0 += VEC) {
            const V w = __builtin_nontemporal_load(reinterpret_cast<const V *>(dAe + I * N + J0));
            float r[VEC];
            __builtin_memcpy(r, &w, sizeof(V));
#pragma unroll
            for (int k = 0; k < VEC; ++k) {
                const int J = J0 + k;
                const int a = I / T::NC, cI = I % T::NC, b = J / T::NC, dJ = J % T::NC;
#pragma unroll
                for (int mu_ = 0; mu_ < DIM; ++mu_)
#pragma unroll
                    for (int nu = 0; nu < DIM; ++nu) {
                        const int g = sym_index(T::GD, mu_ * T::NC + cI, nu * T::NC + dJ);
                        U[g] = fmaf(kval<FORM, DIM>(a, b, mu_, nu), r[k], U[g]);
                    }
            }
        }
    }

    float Jbar[DIM][DIM], mubar, lambar;
    bool flag = false, singular = false;
    if constexpr (sizeof(CT) == 8) {
        double J[DIM][DIM], adj[DIM][DIM];
        jacobian<DIM>(xv, J);
        const double det = adjugate(J, adj);
        singular = (det == 0.0);
        adjoint_chain<FORM, DIM>(adj, det, mu, lam, U, Jbar, mubar, lambar);
    } else {
        float J[DIM][DIM], adj[DIM][DIM];
        jacobian<DIM>(xv, J);
        const float det = adjugate(J, adj);
        flag = needs_fp64<DIM>(J, adj, det, p.tau2);
        if (!flag) {
            adjoint_chain<FORM, DIM>(adj, det, mu, lam, U, Jbar, mubar, lambar);
        } else {
            double Jd[DIM][DIM], adjd[DIM][DIM];
            jacobian<DIM>(xv, Jd);
            const double detd = adjugate(Jd, adjd);
            singular = (detd == 0.0);
            adjoint_chain<FORM, DIM>(adjd, detd, mu, lam, U, Jbar, mubar, lambar);
        }
    }
    count_flags(p.counters, flag, singular);

    float *X[3] = {p.dx, p.dy, p.dz};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        float s0 = 0.f;
#pragma unroll
        for (int m = 0; m < DIM; ++m) {
            unsafeAtomicAdd(X[a] + v[m + 1], Jbar[a][m]);
            s0 += Jbar[a][m];
        }
        unsafeAtomicAdd(X[a] + v[0], -s0);
    }
    if constexpr (FORM == ELA1) {
        if (p.dmu) p.dmu[e] = mubar;
        if (p.dlam) p.dlam[e] = lambar;
    }
}

}  // namespace fei
