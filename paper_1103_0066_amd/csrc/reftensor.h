// Reference ("analytic") tensors K of the supported forms, built at compile
// time in exact integer arithmetic.
//
// Sec. 3, eq. 7: K^{ij}_{mu nu} = int_ref dphi_i/dxi_mu dphi_j/dxi_nu dxi.
// Sec. 3.1 (last paragraph): K is an integral of products of basis functions
// and their derivatives, so it can be computed a priori.  Here every entry is
// an integer multiple of vol_ref / KDEN, and the kernels use the integer
// tensor Kp = K * KDEN / vol_ref with the factor vol_ref / KDEN folded into
// the geometric tensor.  Integer entries with |Kp| <= 64 are exact in FP16 and
// BF16, which is what lets the split-precision MFMA path keep K unsplit.
//
// Reference simplex: vertex 0 at the origin, vertex m+1 at e_m, so the
// barycentric gradients are g_0 = (-1,...,-1) and g_{m+1} = e_m.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define FEI_HD __host__ __device__
#else
#define FEI_HD
#endif

namespace fei {

// WLAP1, WLAP2: the Laplacian with a P1 coefficient w (Sec. 3.1, eqs. 20-23),
// whose reference tensor K^{ijk}_{mu nu} has a third index k over the
// coefficient's nodal values.
enum Form { LAP1 = 1, ELA1 = 2, LAP2 = 3, WLAP1 = 4, WLAP2 = 5 };

FEI_HD constexpr bool is_p2(int form) { return form == LAP2 || form == WLAP2; }
FEI_HD constexpr bool has_coefficient(int form) { return form == WLAP1 || form == WLAP2; }

template <int FORM, int DIM>
struct Traits {
    static constexpr int NV = DIM + 1;                                   // vertices
    static constexpr int NB = is_p2(FORM) ? (DIM + 1) * (DIM + 2) / 2 : DIM + 1;  // scalar basis
    static constexpr int NC = (FORM == ELA1) ? DIM : 1;                  // components
    static constexpr int N = NB * NC;                                    // element matrix side
    static constexpr int GD = NC * DIM;                                  // geometric tensor side
    static constexpr int G = GD * (GD + 1) / 2;                          // its unique entries
    // K = Kp * vol_ref / KDEN with integer Kp: the degree of the integrand's
    // barycentric polynomial sets KDEN (int lambda^alpha / vol_ref has
    // denominator (d+1)...(d+|alpha|))
    static constexpr int KDEN = (FORM == LAP2)    ? (DIM + 1) * (DIM + 2)
                                : (FORM == WLAP1) ? (DIM + 1)
                                : (FORM == WLAP2) ? (DIM + 1) * (DIM + 2) * (DIM + 3)
                                                  : 1;
    static constexpr int FACT = (DIM == 2) ? 2 : 6;                      // d! = 1 / vol_ref
    // Gf = SCALE * |det J| * (J^-1 J^-T, or its Lame analogue)
    static constexpr double SCALE = 1.0 / (double(FACT) * double(KDEN));
};

// barycentric gradient g_a[mu] of the reference simplex
FEI_HD constexpr int gref(int a, int mu) { return a == 0 ? -1 : (a - 1 == mu ? 1 : 0); }

// P2 basis: dphi_i/dxi = sum_a c_ia(lambda) g_a, with c_ia linear in lambda:
//   vertex i = v:      c_iv = 4 lambda_v - 1
//   edge i = (p, q):   c_ip = 4 lambda_q,  c_iq = 4 lambda_p
// lin() returns the constant term (k = -1) or the coefficient of lambda_k.
FEI_HD constexpr void p2_edge(int dim, int e, int &p, int &q)
{
    int idx = 0;
    for (int a = 0; a <= dim; ++a)
        for (int b = a + 1; b <= dim; ++b) {
            if (idx == e) { p = a; q = b; return; }
            ++idx;
        }
    p = q = 0;
}

FEI_HD constexpr int p2_lin(int dim, int i, int a, int k)
{
    if (i <= dim) {                              // vertex function
        if (a != i) return 0;
        return k < 0 ? -1 : (k == i ? 4 : 0);
    }
    int p = 0, q = 0;
    p2_edge(dim, i - dim - 1, p, q);
    if (a == p) return (k == q) ? 4 : 0;
    if (a == q) return (k == p) ? 4 : 0;
    return 0;
}

// KDEN/vol * int_ref c_ia c_jb, using int lambda_k/vol = 1/(d+1) and
// int lambda_k lambda_l/vol = (1 + delta_kl)/((d+1)(d+2)).
FEI_HD constexpr int p2_mass(int dim, int i, int a, int j, int b)
{
    int c0 = p2_lin(dim, i, a, -1), d0 = p2_lin(dim, j, b, -1);
    int s = c0 * d0 * (dim + 1) * (dim + 2);
    for (int k = 0; k <= dim; ++k) {
        s += (c0 * p2_lin(dim, j, b, k) + d0 * p2_lin(dim, i, a, k)) * (dim + 2);
        for (int l = 0; l <= dim; ++l)
            s += p2_lin(dim, i, a, k) * p2_lin(dim, j, b, l) * (1 + (k == l));
    }
    return s;
}

// KDEN/vol * int_ref c_ia c_jb lambda_m with KDEN = (d+1)(d+2)(d+3), using
// int lambda^alpha / vol = alpha! d! / (|alpha| + d)!:
//   lambda_m -> (d+2)(d+3),  lambda_k lambda_m -> (1 + delta_km)(d+3),
//   lambda_k lambda_l lambda_m -> alpha! (6, 2 or 1 by the multiplicities).
FEI_HD constexpr int p2_mass_w(int dim, int i, int a, int j, int b, int m)
{
    const int c0 = p2_lin(dim, i, a, -1), d0 = p2_lin(dim, j, b, -1);
    int s = c0 * d0 * (dim + 2) * (dim + 3);
    for (int k = 0; k <= dim; ++k)
        s += (c0 * p2_lin(dim, j, b, k) + d0 * p2_lin(dim, i, a, k)) * (1 + (k == m)) * (dim + 3);
    for (int k = 0; k <= dim; ++k)
        for (int l = 0; l <= dim; ++l) {
            const int f = (k == l && l == m) ? 6 : ((k == l || l == m || k == m) ? 2 : 1);
            s += p2_lin(dim, i, a, k) * p2_lin(dim, j, b, l) * f;
        }
    return s;
}

// Integer coefficient tensor Kp^{ijm}_{mu nu} = KDEN/vol int_ref dphi_i/dxi_mu
// lambda_m dphi_j/dxi_nu of the forms with a P1 coefficient (eq. 23's K^{ijk}).
// P1: the gradients are constant and int lambda_m / vol = 1/(d+1) = 1/KDEN.
FEI_HD constexpr int kwblock(int form, int dim, int i, int j, int m, int mu, int nu)
{
    if (form == WLAP1) return gref(i, mu) * gref(j, nu);
    int s = 0;
    for (int a = 0; a <= dim; ++a)
        for (int b = 0; b <= dim; ++b)
            s += gref(a, mu) * gref(b, nu) * p2_mass_w(dim, i, a, j, b, m);
    return s;
}

// Integer block tensor Kp^{ij}_{mu nu} over the scalar basis.
FEI_HD constexpr int kblock(int form, int dim, int i, int j, int mu, int nu)
{
    if (form != LAP2) return gref(i, mu) * gref(j, nu);
    int s = 0;
    for (int a = 0; a <= dim; ++a)
        for (int b = 0; b <= dim; ++b)
            s += gref(a, mu) * gref(b, nu) * p2_mass(dim, i, a, j, b);
    return s;
}

// Index of the unique pair (p <= q) of a symmetric GD x GD tensor.
FEI_HD constexpr int sym_index(int gd, int p, int q)
{
    if (p > q) { int t = p; p = q; q = t; }
    return p * gd - p * (p - 1) / 2 + (q - p);
}

// Full (unfolded) tensor Kfull(p, q, I, J) with A_IJ = sum_pq Kfull * Gfull_pq.
// Laplacian forms: p = mu, q = nu.  Elasticity: p = mu*DIM + c, q = nu*DIM + d,
// I = DIM*a + c', J = DIM*b + d', Kfull = Kp^{ab}_{mu nu} delta_cc' delta_dd'.
FEI_HD constexpr int kfull(int form, int dim, int p, int q, int I, int J)
{
    if (form != ELA1) return kblock(form, dim, I, J, p, q);
    int mu = p / dim, c = p % dim, nu = q / dim, d = q % dim;
    int a = I / dim, cI = I % dim, b = J / dim, dJ = J % dim;
    if (c != cI || d != dJ) return 0;
    return kblock(form, dim, a, b, mu, nu);
}

// Folded tensor over unique pairs gamma = (p <= q):
// Kf[gamma][I*n+J] = Kfull(p,q,I,J) + [p != q] Kfull(q,p,I,J).
FEI_HD constexpr int kfolded(int form, int dim, int p, int q, int I, int J)
{
    return kfull(form, dim, p, q, I, J) + (p != q ? kfull(form, dim, q, p, I, J) : 0);
}

// Tables (block K as float, MFMA fragments) are emitted as literals by
// gen_tables.cpp at build time from the functions above: clang's constant
// evaluator is too slow to build them inside the compiler.

}  // namespace fei
