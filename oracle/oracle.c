/* FP64 CPU oracle for finite-element element matrices.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library: it never forms the paper's
 * reference tensor K or geometric tensor G (Sec. 3, eqs. 1, 6-8) and instead
 * integrates each element directly on the physical simplex:
 *
 *   1. vertex coordinates in double;
 *   2. barycentric functions from the inverse of the Vandermonde matrix with
 *      rows [1, x_a] (LU with partial pivoting); volume = |det V| / d!;
 *   3. a Grundmann-Moeller simplex rule (Grundmann & Moeller, SIAM J. Numer.
 *      Anal. 15 (1978)) -- degree 3 by default, exact for P1 and P2 stiffness;
 *   4. basis gradients at the points (P1, or P2 vertex/edge functions);
 *   5. Laplacian: sum_k w_k grad phi_i . grad phi_j  (Sec. 3, eqs. 3-4);
 *      elasticity: sum_k w_k Bv^T D Bv with the Voigt strain-displacement
 *      matrix Bv and isotropic Hooke matrix D (the Lame form of Sec. 3,
 *      eqs. 9-12; mu = 1/2, lambda = 0 gives the form of eq. 24).
 *
 * Gradients of L = sum_IJ dA_IJ A_IJ with respect to vertex coordinates and
 * the Lame coefficients use the complex-step derivative (Squire & Trapp, SIAM
 * Rev. 40 (1998)) of the same routine instantiated on double _Complex:
 * dL/dp = Im L(p + i h) / h, exact to rounding for h = 1e-30.
 *
 * Conventions: reference DOF order is node-major, I = dim*a + c; P2 edges
 * are ordered (0,1),(0,2),...,(d-1,d) after the d+1 vertices.
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_LAPLACE 0
#define ORACLE_ELASTIC 1

#define ORACLE_MAX_QP 128

int oracle_version(void) { return 1; }

/* Threads of the OpenMP loops over elements (n >= 1); returns the count the
 * next parallel region will use.  Timing only: results do not depend on it. */
int oracle_set_threads(int n)
{
    if (n >= 1) omp_set_num_threads(n);
    return omp_get_max_threads();
}

static long factorial(int k)
{
    long f = 1;
    for (int i = 2; i <= k; ++i) f *= i;
    return f;
}

/* Enumerate all beta in N^{m} with |beta| = total, calling back with each. */
static int compositions(int total, int m, int *beta, int pos, int (*out)[4], int count)
{
    if (pos == m - 1) {
        beta[pos] = total;
        for (int j = 0; j < m; ++j) out[count][j] = beta[j];
        return count + 1;
    }
    for (int b = 0; b <= total; ++b) {
        beta[pos] = b;
        count = compositions(total - b, m, beta, pos + 1, out, count);
    }
    return count;
}

/* Grundmann-Moeller rule of degree 2s+1 on the d-simplex.
 * Points in barycentric coordinates (d+1 of them), weights summing to the
 * volume of the unit simplex, 1/d!:
 *   w_i = (-1)^i 2^{-2s} (2s+1+d-2i)^{2s+1} / (i! (2s+1+d-i)!),  i = 0..s,
 *   points ((2 beta_0 + 1), ..., (2 beta_d + 1)) / (2s+1+d-2i), |beta| = s-i.
 * Returns the number of points, or -1 if they do not fit.                 */
int oracle_gm_rule(int dim, int s, double pts[][4], double *w)
{
    const int deg = 2 * s + 1;
    int count = 0;
    for (int i = 0; i <= s; ++i) {
        int betas[ORACLE_MAX_QP][4], beta[4];
        int nb = compositions(s - i, dim + 1, beta, 0, betas, 0);
        if (count + nb > ORACLE_MAX_QP) return -1;
        double wi = pow(2.0, -2.0 * s) * pow((double)(deg + dim - 2 * i), deg)
                    / ((double)factorial(i) * (double)factorial(deg + dim - i));
        if (i % 2) wi = -wi;
        for (int k = 0; k < nb; ++k) {
            for (int j = 0; j <= dim; ++j)
                pts[count][j] = (2.0 * betas[k][j] + 1.0) / (double)(deg + dim - 2 * i);
            for (int j = dim + 1; j < 4; ++j) pts[count][j] = 0.0;
            w[count] = wi;
            ++count;
        }
    }
    return count;
}

/* ---- real instantiation ------------------------------------------------ */
#define R double
#define RE(v) (v)
#define FN(name) name##_d
#include "element.inc"
#undef R
#undef RE
#undef FN

/* ---- complex instantiation (complex-step derivatives) ------------------ */
#define R double _Complex
#define RE(v) creal(v)
#define FN(name) name##_z
#include "element.inc"
#undef R
#undef RE
#undef FN

static int local_size(int kind, int degree, int dim)
{
    int nv = dim + 1;
    int nb = (degree == 1) ? nv : nv * (nv + 1) / 2;
    return (kind == ORACLE_ELASTIC) ? dim * nb : nb;
}

static int check_args(int kind, int degree, int dim, int qs)
{
    if (kind != ORACLE_LAPLACE && kind != ORACLE_ELASTIC) return -1;
    if (degree != 1 && degree != 2) return -1;
    if (dim != 2 && dim != 3) return -1;
    if (qs < 0 || qs > 4) return -1;
    return 0;
}

/* One element: xv[a*dim + alpha].  Returns det V (d! x signed volume) in *detv. */
int oracle_element(int kind, int degree, int dim, const double *xv, double mu,
                   double lam, int qs, double *A, double *detv)
{
    if (check_args(kind, degree, dim, qs)) return -1;
    double d = element_matrix_d(kind, degree, dim, xv, mu, lam, NULL, qs, A);
    if (detv) *detv = d;
    return 0;
}

/* All elements of a mesh.
 *   coords: SoA double arrays x, y (, z) of length nv (z ignored in 2D)
 *   conn:   [ne][dim+1] int32
 *   mu,lam: [ne] (elasticity only; may be NULL otherwise)
 *   A:      [ne][n][n] double output                                     */
int oracle_integrate(int kind, int degree, int dim, int64_t nv,
                     const double *x, const double *y, const double *z,
                     int64_t ne, const int32_t *conn, const double *mu,
                     const double *lam, int qs, double *A)
{
    if (check_args(kind, degree, dim, qs)) return -1;
    if (kind == ORACLE_ELASTIC && (!mu || !lam)) return -1;
    const int n = local_size(kind, degree, dim);
    const double *X[3] = {x, y, z};
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(|:bad)
    for (int64_t e = 0; e < ne; ++e) {
        double xv[12];
        for (int a = 0; a <= dim; ++a) {
            int32_t v = conn[e * (dim + 1) + a];
            if (v < 0 || v >= nv) { bad = 1; v = 0; }
            for (int al = 0; al < dim; ++al) xv[a * dim + al] = X[al][v];
        }
        double m = mu ? mu[e] : 0.0, l = lam ? lam[e] : 0.0;
        element_matrix_d(kind, degree, dim, xv, m, l, NULL, qs, A + e * (int64_t)n * n);
    }
    return bad ? -2 : 0;
}

/* The Laplacian with a P1 coefficient (Sec. 3.1, eqs. 20-21):
 *   A_ij = int_T w grad phi_i . grad phi_j,   w = sum_a w[conn[e][a]] lambda_a,
 * for every element; w is given per vertex ([nv]).  Same layout as
 * oracle_integrate.  The default rule (qs = 1, degree 3) is exact for P1 and
 * P2 (integrand degree 1 and 3).                                          */
int oracle_integrate_w(int degree, int dim, int64_t nv,
                       const double *x, const double *y, const double *z,
                       int64_t ne, const int32_t *conn, const double *w, int qs, double *A)
{
    if (check_args(ORACLE_LAPLACE, degree, dim, qs) || !w) return -1;
    const int n = local_size(ORACLE_LAPLACE, degree, dim);
    const double *X[3] = {x, y, z};
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(|:bad)
    for (int64_t e = 0; e < ne; ++e) {
        double xv[12], wv[4];
        for (int a = 0; a <= dim; ++a) {
            int32_t v = conn[e * (dim + 1) + a];
            if (v < 0 || v >= nv) { bad = 1; v = 0; }
            for (int al = 0; al < dim; ++al) xv[a * dim + al] = X[al][v];
            wv[a] = w[v];
        }
        element_matrix_d(ORACLE_LAPLACE, degree, dim, xv, 0.0, 0.0, wv, qs,
                         A + e * (int64_t)n * n);
    }
    return bad ? -2 : 0;
}

/* Values of the scalar basis at barycentric point bc (P1: lambda_a; P2: vertex
 * a: lambda_a (2 lambda_a - 1); edge (a,b): 4 lambda_a lambda_b, edges in the
 * order of basis_gradients).                                               */
static void basis_values(int degree, int dim, const double *bc, double *phi)
{
    const int nv = dim + 1;
    if (degree == 1) {
        for (int a = 0; a < nv; ++a) phi[a] = bc[a];
        return;
    }
    for (int a = 0; a < nv; ++a) phi[a] = bc[a] * (2.0 * bc[a] - 1.0);
    int e = nv;
    for (int a = 0; a < nv; ++a)
        for (int b = a + 1; b < nv; ++b, ++e) phi[e] = 4.0 * bc[a] * bc[b];
}

/* A general bilinear form of Lagrange elements (degree 1 or 2, ncomp = 1 or
 * dim components, node-major DOFs I = ncomp * i + c):
 *
 *   A_{(i,c),(j,d)} = int_T sum_{a,b} C[(a,c),(b,d)] D_a phi_i D_b phi_j,
 *
 * with D_0 = the value and D_{1+alpha} = d/dx_alpha (physical derivatives),
 * C[(a,c),(b,d)] = W_0 + sum_k coef_k(e) W_k a per-element combination of
 * the tables W ([n_coef + 1][m][m], m = (dim + 1) * ncomp, index a * ncomp + c).
 * This is the plain definition of the forms a form language describes
 * (Sec. 3.2): quadrature on the physical element, physical gradients from
 * the Vandermonde inverse, no reference tensor.  coef: [n_coef][ne].      */
int oracle_integrate_general(int degree, int dim, int ncomp, int64_t nv,
                             const double *x, const double *y, const double *z,
                             int64_t ne, const int32_t *conn, int n_coef, const double *W,
                             const double *coef, int qs, double *A)
{
    if ((degree != 1 && degree != 2) || (dim != 2 && dim != 3) ||
        (ncomp != 1 && ncomp != dim) || n_coef < 0 || n_coef > 8 || qs < 0 || qs > 4)
        return -1;
    const int nvert = dim + 1;
    const int nb = (degree == 1) ? nvert : nvert * (nvert + 1) / 2;
    const int n = ncomp * nb;
    const int m = (dim + 1) * ncomp;
    const double *X[3] = {x, y, z};
    double pts[ORACLE_MAX_QP][4], w[ORACLE_MAX_QP];
    const int nq = oracle_gm_rule(dim, qs, pts, w);
    if (nq < 0) return -1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(|:bad)
    for (int64_t e = 0; e < ne; ++e) {
        double V[4][4], Cv[4][4], gl[4][3];
        for (int a = 0; a < nvert; ++a) {
            int32_t v = conn[e * nvert + a];
            if (v < 0 || v >= nv) { bad = 1; v = 0; }
            V[a][0] = 1.0;
            for (int al = 0; al < dim; ++al) V[a][1 + al] = X[al][v];
        }
        const double detV = vandermonde_inverse_d(nvert, V, Cv);
        const double absdet = detV < 0.0 ? -detV : detV;
        for (int a = 0; a < nvert; ++a)
            for (int al = 0; al < dim; ++al) gl[a][al] = Cv[1 + al][a];
        double C[36 * 36];
        for (int t = 0; t < m * m; ++t) {
            double c = W[t];
            for (int k = 0; k < n_coef; ++k) c += coef[k * ne + e] * W[(size_t)(k + 1) * m * m + t];
            C[t] = c;
        }
        double *Ae = A + e * (int64_t)n * n;
        for (int t = 0; t < n * n; ++t) Ae[t] = 0.0;
        for (int q = 0; q < nq; ++q) {
            double g[10][3], phi[10], D[4][10];
            basis_gradients_d(degree, dim, pts[q], gl, g);
            basis_values(degree, dim, pts[q], phi);
            for (int i = 0; i < nb; ++i) {
                D[0][i] = phi[i];
                for (int al = 0; al < dim; ++al) D[1 + al][i] = g[i][al];
            }
            const double wq = w[q] * absdet;
            for (int i = 0; i < nb; ++i)
                for (int c = 0; c < ncomp; ++c)
                    for (int j = 0; j < nb; ++j)
                        for (int d = 0; d < ncomp; ++d) {
                            double s = 0.0;
                            for (int a = 0; a <= dim; ++a)
                                for (int b = 0; b <= dim; ++b)
                                    s += C[(a * ncomp + c) * m + b * ncomp + d] * D[a][i] * D[b][j];
                            Ae[(ncomp * i + c) * n + ncomp * j + d] += wq * s;
                        }
        }
    }
    return bad ? -2 : 0;
}

/* ---- isoparametric P2 Laplacian (Sec. 3.1, eqs. 16-19) ------------------ */

/* Reference gradients d psi_n / d xi_mu of the P2 basis (vertices, then edges
 * (0,1),(0,2),..) at the barycentric point bc; lambda_0 = 1 - sum xi,
 * lambda_{m+1} = xi_m.                                                      */
static void p2_ref_gradients(int dim, const double *bc, double g[10][3])
{
    const int nv = dim + 1;
    double gl[4][3];
    for (int a = 0; a < nv; ++a)
        for (int mu = 0; mu < dim; ++mu) gl[a][mu] = (a == 0) ? -1.0 : (a - 1 == mu ? 1.0 : 0.0);
    for (int a = 0; a < nv; ++a)
        for (int mu = 0; mu < dim; ++mu) g[a][mu] = (4.0 * bc[a] - 1.0) * gl[a][mu];
    int e = nv;
    for (int a = 0; a < nv; ++a)
        for (int b = a + 1; b < nv; ++b, ++e)
            for (int mu = 0; mu < dim; ++mu) g[e][mu] = 4.0 * (bc[a] * gl[b][mu] + bc[b] * gl[a][mu]);
}

/* J[alpha][mu] = sum_n x_n[alpha] dpsi_n/dxi_mu at bc; B = J^-1 (rows mu,
 * columns alpha) by cofactors; returns det J.                              */
static double iso_jacobian(int dim, int nb, const double xn[10][3], const double *bc,
                           double B[3][3])
{
    double g[10][3], J[3][3];
    p2_ref_gradients(dim, bc, g);
    for (int al = 0; al < dim; ++al)
        for (int mu = 0; mu < dim; ++mu) {
            double s = 0.0;
            for (int n = 0; n < nb; ++n) s += xn[n][al] * g[n][mu];
            J[al][mu] = s;
        }
    double det;
    if (dim == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        B[0][0] = J[1][1] / det;  B[0][1] = -J[0][1] / det;
        B[1][0] = -J[1][0] / det; B[1][1] = J[0][0] / det;
    } else {
        double c[3][3];
        c[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        c[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
        c[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
        c[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        c[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
        c[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
        c[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        c[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
        c[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        det = J[0][0] * c[0][0] + J[0][1] * c[1][0] + J[0][2] * c[2][0];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) B[i][j] = c[i][j] / det;
    }
    return det;
}

/* Isoparametric P2 Laplacian on elements with quadratic geometry: conn
 * [ne][nb] lists each element's nodes (vertices, then edge nodes in the P2
 * order), which carry both the geometry map x(xi) = sum_n x_n psi_n(xi) and
 * the solution basis phi_i = psi_i.
 *   mode 0, the paper's scheme: the inverse Jacobian projected onto P1 by its
 *     values at the vertices, J^-1(xi) ~ sum_k lambda_k(xi) J(xi_k)^-1, and
 *     |J| taken out of the integral as a constant, |det J| at the barycenter:
 *       A_ij = |J_c| int_ref (Bp^T dphi_i) . (Bp^T dphi_j) dxi,
 *     an integrand of degree 4 (GM degree 2qs+1 >= 5 integrates it exactly);
 *   mode 1, the isoparametric integral itself, J(xi) at every point:
 *       A_ij = int_ref (J^-T dphi_i) . (J^-T dphi_j) |det J(xi)| dxi
 *     (a rational integrand: the rule's degree sets its accuracy).        */
int oracle_integrate_iso(int dim, int64_t nv, const double *x, const double *y,
                         const double *z, int64_t ne, const int32_t *conn, int mode, int qs,
                         double *A)
{
    if ((dim != 2 && dim != 3) || (mode != 0 && mode != 1) || qs < 0 || qs > 4) return -1;
    const int nvert = dim + 1, nb = nvert * (nvert + 1) / 2;
    const double *X[3] = {x, y, z};
    double pts[ORACLE_MAX_QP][4], w[ORACLE_MAX_QP];
    const int nq = oracle_gm_rule(dim, qs, pts, w);
    if (nq < 0) return -1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(|:bad)
    for (int64_t e = 0; e < ne; ++e) {
        double xn[10][3];
        for (int n = 0; n < nb; ++n) {
            int32_t v = conn[e * nb + n];
            if (v < 0 || v >= nv) { bad = 1; v = 0; }
            for (int al = 0; al < dim; ++al) xn[n][al] = X[al][v];
        }
        double Bk[4][3][3], sc = 0.0;
        if (mode == 0) {
            for (int k = 0; k < nvert; ++k) {
                double bc[4] = {0.0, 0.0, 0.0, 0.0};
                bc[k] = 1.0;
                iso_jacobian(dim, nb, xn, bc, Bk[k]);
            }
            double bc[4], Bc[3][3];
            for (int a = 0; a < nvert; ++a) bc[a] = 1.0 / nvert;
            sc = fabs(iso_jacobian(dim, nb, xn, bc, Bc));
        }
        double *Ae = A + e * (int64_t)nb * nb;
        for (int t = 0; t < nb * nb; ++t) Ae[t] = 0.0;
        for (int q = 0; q < nq; ++q) {
            double B[3][3], wq;
            if (mode == 0) {
                for (int mu = 0; mu < dim; ++mu)
                    for (int al = 0; al < dim; ++al) {
                        double s = 0.0;
                        for (int k = 0; k < nvert; ++k) s += pts[q][k] * Bk[k][mu][al];
                        B[mu][al] = s;
                    }
                wq = w[q] * sc;
            } else {
                wq = w[q] * fabs(iso_jacobian(dim, nb, xn, pts[q], B));
            }
            double g[10][3], gx[10][3];
            p2_ref_gradients(dim, pts[q], g);
            for (int i = 0; i < nb; ++i)
                for (int al = 0; al < dim; ++al) {
                    double s = 0.0;
                    for (int mu = 0; mu < dim; ++mu) s += B[mu][al] * g[i][mu];
                    gx[i][al] = s;
                }
            for (int i = 0; i < nb; ++i)
                for (int j = 0; j < nb; ++j) {
                    double s = 0.0;
                    for (int al = 0; al < dim; ++al) s += gx[i][al] * gx[j][al];
                    Ae[i * nb + j] += wq * s;
                }
        }
    }
    return bad ? -2 : 0;
}

/* Complex-step gradient of L_e = sum_IJ dA_e[I][J] A_e[I][J] for each element.
 *   gvert: [ne][dim+1][dim]  dL_e / d x_{conn[e][a]}[alpha]
 *   gmu, glam: [ne] or NULL  dL_e / d mu_e, dL_e / d lambda_e
 *   Lval: [ne] or NULL       L_e itself                                     */
int oracle_gradient(int kind, int degree, int dim, int64_t nv,
                    const double *x, const double *y, const double *z,
                    int64_t ne, const int32_t *conn, const double *mu,
                    const double *lam, const double *dA, int qs,
                    double *gvert, double *gmu, double *glam, double *Lval)
{
    if (check_args(kind, degree, dim, qs)) return -1;
    if (kind == ORACLE_ELASTIC && (!mu || !lam)) return -1;
    const int n = local_size(kind, degree, dim);
    const double *X[3] = {x, y, z};
    const double h = 1e-30;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(|:bad)
    for (int64_t e = 0; e < ne; ++e) {
        double xv[12];
        for (int a = 0; a <= dim; ++a) {
            int32_t v = conn[e * (dim + 1) + a];
            if (v < 0 || v >= nv) { bad = 1; v = 0; }
            for (int al = 0; al < dim; ++al) xv[a * dim + al] = X[al][v];
        }
        const double *dAe = dA + e * (int64_t)n * n;
        double m = mu ? mu[e] : 0.0, l = lam ? lam[e] : 0.0;
        const int np = (dim + 1) * dim;
        const int nparam = np + ((kind == ORACLE_ELASTIC) ? 2 : 0);
        double _Complex Az[30 * 30];
        for (int p = -1; p < nparam; ++p) {
            double _Complex xz[12], mz = m, lz = l;
            for (int k = 0; k < np; ++k) xz[k] = xv[k];
            if (p >= 0 && p < np) xz[p] += h * I;
            if (p == np) mz += h * I;
            if (p == np + 1) lz += h * I;
            element_matrix_z(kind, degree, dim, xz, mz, lz, NULL, qs, Az);
            double _Complex L = 0.0;
            for (int k = 0; k < n * n; ++k) L += dAe[k] * Az[k];
            if (p < 0) {
                if (Lval) Lval[e] = creal(L);
            } else if (p < np) {
                gvert[e * np + p] = cimag(L) / h;
            } else if (p == np) {
                if (gmu) gmu[e] = cimag(L) / h;
            } else {
                if (glam) glam[e] = cimag(L) / h;
            }
        }
    }
    return bad ? -2 : 0;
}
