// Form front end, library side (fei_form_*): from a weak-form description --
// the element (dimension, Lagrange degree, components) and the operator
// tables W of A_{(i,c),(j,d)} = int sum_{a,b} C[(a,c),(b,d)] D_a phi_i D_b phi_j
// (D_0 the value, D_{1+alpha} = d/dx_alpha, C = W_0 + sum_k coef_k W_k) --
// it builds what the contraction of Sec. 3, eq. 1 needs:
//
//   * the reference tensor Khat_ij^{pq} = int_ref Dhat_p phi_i Dhat_q phi_j
//     (eq. 7 over values and reference derivatives), exactly, in rational
//     arithmetic on barycentric monomials: int_ref lambda^alpha = alpha! /
//     (|alpha| + dim)!  (Sec. 3.1: K is computable a priori, independent of the
//     mesh and the form's coefficients);
//   * the recipe of the geometric tensor: W itself, which the kernel turns into
//     G = |J| That^T C_e That per element (fwd_form.h).
#include <hip/hip_runtime.h>

#include <array>
#include <cmath>
#include <cstdlib>
#include <map>
#include <new>
#include <numeric>
#include <vector>

#include "fei.h"
#include "host.h"
#include "params.h"
#include "polyint.h"

using namespace fei;
using namespace fei::host;
using namespace fei::poly;

struct fei_weak_form {
    int dim = 0, degree = 0, ncomp = 0, n_coef = 0, sym = 0, noval = 0;
    int nb = 0, n = 0, m = 0, nd = 0;
    float kscale = 1.f;
    float *d_W = nullptr, *d_K = nullptr;
};

namespace {

// Khat [nb][nb][nd][nd] exactly; returns the common denominator of all its
// entries (0 if it or a scaled numerator would not be exact in FP32).
int64_t reference_tensor(int dim, int degree, std::vector<Rat> &K)
{
    const std::vector<Poly> B = lagrange_basis(dim, degree);
    const int nb = int(B.size()), nd = dim + 1;
    std::vector<std::vector<Poly>> D(nb, std::vector<Poly>(nd));
    for (int i = 0; i < nb; ++i) {
        D[i][0] = B[i];
        for (int mu = 0; mu < dim; ++mu) D[i][1 + mu] = dxi(B[i], mu);
    }
    K.assign(size_t(nb) * nb * nd * nd, Rat(0));
    int64_t lcd = 1;
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j)
            for (int pp = 0; pp < nd; ++pp)
                for (int q = 0; q < nd; ++q) {
                    const Rat v = integrate_ref(mul(D[i][pp], D[j][q]), dim);
                    K[((size_t(i) * nb + j) * nd + pp) * nd + q] = v;
                    lcd = lcd / std::gcd(lcd, v.q) * v.q;
                    if (lcd > (int64_t(1) << 40)) lcd = 0;
                    if (lcd == 0) return 0;
                }
    for (const Rat &v : K) {
        const int64_t scaled = v.p * (lcd / v.q);
        if ((scaled < 0 ? -scaled : scaled) >= (int64_t(1) << 24)) return 0;
    }
    return lcd;
}

void release(fei_weak_form *f)
{
    if (f->d_W) (void)hipFree(f->d_W);
    if (f->d_K) (void)hipFree(f->d_K);
    delete f;
}

}  // namespace

extern "C" {

int fei_form_create(int dim, int degree, int ncomp, int n_coef, const double *W, fei_weak_form **out)
{
    if (!out) return fail(FEI_EINVAL, "out is NULL");
    *out = nullptr;
    if (dim != 2 && dim != 3) return fail(FEI_EINVAL, "dim must be 2 or 3 (got %d)", dim);
    if (degree != 1 && degree != 2) return fail(FEI_EINVAL, "degree must be 1 or 2 (got %d)", degree);
    if (ncomp != 1 && ncomp != dim)
        return fail(FEI_EINVAL, "ncomp must be 1 or dim (got %d)", ncomp);
    if (n_coef < 0 || n_coef > kFormMaxCoef)
        return fail(FEI_EINVAL, "n_coef must be in [0, %d] (got %d)", kFormMaxCoef, n_coef);
    if (!W) return fail(FEI_EINVAL, "W is NULL");
    const int nd = dim + 1, m = nd * ncomp;
    const size_t nw = size_t(n_coef + 1) * m * m;
    for (size_t t = 0; t < nw; ++t)
        if (!std::isfinite(W[t])) return fail(FEI_EINVAL, "W[%zu] is not finite", t);

    std::vector<Rat> Kr;
    const int64_t lcd = reference_tensor(dim, degree, Kr);
    fei_weak_form *f = new (std::nothrow) fei_weak_form();
    if (!f) return fail(FEI_ENOMEM, "form");
    f->dim = dim;
    f->degree = degree;
    f->ncomp = ncomp;
    f->n_coef = n_coef;
    f->nd = nd;
    f->m = m;
    f->nb = degree == 1 ? dim + 1 : (dim + 1) * (dim + 2) / 2;
    f->n = ncomp * f->nb;
    int sym = 1;
    for (int k = 0; k <= n_coef && sym; ++k)
        for (int r = 0; r < m && sym; ++r)
            for (int c = r + 1; c < m; ++c)
                if (W[(size_t(k) * m + r) * m + c] != W[(size_t(k) * m + c) * m + r]) { sym = 0; break; }
    f->sym = sym;
    // no value operator on either side: G and Khat reduce to the derivative
    // operators (the kernel skips the value rows and columns)
    int noval = 1;
    for (int k = 0; k <= n_coef && noval; ++k)
        for (int c = 0; c < ncomp && noval; ++c)
            for (int t = 0; t < m; ++t)
                if (W[(size_t(k) * m + c) * m + t] != 0.0 || W[(size_t(k) * m + t) * m + c] != 0.0) {
                    noval = 0;
                    break;
                }
    f->noval = noval;
    // Khat as integers over the common denominator when that is exact in FP32
    // (1 / lcd folds into |det J|), else as rounded values
    f->kscale = lcd ? float(1.0 / double(lcd)) : 1.f;
    std::vector<float> Kf(Kr.size()), Wf(nw);
    for (size_t t = 0; t < Kr.size(); ++t)
        Kf[t] = lcd ? float(Kr[t].p * (lcd / Kr[t].q)) : float(Kr[t].value());
    for (size_t t = 0; t < nw; ++t) Wf[t] = float(W[t]);
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&f->d_W), nw * 4);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&f->d_K), Kf.size() * 4);
    if (e != hipSuccess) {
        release(f);
        return fail(FEI_ENOMEM, "form tables: %s", hipGetErrorString(e));
    }
    if ((e = hipMemcpy(f->d_W, Wf.data(), nw * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(f->d_K, Kf.data(), Kf.size() * 4, hipMemcpyHostToDevice)) != hipSuccess) {
        release(f);
        return hip_fail(e, "form tables upload");
    }
    *out = f;
    return FEI_OK;
}

int fei_form_info(const fei_weak_form *f, int32_t *n, int32_t *symmetric, int32_t *n_coef)
{
    if (!f) return fail(FEI_EINVAL, "form is NULL");
    if (n) *n = f->n;
    if (symmetric) *symmetric = f->sym;
    if (n_coef) *n_coef = f->n_coef;
    return FEI_OK;
}

int fei_form_reference_tensor(int dim, int degree, double *K, int64_t *len)
{
    if (!len) return fail(FEI_EINVAL, "len is NULL");
    if ((dim != 2 && dim != 3) || (degree != 1 && degree != 2))
        return fail(FEI_EINVAL, "bad dim %d or degree %d", dim, degree);
    std::vector<Rat> Kr;
    reference_tensor(dim, degree, Kr);
    *len = int64_t(Kr.size());
    if (K)
        for (size_t t = 0; t < Kr.size(); ++t) K[t] = Kr[t].value();
    return FEI_OK;
}

int fei_form_integrate(const fei_weak_form *f, const fei_mesh *m, const float *coef, float *A,
                       const fei_options *opt, void *stream)
{
    if (!f) return fail(FEI_EINVAL, "form is NULL");
    MeshView mv;
    int rc = check_mesh(m, mv);
    if (rc) return rc;
    if (m->dim != f->dim)
        return fail(FEI_EINVAL, "mesh dimension %d, form dimension %d", m->dim, f->dim);
    if (m->coord_dtype != FEI_F32)
        return fail(FEI_EUNSUPPORTED, "forms take FP32 coordinates");
    fei_options o = opt ? *opt : defaults();
    if ((rc = check_options(o))) return rc;
    if (o.precision != FEI_PREC_FP32)
        return fail(FEI_EUNSUPPORTED, "forms contract in FP32");
    if (o.store_rows != 0) return fail(FEI_EUNSUPPORTED, "forms use their own output staging");
    if (m->n_elements == 0) return FEI_OK;
    if (f->n_coef > 0 && (!coef || !aligned(coef, 4)))
        return fail(FEI_EINVAL, "the form has %d coefficients: coef NULL or misaligned", f->n_coef);
    if (!A || !aligned(A, 16)) return fail(FEI_EINVAL, "A NULL or not 16-byte aligned");
    FormParams p;
    p.m = mv;
    p.coef = f->n_coef > 0 ? coef : nullptr;
    p.n_coef = f->n_coef;
    p.W = f->d_W;
    p.K = f->d_K;
    p.kscale = f->kscale;
    p.A = A;
    p.counters = o.counters;
    p.tau2 = tau2_of(o.tau);
    hipError_t e = launch_form(f->dim, f->degree, f->ncomp, f->sym != 0, f->noval != 0, p,
                               static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FEI_OK : hip_fail(e, "form launch");
}

int fei_form_destroy(fei_weak_form *f)
{
    if (f) release(f);
    return FEI_OK;
}

}  // extern "C"
