// Host side of libfei: argument validation, kernel dispatch, status codes.
// Implements every entry point declared in include/fei.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fei.h"
#include "params.h"
#include "shapes.h"
#include "host.h"

using namespace fei;

namespace fei {
namespace host {

thread_local std::string g_last_error;

int fail(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(FEI_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

bool valid_form(int form) { return form == FEI_LAPLACE_P1 || form == FEI_ELASTIC_P1 || form == FEI_LAPLACE_P2; }

int local_size(int form, int dim)
{
    if (!valid_form(form) || (dim != 2 && dim != 3)) return -1;
    const int nb = (form == FEI_LAPLACE_P2) ? (dim + 1) * (dim + 2) / 2 : dim + 1;
    return form == FEI_ELASTIC_P1 ? dim * nb : nb;
}

fei_options defaults()
{
    fei_options o;
    std::memset(&o, 0, sizeof o);
    o.precision = FEI_PREC_FP32;
    o.tau = 100.0f;
    o.counters = nullptr;
    o.store_rows = 0;
    return o;
}

int check_options(const fei_options &o)
{
    if (o.precision < FEI_PREC_FP32 || o.precision > FEI_PREC_BF16X3)
        return fail(FEI_EINVAL, "unknown precision %d", o.precision);
    if (std::isnan(o.tau)) return fail(FEI_EINVAL, "tau is NaN");
    for (int r : o.reserved)
        if (r != 0) return fail(FEI_EINVAL, "fei_options.reserved must be zero");
    if (o.block_elements != 0 && o.block_elements != 64 && o.block_elements != 128 &&
        o.block_elements != 256 && o.block_elements != 512)
        return fail(FEI_EINVAL, "block_elements must be 0, 64, 128, 256 or 512 (got %d)",
                    o.block_elements);
    if (o.counters && !aligned(o.counters, 4)) return fail(FEI_EINVAL, "counters misaligned");
    return FEI_OK;
}

float tau2_of(float tau)
{
    if (tau <= 0.0f) return -1.0f;   // every element takes the FP64 path
    return tau * tau;                // +Inf stays +Inf
}

// Validates the mesh struct and fills the kernel view.
int check_mesh(const fei_mesh *m, MeshView &mv)
{
    if (!m) return fail(FEI_EINVAL, "mesh is NULL");
    if (m->dim != 2 && m->dim != 3) return fail(FEI_EINVAL, "dim must be 2 or 3 (got %d)", m->dim);
    if (m->coord_dtype != FEI_F32 && m->coord_dtype != FEI_F64)
        return fail(FEI_EINVAL, "unknown coord_dtype %d", m->coord_dtype);
    if (m->n_elements < 0) return fail(FEI_EINVAL, "n_elements < 0");
    if (m->n_elements > kMaxElements)
        return fail(FEI_EINVAL, "n_elements exceeds %lld (one launch covers at most 2^32 threads)",
                    (long long)kMaxElements);
    if (m->n_elements > 0) {
        if (m->n_vertices < 1) return fail(FEI_EINVAL, "n_vertices < 1");
        if (m->n_vertices > int64_t(INT32_MAX) + 1)
            return fail(FEI_EINVAL, "n_vertices exceeds the int32 connectivity range");
        const size_t cs = m->coord_dtype == FEI_F64 ? 8 : 4;
        if (!m->x || !m->y) return fail(FEI_EINVAL, "x or y is NULL");
        if (m->dim == 3 && !m->z) return fail(FEI_EINVAL, "z is NULL for a 3D mesh");
        if (!aligned(m->x, cs) || !aligned(m->y, cs) || (m->dim == 3 && !aligned(m->z, cs)))
            return fail(FEI_EINVAL, "coordinate arrays misaligned");
        if (!m->conn) return fail(FEI_EINVAL, "conn is NULL");
        if (!aligned(m->conn, m->dim == 3 ? 16 : 4))
            return fail(FEI_EINVAL, "conn must be %d-byte aligned", m->dim == 3 ? 16 : 4);
    }
    mv.x = m->x;
    mv.y = m->y;
    mv.z = m->dim == 3 ? m->z : nullptr;
    mv.conn = m->conn;
    mv.n_elements = m->n_elements;
    mv.n_vertices = m->n_vertices;
    return FEI_OK;
}

int check_coeffs(int form, const float *mu, const float *lam, int64_t E)
{
    if (form == FEI_ELASTIC_P1) {
        if (E > 0 && (!mu || !lam)) return fail(FEI_EINVAL, "elasticity needs mu and lam");
        if ((mu && !aligned(mu, 4)) || (lam && !aligned(lam, 4)))
            return fail(FEI_EINVAL, "mu/lam misaligned");
    } else if (mu || lam) {
        return fail(FEI_EINVAL, "mu/lam must be NULL for a Laplacian form");
    }
    return FEI_OK;
}

// Shared argument checks of the adjoint entry points.  Returns a negative
// status, FEI_OK with p and v filled, or 1 when there is nothing to do (E = 0).
int prepare_adjoint(const fei_mesh *m, int form, const float *mu, const float *lam,
                    const float *dA, float *dx, float *dy, float *dz, float *dmu, float *dlam,
                    const fei_options *opt, AdjParams &p, Variant &v)
{
    MeshView mv;
    int rc = check_mesh(m, mv);
    if (rc) return rc;
    if (!valid_form(form)) return fail(FEI_EINVAL, "unknown form %d", form);
    fei_options o = opt ? *opt : defaults();
    if ((rc = check_options(o))) return rc;
    if (o.precision != FEI_PREC_FP32 && m->coord_dtype != FEI_F32)
        return fail(FEI_EUNSUPPORTED, "the split-precision adjoint takes FP32 coordinates");
    if ((rc = check_coeffs(form, mu, lam, m->n_elements))) return rc;
    if (form != FEI_ELASTIC_P1 && (dmu || dlam))
        return fail(FEI_EINVAL, "dmu/dlam must be NULL for a Laplacian form");
    if (m->n_elements == 0) return 1;
    if (!dA || !aligned(dA, 16)) return fail(FEI_EINVAL, "dA NULL or not 16-byte aligned");
    if (!dx || !dy || (m->dim == 3 && !dz)) return fail(FEI_EINVAL, "dx/dy/dz missing");
    if (!aligned(dx, 4) || !aligned(dy, 4) || (dz && !aligned(dz, 4)))
        return fail(FEI_EINVAL, "dx/dy/dz misaligned");
    v = Variant{form, m->dim, m->coord_dtype == FEI_F64, o.precision, o.store_rows, 0};
    p.m = mv;
    p.mu = mu;
    p.lam = lam;
    p.dA = dA;
    p.dx = dx;
    p.dy = dy;
    p.dz = m->dim == 3 ? dz : nullptr;
    p.dmu = dmu;
    p.dlam = dlam;
    p.counters = o.counters;
    p.tau2 = tau2_of(o.tau);
    p.jbar = nullptr;
    return FEI_OK;
}

DetLayout det_layout(int dim, int64_t E, int64_t Nv)
{
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    DetLayout L;
    size_t o = 0;
    L.ptr = o;
    o += up(size_t(Nv + 1) * 4);
    L.cursor = o;
    o += up(size_t(Nv) * 4);
    L.inc = o;
    o += up(size_t(E) * size_t(dim + 1) * 4);
    L.jbar = o;
    o += up(size_t(E) * size_t(dim) * size_t(dim) * 4);
    L.total = o;
    return L;
}

int check_det(const fei_mesh *m, Variant &v)
{
    if (m->coord_dtype != FEI_F32)
        return fail(FEI_EUNSUPPORTED, "the deterministic adjoint takes FP32 coordinates");
    if (v.rows != 0)
        return fail(FEI_EUNSUPPORTED, "the deterministic adjoint uses its own dA staging "
                                      "(store_rows must be 0)");
    if (m->n_elements * (m->dim + 1) > int64_t(INT32_MAX))
        return fail(FEI_EUNSUPPORTED, "the deterministic adjoint needs (dim+1) * n_elements < 2^31");
    v.gather = 1;
    return find_adjoint(v) ? FEI_OK : fail(FEI_EUNSUPPORTED, "no adjoint kernel for this variant");
}

// Incidence build, J-bar adjoint and vertex gather on stream s, in the
// workspace at base (layout L, 256-byte aligned parts).  Every part that must
// start at zero is cleared by the incidence build's own kernels.
int enqueue_adjoint_det(AdjParams p, const Variant &v, void *base, const DetLayout &L,
                        hipStream_t s)
{
    char *b = static_cast<char *>(base);
    int32_t *ptr = reinterpret_cast<int32_t *>(b + L.ptr);
    int32_t *cursor = reinterpret_cast<int32_t *>(b + L.cursor);
    int32_t *inc = reinterpret_cast<int32_t *>(b + L.inc);
    float *jbar = reinterpret_cast<float *>(b + L.jbar);
    const int nv = p.m.n_elements > 0 ? v.dim + 1 : 0;
    Incidence g{p.m.conn, p.m.n_elements, p.m.n_vertices, nv, ptr, inc, cursor};
    hipError_t e = launch_incidence_build(g, s);
    if (e != hipSuccess) return hip_fail(e, "incidence build");
    p.jbar = jbar;
    const AdjLauncher launch = find_adjoint(v);
    if (!launch) return fail(FEI_EUNSUPPORTED, "no adjoint kernel for this variant");
    if ((e = launch(p, s)) != hipSuccess) return hip_fail(e, "adjoint launch");
    GatherItem gi{};
    gi.ptr = ptr;
    gi.inc = inc;
    gi.jbar = jbar;
    gi.dx = p.dx;
    gi.dy = p.dy;
    gi.dz = p.dz;
    gi.v_begin = 0;
    gi.n_vertices = p.m.n_vertices;
    gi.dim = v.dim;
    gi.atomic = 0;
    if ((e = launch_vertex_gather_one(gi, s)) != hipSuccess) return hip_fail(e, "vertex gather");
    return FEI_OK;
}

}  // namespace host
}  // namespace fei

using namespace fei::host;

namespace {

// K of (form, dim) through the same functions the kernels' tables come from.
template <typename F>
int with_traits(int form, int dim, F &&f)
{
    if (dim == 2) {
        if (form == FEI_LAPLACE_P1) return f(Traits<LAP1, 2>{});
        if (form == FEI_ELASTIC_P1) return f(Traits<ELA1, 2>{});
        if (form == FEI_LAPLACE_P2) return f(Traits<LAP2, 2>{});
    } else if (dim == 3) {
        if (form == FEI_LAPLACE_P1) return f(Traits<LAP1, 3>{});
        if (form == FEI_ELASTIC_P1) return f(Traits<ELA1, 3>{});
        if (form == FEI_LAPLACE_P2) return f(Traits<LAP2, 3>{});
    }
    return fail(FEI_EINVAL, "bad form %d or dim %d", form, dim);
}

}  // namespace

extern "C" {

int fei_abi_version(void) { return FEI_ABI_VERSION; }

const char *fei_status_str(int status)
{
    switch (status) {
    case FEI_OK: return "success";
    case FEI_EINVAL: return "invalid argument";
    case FEI_EDEVICE: return "device (HIP) error";
    case FEI_ENOMEM: return "out of memory";
    case FEI_EUNSUPPORTED: return "unsupported variant";
    default: return "unknown status";
    }
}

const char *fei_last_error(void) { return g_last_error.c_str(); }

int fei_options_default(fei_options *opt)
{
    if (!opt) return fail(FEI_EINVAL, "opt is NULL");
    *opt = defaults();
    return FEI_OK;
}

int fei_local_size(int form, int dim)
{
    const int n = local_size(form, dim);
    return n < 0 ? fail(FEI_EINVAL, "bad form %d or dim %d", form, dim) : n;
}

double fei_reference_scale(int form, int dim)
{
    double s = 0.0;
    with_traits(form, dim, [&](auto t) {
        s = decltype(t)::SCALE;
        return FEI_OK;
    });
    return s;
}

int fei_reference_tensor(int form, int dim, int layout, float *K, int64_t *len, int32_t *g_out)
{
    if (!len) return fail(FEI_EINVAL, "len is NULL");
    if (layout != FEI_LAYOUT_BLOCK && layout != FEI_LAYOUT_FOLDED)
        return fail(FEI_EINVAL, "unknown layout %d", layout);
    return with_traits(form, dim, [&](auto t) {
        using T = decltype(t);
        const int F = form == FEI_LAPLACE_P1 ? LAP1 : form == FEI_ELASTIC_P1 ? ELA1 : LAP2;
        if (layout == FEI_LAYOUT_BLOCK) {
            *len = int64_t(T::NB) * T::NB * dim * dim;
            if (g_out) *g_out = T::G;
            if (!K) return FEI_OK;
            // eq. 7 values: the integer tensor times vol_ref / KDEN
            for (int i = 0; i < T::NB; ++i)
                for (int j = 0; j < T::NB; ++j)
                    for (int mu = 0; mu < dim; ++mu)
                        for (int nu = 0; nu < dim; ++nu)
                            K[((i * T::NB + j) * dim + mu) * dim + nu] =
                                float(double(kblock(F, dim, i, j, mu, nu)) * T::SCALE);
            return FEI_OK;
        }
        const int nn = T::N * T::N;
        *len = int64_t(T::G) * nn;
        if (g_out) *g_out = T::G;
        if (!K) return FEI_OK;
        for (int g = 0; g < T::G; ++g) {
            int p = 0, q = 0;
            sym_pair(T::GD, g, p, q);
            for (int I = 0; I < T::N; ++I)
                for (int J = 0; J < T::N; ++J)
                    K[int64_t(g) * nn + I * T::N + J] = float(kfolded(F, dim, p, q, I, J));
        }
        return FEI_OK;
    });
}

int fei_integrate(const fei_mesh *m, int form, const float *mu, const float *lam, float *A,
                  const fei_options *opt, void *stream)
{
    MeshView mv;
    int rc = check_mesh(m, mv);
    if (rc) return rc;
    if (!valid_form(form)) return fail(FEI_EINVAL, "unknown form %d", form);
    fei_options o = opt ? *opt : defaults();
    if ((rc = check_options(o))) return rc;
    if ((rc = check_coeffs(form, mu, lam, m->n_elements))) return rc;
    if (m->n_elements == 0) return FEI_OK;
    if (!A) return fail(FEI_EINVAL, "A is NULL");
    if (!aligned(A, 16)) return fail(FEI_EINVAL, "A must be 16-byte aligned");
    Variant v{form, m->dim, m->coord_dtype == FEI_F64, o.precision, o.store_rows, 0,
              o.block_elements};
    if (o.block_elements == 0 && o.store_rows == 0) {
        fei_tune_result t;
        if (tune_find(form, m->dim, o.precision, m->coord_dtype, m->n_elements, t)) {
            v.block = t.block_elements;
            v.rows = t.store_rows;
        }
    }
    FwdLauncher launch = find_forward(v);
    if (!launch) return fail(FEI_EUNSUPPORTED, "no forward kernel for this variant");
    FwdParams p;
    p.m = mv;
    p.mu = mu;
    p.lam = lam;
    p.w = nullptr;
    p.A = A;
    p.counters = o.counters;
    p.tau2 = tau2_of(o.tau);
    hipError_t e = launch(p, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    return FEI_OK;
}

int fei_integrate_coefficient(const fei_mesh *m, int form, const float *w, float *A,
                              const fei_options *opt, void *stream)
{
    MeshView mv;
    int rc = check_mesh(m, mv);
    if (rc) return rc;
    if (form != FEI_LAPLACE_P1 && form != FEI_LAPLACE_P2)
        return fail(valid_form(form) ? FEI_EUNSUPPORTED : FEI_EINVAL,
                    "a P1 coefficient is taken by the Laplacian forms (form %d)", form);
    fei_options o = opt ? *opt : defaults();
    if ((rc = check_options(o))) return rc;
    if (m->n_elements == 0) return FEI_OK;
    if (!w || !aligned(w, 4)) return fail(FEI_EINVAL, "w NULL or misaligned");
    if (!A) return fail(FEI_EINVAL, "A is NULL");
    if (!aligned(A, 16)) return fail(FEI_EINVAL, "A must be 16-byte aligned");
    const Variant v{form == FEI_LAPLACE_P1 ? int(WLAP1) : int(WLAP2), m->dim,
                    m->coord_dtype == FEI_F64, o.precision, o.store_rows, 0};
    FwdLauncher launch = find_forward_coefficient(v);
    if (!launch)
        return fail(FEI_EUNSUPPORTED, "no kernel for this variant (the contraction is FP32; "
                                      "store_rows 0, -1, n or 2)");
    FwdParams p;
    p.m = mv;
    p.mu = nullptr;
    p.lam = nullptr;
    p.w = w;
    p.A = A;
    p.counters = o.counters;
    p.tau2 = tau2_of(o.tau);
    hipError_t e = launch(p, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "forward launch");
    return FEI_OK;
}

int fei_integrate_iso(const fei_mesh *m, float *A, const fei_options *opt, void *stream)
{
    MeshView mv;
    int rc = check_mesh(m, mv);
    if (rc) return rc;
    if (m->coord_dtype != FEI_F32)
        return fail(FEI_EUNSUPPORTED, "the isoparametric form takes FP32 coordinates");
    fei_options o = opt ? *opt : defaults();
    if ((rc = check_options(o))) return rc;
    if (o.precision != FEI_PREC_FP32)
        return fail(FEI_EUNSUPPORTED, "the isoparametric form contracts in FP32");
    if (o.store_rows != 0)
        return fail(FEI_EUNSUPPORTED, "the isoparametric form stages whole matrices");
    if (m->n_elements == 0) return FEI_OK;
    if (!A || !aligned(A, 16)) return fail(FEI_EINVAL, "A NULL or not 16-byte aligned");
    FwdParams p;
    p.m = mv;
    p.mu = p.lam = p.w = nullptr;
    p.A = A;
    p.counters = o.counters;
    p.tau2 = tau2_of(o.tau);
    hipError_t e = launch_iso(m->dim, p, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FEI_OK : hip_fail(e, "isoparametric launch");
}

int fei_reference_tensor_coefficient(int form, int dim, float *K, int64_t *len)
{
    if (!len) return fail(FEI_EINVAL, "len is NULL");
    if ((form != FEI_LAPLACE_P1 && form != FEI_LAPLACE_P2) || (dim != 2 && dim != 3))
        return fail(FEI_EINVAL, "bad form %d or dim %d", form, dim);
    const int F = form == FEI_LAPLACE_P1 ? WLAP1 : WLAP2;
    const int nb = form == FEI_LAPLACE_P1 ? dim + 1 : (dim + 1) * (dim + 2) / 2;
    const int kden = form == FEI_LAPLACE_P1 ? dim + 1 : (dim + 1) * (dim + 2) * (dim + 3);
    const double scale = 1.0 / (double(dim == 2 ? 2 : 6) * kden);
    *len = int64_t(nb) * nb * (dim + 1) * dim * dim;
    if (!K) return FEI_OK;
    int64_t t = 0;
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j)
            for (int k = 0; k <= dim; ++k)
                for (int mu = 0; mu < dim; ++mu)
                    for (int nu = 0; nu < dim; ++nu)
                        K[t++] = float(double(kwblock(F, dim, i, j, k, mu, nu)) * scale);
    return FEI_OK;
}

int fei_integrate_adjoint(const fei_mesh *m, int form, const float *mu, const float *lam,
                          const float *dA, float *dx, float *dy, float *dz, float *dmu,
                          float *dlam, const fei_options *opt, void *stream)
{
    AdjParams p;
    Variant v;
    int rc = prepare_adjoint(m, form, mu, lam, dA, dx, dy, dz, dmu, dlam, opt, p, v);
    if (rc) return rc < 0 ? rc : FEI_OK;
    AdjLauncher launch = find_adjoint(v);
    if (!launch) return fail(FEI_EUNSUPPORTED, "no adjoint kernel for this variant");
    hipError_t e = launch(p, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "adjoint launch");
    return FEI_OK;
}

int fei_integrate_adjoint_det(const fei_mesh *m, int form, const float *mu, const float *lam,
                              const float *dA, float *dx, float *dy, float *dz, float *dmu,
                              float *dlam, const fei_options *opt, void *stream)
{
    AdjParams p;
    Variant v;
    int rc = prepare_adjoint(m, form, mu, lam, dA, dx, dy, dz, dmu, dlam, opt, p, v);
    if (rc) return rc < 0 ? rc : FEI_OK;
    if ((rc = check_det(m, v))) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const DetLayout L = det_layout(m->dim, m->n_elements, m->n_vertices);
    void *base = nullptr;
    hipError_t e = hipMallocAsync(&base, L.total, s);
    if (e != hipSuccess) return fail(FEI_ENOMEM, "deterministic adjoint workspace: %s",
                                     hipGetErrorString(e));
    rc = enqueue_adjoint_det(p, v, base, L, s);
    e = hipFreeAsync(base, s);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "hipFreeAsync");
    return FEI_OK;
}

int fei_validate_mesh(const fei_mesh *m, int64_t *n_bad, void *stream)
{
    MeshView mv;
    int rc = check_mesh(m, mv);
    if (rc) return rc;
    if (!n_bad) return fail(FEI_EINVAL, "n_bad is NULL");
    *n_bad = 0;
    if (m->n_elements == 0) return FEI_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned long long *dev = nullptr;
    hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&dev), sizeof(unsigned long long), s);
    if (e != hipSuccess) return hip_fail(e, "hipMallocAsync");
    unsigned long long host = 0;
    if ((e = hipMemsetAsync(dev, 0, sizeof host, s)) == hipSuccess &&
        (e = launch_validate(mv, m->dim, dev, s)) == hipSuccess &&
        (e = hipMemcpyAsync(&host, dev, sizeof host, hipMemcpyDeviceToHost, s)) == hipSuccess)
        e = hipStreamSynchronize(s);
    hipError_t e2 = hipFreeAsync(dev, s);
    if (e != hipSuccess) return hip_fail(e, "validate");
    if (e2 != hipSuccess) return hip_fail(e2, "hipFreeAsync");
    *n_bad = int64_t(host);
    return FEI_OK;
}

}  // extern "C"
