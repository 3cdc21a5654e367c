// Fused global assembly (fei_assembly_*): the host builds, once per mesh, the
// sparsity pattern of the global matrix and the vertex-to-element incidence
// the assembly kernel walks, then each fei_assemble call integrates every
// element and sums it into the matrix values on the device (assemble.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "fei.h"
#include "host.h"
#include "params.h"
#include "schedule.h"

using namespace fei;
using namespace fei::host;

struct fei_assembly {
    int form = 0, dim = 0, nc = 1;
    int64_t n_vertices = 0, n_elements = 0, nnz = 0;
    int64_t n_chunks = 0, n_sched = 0;
    int32_t *d_ptr = nullptr, *d_inc = nullptr, *d_rowptr = nullptr, *d_colidx = nullptr,
            *d_chunks = nullptr, *d_slots = nullptr;
};

namespace {

void release(fei_assembly *a)
{
    for (int32_t *p : {a->d_ptr, a->d_inc, a->d_rowptr, a->d_colidx, a->d_chunks, a->d_slots})
        if (p) (void)hipFree(p);
    delete a;
}

int upload(const std::vector<int32_t> &v, int32_t **dst)
{
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), std::max<size_t>(v.size(), 1) * 4);
    if (e != hipSuccess) return fail(FEI_ENOMEM, "assembly pattern: %s", hipGetErrorString(e));
    if (!v.empty() &&
        (e = hipMemcpy(*dst, v.data(), v.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "assembly pattern upload");
    return FEI_OK;
}

}  // namespace

extern "C" {

int fei_assembly_create(const fei_mesh *m, int form, fei_assembly **out)
{
    if (!out) return fail(FEI_EINVAL, "out is NULL");
    *out = nullptr;
    MeshView mv;
    int rc = check_mesh(m, mv);
    if (rc) return rc;
    if (form != FEI_LAPLACE_P1 && form != FEI_ELASTIC_P1)
        return fail(valid_form(form) ? FEI_EUNSUPPORTED : FEI_EINVAL,
                    "fused assembly is for the P1 forms (form %d)", form);
    const int nv = m->dim + 1;
    const int64_t E = m->n_elements, Nv = m->n_vertices;
    if (E * nv > int64_t(INT32_MAX) || Nv >= int64_t(INT32_MAX))
        return fail(FEI_EUNSUPPORTED, "fused assembly needs (dim+1) * n_elements < 2^31");

    // connectivity on the host (device-synchronizing), validated
    std::vector<int32_t> conn(size_t(E) * nv);
    if (E > 0) {
        hipError_t e = hipDeviceSynchronize();
        if (e == hipSuccess)
            e = hipMemcpy(conn.data(), m->conn, conn.size() * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "connectivity download");
    }
    for (int32_t v : conn)
        if (v < 0 || int64_t(v) >= Nv)
            return fail(FEI_EINVAL, "connectivity entry %d outside [0, %lld)", v, (long long)Nv);

    // vertex-to-element incidence, entries e * nv + a in increasing order
    std::vector<int32_t> ptr(size_t(Nv) + 1, 0), inc(conn.size());
    for (int32_t v : conn) ++ptr[size_t(v) + 1];
    for (int64_t v = 0; v < Nv; ++v) ptr[v + 1] += ptr[v];
    {
        std::vector<int32_t> cur(ptr.begin(), ptr.end() - 1);
        for (size_t i = 0; i < conn.size(); ++i) inc[cur[conn[i]]++] = int32_t(i);
    }
    // pattern: row v holds every vertex that shares an element with v, sorted
    std::vector<int32_t> rowptr(size_t(Nv) + 1, 0), colidx;
    colidx.reserve(conn.size() * 4);
    std::vector<int32_t> row;
    const int max_slots = assemble_chunk_slots(), max_rows = assemble_chunk_rows();
    for (int64_t v = 0; v < Nv; ++v) {
        row.clear();
        for (int32_t j = ptr[v]; j < ptr[v + 1]; ++j) {
            const int64_t e = inc[j] / nv;
            for (int b = 0; b < nv; ++b) row.push_back(conn[size_t(e) * nv + b]);
        }
        std::sort(row.begin(), row.end());
        row.erase(std::unique(row.begin(), row.end()), row.end());
        if (int(row.size()) > max_slots)
            return fail(FEI_EUNSUPPORTED,
                        "vertex %lld has %zu neighbours; fused assembly takes at most %d",
                        (long long)v, row.size(), max_slots);
        colidx.insert(colidx.end(), row.begin(), row.end());
        if (colidx.size() > size_t(INT32_MAX))
            return fail(FEI_EUNSUPPORTED, "the pattern exceeds 2^31 blocks");
        rowptr[v + 1] = int32_t(colidx.size());
    }
    // chunks of consecutive rows, one per wave: at most max_rows rows and
    // max_slots blocks each
    std::vector<int32_t> chunks{0};
    {
        int64_t r0 = 0;
        for (int64_t v = 0; v < Nv; ++v) {
            if (v - r0 + 1 > max_rows || rowptr[v + 1] - rowptr[r0] > max_slots) {
                chunks.push_back(int32_t(v));
                r0 = v;
            }
        }
        if (Nv > 0) chunks.push_back(int32_t(Nv));
    }

    // the kernel walks each row's incidences in conflict-free steps
    std::vector<int32_t> sptr(size_t(Nv) + 1, 0), sinc;
    sinc.reserve(inc.size() + inc.size() / 4);
    {
        const int lanes = assemble_lanes();
        for (int64_t v = 0; v < Nv; ++v) {
            schedule_row(int32_t(v), inc.data() + ptr[v], ptr[v + 1] - ptr[v], conn, nv, lanes, sinc);
            if (sinc.size() > size_t(INT32_MAX))
                return fail(FEI_EUNSUPPORTED, "the incidence schedule exceeds 2^31 entries");
            sptr[v + 1] = int32_t(sinc.size());
        }
    }
    // per schedule entry, the slots of its element's vertices in the row's
    // sorted columns, relative to the row's first (one byte per vertex: a row
    // has at most max_slots < 256 columns)
    std::vector<int32_t> sslot(sinc.size(), 0);
    for (int64_t v = 0; v < Nv; ++v) {
        const int32_t *c0 = colidx.data() + rowptr[v], *c1 = colidx.data() + rowptr[v + 1];
        for (int32_t j = sptr[v]; j < sptr[v + 1]; ++j) {
            if (sinc[j] < 0) continue;
            const int64_t e = sinc[j] / nv;
            uint32_t packed = 0;
            for (int b = 0; b < nv; ++b) {
                const int32_t w = conn[size_t(e) * nv + b];
                const uint32_t rel = uint32_t(std::lower_bound(c0, c1, w) - c0);
                packed |= rel << (8 * b);
            }
            sslot[j] = int32_t(packed);
        }
    }

    fei_assembly *a = new (std::nothrow) fei_assembly();
    if (!a) return fail(FEI_ENOMEM, "assembly plan");
    a->form = form;
    a->dim = m->dim;
    a->nc = form == FEI_ELASTIC_P1 ? m->dim : 1;
    a->n_vertices = Nv;
    a->n_elements = E;
    a->nnz = int64_t(colidx.size());
    a->n_chunks = int64_t(chunks.size()) - 1;
    a->n_sched = int64_t(sinc.size());
    if ((rc = upload(sptr, &a->d_ptr)) || (rc = upload(sinc, &a->d_inc)) || (rc = upload(sslot, &a->d_slots)) ||
        (rc = upload(rowptr, &a->d_rowptr)) || (rc = upload(colidx, &a->d_colidx)) ||
        (rc = upload(chunks, &a->d_chunks))) {
        release(a);
        return rc;
    }
    *out = a;
    return FEI_OK;
}

int fei_assembly_info(const fei_assembly *a, int64_t *n_rows, int64_t *nnz, int32_t *block)
{
    if (!a) return fail(FEI_EINVAL, "plan is NULL");
    if (n_rows) *n_rows = a->n_vertices;
    if (nnz) *nnz = a->nnz;
    if (block) *block = a->nc;
    return FEI_OK;
}

int fei_assembly_copy_pattern(const fei_assembly *a, int32_t *rowptr, int32_t *colidx,
                              void *stream)
{
    if (!a || !rowptr || (!colidx && a->nnz > 0)) return fail(FEI_EINVAL, "bad argument");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(rowptr, a->d_rowptr, size_t(a->n_vertices + 1) * 4,
                                  hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && a->nnz > 0)
        e = hipMemcpyAsync(colidx, a->d_colidx, size_t(a->nnz) * 4, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? FEI_OK : hip_fail(e, "pattern copy");
}

int fei_assembly_copy_schedule(const fei_assembly *a, int64_t *n_entries, int32_t *ptr,
                               int32_t *inc, void *stream)
{
    if (!a || !n_entries) return fail(FEI_EINVAL, "bad argument");
    *n_entries = a->n_sched;
    if (!ptr && !inc) return FEI_OK;
    if (!ptr || (!inc && a->n_sched > 0)) return fail(FEI_EINVAL, "ptr or inc is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(ptr, a->d_ptr, size_t(a->n_vertices + 1) * 4,
                                  hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && a->n_sched > 0)
        e = hipMemcpyAsync(inc, a->d_inc, size_t(a->n_sched) * 4, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? FEI_OK : hip_fail(e, "schedule copy");
}

int fei_assemble(const fei_assembly *a, const fei_mesh *m, const float *mu, const float *lam,
                 float *values, const fei_options *opt, void *stream)
{
    if (!a) return fail(FEI_EINVAL, "plan is NULL");
    MeshView mv;
    int rc = check_mesh(m, mv);
    if (rc) return rc;
    if (m->dim != a->dim || m->n_vertices != a->n_vertices || m->n_elements != a->n_elements)
        return fail(FEI_EINVAL, "the mesh differs from the one the plan was built for");
    if (m->coord_dtype != FEI_F32)
        return fail(FEI_EUNSUPPORTED, "fused assembly takes FP32 coordinates");
    fei_options o = opt ? *opt : defaults();
    if ((rc = check_options(o))) return rc;
    if (o.precision != FEI_PREC_FP32)
        return fail(FEI_EUNSUPPORTED, "fused assembly contracts in FP32");
    if ((rc = check_coeffs(a->form, mu, lam, m->n_elements))) return rc;
    if (a->nnz == 0) return FEI_OK;
    if (!values || !aligned(values, 4)) return fail(FEI_EINVAL, "values NULL or misaligned");
    AsmParams p;
    p.m = mv;
    p.mu = mu;
    p.lam = lam;
    p.ptr = a->d_ptr;
    p.inc = a->d_inc;
    p.slots = a->d_slots;
    p.rowptr = a->d_rowptr;
    p.colidx = a->d_colidx;
    p.chunks = a->d_chunks;
    p.n_chunks = a->n_chunks;
    p.values = values;
    p.counters = o.counters;
    p.tau2 = tau2_of(o.tau);
    hipError_t e = launch_assemble(a->form, a->dim, p, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FEI_OK : hip_fail(e, "assembly launch");
}

int fei_assembly_destroy(fei_assembly *a)
{
    if (a) release(a);
    return FEI_OK;
}

}  // extern "C"
