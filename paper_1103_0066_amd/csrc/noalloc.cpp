// fei_integrate_adjoint_det_noalloc: the deterministic adjoint with its
// workspace (vertex-to-element incidence and J-bar per element) in a fixed
// device array of this library instead of a stream-ordered allocation, for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, allocation-free harnesses).
//
// The array `scratch` exists once per device that loads this library and lives
// until the process ends.  In host code its name only stands for the variable:
// its device address is resolved once per device with hipGetSymbolAddress
// (with that device current) and kept; kernels receive that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fei.h"
#include "host.h"

using namespace fei;
using namespace fei::host;

namespace {

constexpr size_t kScratchBytes = FEI_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size must keep 256-byte alignment");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices];   // device address of `scratch`, per device id

// Device address of `scratch` on the current device, resolved on first use.
int scratch_address(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(FEI_EUNSUPPORTED, "device id %d beyond the %d devices the scratch table keeps",
                    dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(FEI_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return FEI_OK;
}

}  // namespace

extern "C" int fei_integrate_adjoint_det_noalloc(const fei_mesh *m, int form, const float *mu,
                                                 const float *lam, const float *dA, float *dx,
                                                 float *dy, float *dz, float *dmu, float *dlam,
                                                 const fei_options *opt, void *stream)
{
    AdjParams p;
    Variant v;
    int rc = prepare_adjoint(m, form, mu, lam, dA, dx, dy, dz, dmu, dlam, opt, p, v);
    if (rc) return rc < 0 ? rc : FEI_OK;
    if ((rc = check_det(m, v))) return rc;
    const DetLayout L = det_layout(m->dim, m->n_elements, m->n_vertices);
    if (L.total > kScratchBytes)
        return fail(FEI_EINVAL,
                    "mesh needs %zu bytes of workspace (%lld elements, %lld vertices); the "
                    "allocation-free adjoint holds at most %zu",
                    L.total, (long long)m->n_elements, (long long)m->n_vertices, kScratchBytes);
    void *base = nullptr;
    if ((rc = scratch_address(&base))) return rc;
    // Every part of the workspace that must start at zero is cleared by the
    // incidence build's own kernels (no memset nodes, so the call may be
    // captured into a graph).
    return enqueue_adjoint_det(p, v, base, L, static_cast<hipStream_t>(stream));
}
