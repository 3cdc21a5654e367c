// Host-side helpers shared by the entry points (api.cpp, batch.cpp):
// thread-local error text, argument checks, option defaults.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "fei.h"
#include "params.h"

namespace fei {
namespace host {

// Largest mesh one call accepts: a launch covers at most 2^32 threads, one per
// element (grids of 256-thread workgroups).
constexpr int64_t kMaxElements = (int64_t(1) << 32) - 256;

int fail(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_fail(hipError_t e, const char *what);
bool aligned(const void *p, size_t a);
bool valid_form(int form);
int local_size(int form, int dim);
fei_options defaults();
int check_options(const fei_options &o);
float tau2_of(float tau);
int check_mesh(const fei_mesh *m, MeshView &mv);
int check_coeffs(int form, const float *mu, const float *lam, int64_t E);
int prepare_adjoint(const fei_mesh *m, int form, const float *mu, const float *lam,
                    const float *dA, float *dx, float *dy, float *dz, float *dmu, float *dlam,
                    const fei_options *opt, AdjParams &p, Variant &v);

// Workspace of the deterministic adjoint: the vertex-to-element incidence
// (ptr, cursor, inc) and J-bar per element, each part 256-byte aligned.
struct DetLayout {
    size_t ptr, cursor, inc, jbar, total;
};
DetLayout det_layout(int dim, int64_t E, int64_t Nv);
// Checks a prepared adjoint for the deterministic path; sets v.gather.
int check_det(const fei_mesh *m, Variant &v);
int enqueue_adjoint_det(AdjParams p, const Variant &v, void *base, const DetLayout &L,
                        hipStream_t s);

// Tune table (tune.cpp): the entry for a forward call, if any.
bool tune_find(int form, int dim, int precision, int coord_dtype, int64_t n_elements,
               fei_tune_result &out);

}  // namespace host
}  // namespace fei
