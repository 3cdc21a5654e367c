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

}  // namespace host
}  // namespace fei
