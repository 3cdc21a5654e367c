// Heterogeneous batches (fei_batch_*).
#include <hip/hip_runtime.h>

#include "fei.h"

extern "C" {

struct fei_batch {
    int unused;
};

int fei_batch_create(const fei_batch_item *, int, const fei_options *, fei_batch **out)
{
    if (out) *out = nullptr;
    return FEI_EUNSUPPORTED;
}
int fei_batch_run(fei_batch *, void *) { return FEI_EUNSUPPORTED; }
int fei_batch_run_adjoint(fei_batch *, void *) { return FEI_EUNSUPPORTED; }
int fei_batch_destroy(fei_batch *) { return FEI_OK; }

}  // extern "C"
