// Batched independent systems.
#include "md_internal.h"

using namespace mdlj;

struct md_batch {
    int dummy;
};

extern "C" int md_batch_create(const md_config *, int32_t, const int64_t *, const double *, md_batch **out)
{
    if (out) *out = nullptr;
    return fail(MD_ERR_INVALID_ARG, "batched systems are not available in this build");
}
extern "C" void md_batch_destroy(md_batch *b) { delete b; }
extern "C" int md_batch_build_cells(md_batch *, double *, void *, void *, int32_t *, int32_t *, void *)
{
    return fail(MD_ERR_INVALID_ARG, "batched systems are not available in this build");
}
extern "C" int md_batch_compute_forces(md_batch *, const double *, const int32_t *, const double *, void *, double *,
                                       void *)
{
    return fail(MD_ERR_INVALID_ARG, "batched systems are not available in this build");
}
extern "C" int md_batch_step(md_batch *, double *, void *, void *, int32_t *, int32_t *, const double *,
                             const double *, double, int32_t, int32_t, void *)
{
    return fail(MD_ERR_INVALID_ARG, "batched systems are not available in this build");
}
