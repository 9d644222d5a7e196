// Cluster-pair lists (8-particle clusters).
#include "md_internal.h"

struct md_handle;

namespace mdlj {

int cluster_build_impl(md_handle *h, const double *pos, hipStream_t s)
{
    (void)h;
    (void)pos;
    (void)s;
    return fail(MD_ERR_INVALID_ARG, "cluster lists are not available in this build");
}

void launch_cluster_force(const ForceArgs &a, const Geom &g, hipStream_t s)
{
    (void)a;
    (void)g;
    (void)s;
}

}  // namespace mdlj
