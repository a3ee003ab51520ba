// Placeholder entry points for the tetrahedral-mesh and batched forms.
#include "runtime.h"

using namespace sal;

extern "C" {
sal_status sal_tet_mesh_create_lattice(sal_context *, const double *, double, const int32_t *,
                                       sal_tet_mesh **out) {
    if (out) *out = nullptr;
    return set_error(SAL_ERR_INTERNAL, "tetrahedral mesh not available in this build");
}
void sal_tet_mesh_destroy(sal_tet_mesh *) {}
sal_status sal_refine_relabel(sal_context *, sal_tet_mesh *, const sal_surface_set *, int32_t,
                              const sal_label_options *, sal_refine_stats *) {
    return set_error(SAL_ERR_INTERNAL, "refinement not available in this build");
}
sal_status sal_tet_mesh_size(const sal_tet_mesh *, int64_t *, int32_t *) {
    return set_error(SAL_ERR_INTERNAL, "tetrahedral mesh not available in this build");
}
sal_status sal_tet_mesh_export(sal_context *, const sal_tet_mesh *, uint64_t *, int32_t *, float *,
                               float *, float *) {
    return set_error(SAL_ERR_INTERNAL, "tetrahedral mesh not available in this build");
}
sal_status sal_label_batch(sal_context *, const sal_instance *, int32_t, const sal_label_options *,
                           sal_label_stats *) {
    return set_error(SAL_ERR_INTERNAL, "batched form not available in this build");
}
}
