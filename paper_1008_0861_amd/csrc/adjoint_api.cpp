// placeholder, replaced by the adjoint implementation
#include "asd_internal.h"
extern "C" int asd_adjoint_workspace_bytes(asd_grid g, int32_t, int32_t, size_t*) {
    if (!g) return asd_fail(ASD_EINVAL, "grid is NULL");
    return asd_fail(ASD_EUNSUPPORTED, "adjoint not built yet");
}
extern "C" int asd_adjoint_step(asd_grid g, double, int32_t, int32_t, const void*, const void*, void*, void*, void*, size_t) {
    if (!g) return asd_fail(ASD_EINVAL, "grid is NULL");
    return asd_fail(ASD_EUNSUPPORTED, "adjoint not built yet");
}
