// placeholder, replaced by the batched implementation
#include "../../include/asd_extra.h"
#include "asd_internal.h"
extern "C" int asd_batch_workspace_bytes(const asd_desc*, int32_t, size_t*) { return asd_fail(ASD_EUNSUPPORTED, "batch not built yet"); }
extern "C" int asd_batch_init(const asd_desc*, int32_t, void*, size_t, void*, asd_batch*) { return asd_fail(ASD_EUNSUPPORTED, "batch not built yet"); }
extern "C" int asd_batch_set_problem(asd_batch, int32_t, void*, void*, void*, double) { return asd_fail(ASD_EUNSUPPORTED, "batch not built yet"); }
extern "C" int asd_batch_step(asd_batch, int32_t, int32_t) { return asd_fail(ASD_EUNSUPPORTED, "batch not built yet"); }
extern "C" int asd_batch_destroy(asd_batch) { return asd_fail(ASD_EUNSUPPORTED, "batch not built yet"); }
