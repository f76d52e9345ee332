// axf_batch.hip -- batches of runs and the continuous-batching server.
#include "axf_runtime.h"

using namespace axf;

extern "C" {

int axf_batch_footprint(const axf_config *, int32_t, size_t *) { return fail(AXF_EINVAL, "batches not built yet"); }
int axf_batch_create(const axf_config *, int32_t, void *, size_t, void *, axf_batch **) { return fail(AXF_EINVAL, "batches not built yet"); }
int axf_batch_step(axf_batch *, const int64_t *) { return fail(AXF_EINVAL, "batches not built yet"); }
int axf_batch_run(axf_batch *, int32_t, axf_run **) { return fail(AXF_EINVAL, "batches not built yet"); }
int axf_batch_destroy(axf_batch *) { return AXF_OK; }
int axf_server_create(void *, size_t, int32_t, int32_t, void *, axf_server **) { return fail(AXF_EINVAL, "server not built yet"); }
int axf_server_submit(axf_server *, const axf_config *, int64_t, uint64_t *) { return fail(AXF_EINVAL, "server not built yet"); }
int axf_server_cancel(axf_server *, uint64_t) { return fail(AXF_EINVAL, "server not built yet"); }
int axf_server_poll(axf_server *, axf_result *, int32_t, int32_t *) { return fail(AXF_EINVAL, "server not built yet"); }
int axf_server_stats(axf_server *, int32_t *, int32_t *, size_t *) { return fail(AXF_EINVAL, "server not built yet"); }
int axf_server_destroy(axf_server *) { return AXF_OK; }

}
