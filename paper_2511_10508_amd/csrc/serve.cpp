// Serving engine (continuous batching).  Placeholder until the scheduler lands.
#include "../../include/pfmi.h"
#include "pf_runtime.h"

using namespace pf;
#define PF_API extern "C" __attribute__((visibility("default")))

PF_API pf_status pf_server_create(int32_t, uint64_t, int32_t, int32_t, pf_server **out)
{
    if (out) *out = nullptr;
    return fail(PF_ERR_UNSUPPORTED, "serving not built yet");
}
PF_API pf_status pf_server_submit(pf_server *, const pf_desc *, int32_t, uint64_t, const double *,
                                  int32_t, int64_t, uint64_t *)
{
    return fail(PF_ERR_UNSUPPORTED, "serving not built yet");
}
PF_API pf_status pf_server_poll(pf_server *, pf_result *, int32_t, int32_t *n)
{
    if (n) *n = 0;
    return fail(PF_ERR_UNSUPPORTED, "serving not built yet");
}
PF_API pf_status pf_server_fetch(pf_server *, uint64_t, int32_t, double *, int64_t)
{
    return fail(PF_ERR_UNSUPPORTED, "serving not built yet");
}
PF_API pf_status pf_server_release(pf_server *, uint64_t) { return fail(PF_ERR_UNSUPPORTED, "serving not built yet"); }
PF_API pf_status pf_server_cancel(pf_server *, uint64_t) { return fail(PF_ERR_UNSUPPORTED, "serving not built yet"); }
PF_API pf_status pf_server_drain(pf_server *, double) { return fail(PF_ERR_UNSUPPORTED, "serving not built yet"); }
PF_API pf_status pf_server_stats(pf_server *, int64_t *, int64_t *, int64_t *, int64_t *)
{
    return fail(PF_ERR_UNSUPPORTED, "serving not built yet");
}
PF_API void pf_server_destroy(pf_server *) {}
