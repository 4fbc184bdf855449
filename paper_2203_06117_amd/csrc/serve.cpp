// Batching and serving entry points (filled in once the plain path is validated).
#include "host.h"

extern "C" gs_status gs_serve_start(gs_ctx *ctx, int32_t, const int32_t *, const int32_t *, const int32_t *,
                                    const int32_t *, int32_t)
{
    return gs_fail(ctx, GS_E_STATE, "serving not available in this build");
}
extern "C" gs_status gs_submit(gs_ctx *ctx, const gs_request *, uint64_t *)
{
    return gs_fail(ctx, GS_E_STATE, "serving not available in this build");
}
extern "C" gs_status gs_poll(gs_ctx *ctx, uint64_t, int32_t, gs_result *)
{
    return gs_fail(ctx, GS_E_STATE, "serving not available in this build");
}
extern "C" gs_status gs_release(gs_ctx *ctx, uint64_t)
{
    return gs_fail(ctx, GS_E_STATE, "serving not available in this build");
}
extern "C" gs_status gs_serve_stop(gs_ctx *ctx)
{
    return gs_fail(ctx, GS_E_STATE, "serving not available in this build");
}
void gs_serve_shutdown(gs_ctx *) {}
