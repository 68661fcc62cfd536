// Serving loop: trig_stream_submit / trig_stream_poll (filled in below).
#include "api_internal.h"

struct ServeState {};

void serve_shutdown(trig_ctx *c) {
    delete c->serve;
    c->serve = nullptr;
}

extern "C" {

int trig_stream_submit(trig_ctx *c, const trig_slice_desc *, const trig_params *, uint64_t *) {
    if (!c) return TRIG_EINVAL;
    ctx_set_error(c, "serving loop not available");
    return TRIG_EINVAL;
}

int trig_stream_poll(trig_ctx *c, uint64_t, trig_result *, int32_t) {
    if (!c) return TRIG_EINVAL;
    ctx_set_error(c, "serving loop not available");
    return TRIG_EINVAL;
}

int trig_stream_stats_get(trig_ctx *c, trig_stream_stats *out) {
    if (!c || !out) return TRIG_EINVAL;
    *out = trig_stream_stats{};
    return TRIG_OK;
}

}  // extern "C"
