// Serving loop of libcrb (continuous, iteration-level batching).  Placeholder
// until the batched path is verified: every call reports that serving is absent.
#include "api_internal.h"

extern "C" {
crb_status crb_server_create(size_t, int32_t, crb_server **out) {
    if (out)
        *out = nullptr;
    return crb::fail(CRB_EDEVICE, "serving is not built yet");
}
crb_status crb_server_submit(crb_server *, const float *, int32_t, int32_t, float, float, float,
                             float, float, float, int32_t, float *, uint8_t *, int64_t *) {
    return crb::fail(CRB_EDEVICE, "serving is not built yet");
}
crb_status crb_server_poll(crb_server *, int64_t *, double *, int32_t, int32_t *) {
    return crb::fail(CRB_EDEVICE, "serving is not built yet");
}
int32_t crb_server_pending(crb_server *) { return 0; }
void crb_server_destroy(crb_server *) {}
}
