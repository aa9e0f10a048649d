// Entry points declared in rplu.h that are not built yet.
#include "rplu.h"
#include "runtime.hpp"

extern "C" {
rplu_status rplu_server_create(rplu_ctx, const rplu_server_cfg*, rplu_server* out) {
    if (out) *out = nullptr;
    return rplu::fail(RPLU_E_UNSUPPORTED, "rplu_server: not available in this build");
}
rplu_status rplu_server_submit(rplu_server, const rplu_job*, uint64_t*) {
    return rplu::fail(RPLU_E_UNSUPPORTED, "rplu_server: not available in this build");
}
rplu_status rplu_server_poll(rplu_server, uint64_t, rplu_info*) {
    return rplu::fail(RPLU_E_UNSUPPORTED, "rplu_server: not available in this build");
}
rplu_status rplu_server_stats(rplu_server, rplu_server_stats_t*) {
    return rplu::fail(RPLU_E_UNSUPPORTED, "rplu_server: not available in this build");
}
rplu_status rplu_server_destroy(rplu_server) { return RPLU_OK; }
}
