// Serving loop.  Placeholder until the scheduler lands.
#include "core.hpp"

using namespace dsm;

DSM_API void dsm_server_opts_default(dsm_server_opts *o) {
    if (!o) return;
    o->slots = 64;
    o->hbm_budget = 0;
    o->streams = 4;
    o->small_rows = 40000;
    o->batch_max = 256;
}
DSM_API dsm_status dsm_server_create(dsm_ctx, const dsm_server_opts *, dsm_server *) {
    return guard([&] { fail(DSM_E_UNSUPPORTED, "server not built yet"); });
}
DSM_API dsm_status dsm_server_submit(dsm_server, dsm_matrix, const double *, double *, const dsm_cg_opts *, uint64_t *) {
    return guard([&] { fail(DSM_E_UNSUPPORTED, "server not built yet"); });
}
DSM_API dsm_status dsm_server_poll(dsm_server, uint64_t, dsm_cg_result *, dsm_timestamps *) {
    return guard([&] { fail(DSM_E_UNSUPPORTED, "server not built yet"); });
}
DSM_API dsm_status dsm_server_wait(dsm_server, uint64_t, dsm_cg_result *, dsm_timestamps *) {
    return guard([&] { fail(DSM_E_UNSUPPORTED, "server not built yet"); });
}
DSM_API double dsm_server_now(dsm_server) { return 0.0; }
DSM_API dsm_status dsm_server_destroy(dsm_server) {
    return guard([&] { fail(DSM_E_UNSUPPORTED, "server not built yet"); });
}
