// Placeholder translation unit for the batch and serving entry points.
#include "internal.h"

using namespace tpt;

extern "C" {
int tpt_batch_create(int, const tpt_plan*, tpt_batch*) { return fail(TPT_ERR_UNSUPPORTED, "not built yet"); }
int tpt_batch_destroy(tpt_batch) { return TPT_OK; }
int tpt_batch_workspace_bytes(tpt_batch, size_t*) { return fail(TPT_ERR_UNSUPPORTED, "not built yet"); }
int tpt_batch_solve(tpt_batch, const double* const*, double* const*, void*, size_t, void*, int) {
    return fail(TPT_ERR_UNSUPPORTED, "not built yet");
}
int tpt_autotune(int, const tpt_plan*, void*) { return fail(TPT_ERR_UNSUPPORTED, "not built yet"); }
int tpt_server_create(size_t, int, tpt_server*) { return fail(TPT_ERR_UNSUPPORTED, "not built yet"); }
int tpt_server_submit(tpt_server, tpt_plan, const double*, double*, unsigned long long*) {
    return fail(TPT_ERR_UNSUPPORTED, "not built yet");
}
int tpt_server_poll(tpt_server, unsigned long long, tpt_info*, double*, double*, double*) {
    return fail(TPT_ERR_UNSUPPORTED, "not built yet");
}
int tpt_server_drain(tpt_server) { return fail(TPT_ERR_UNSUPPORTED, "not built yet"); }
int tpt_server_destroy(tpt_server) { return TPT_OK; }
}
