// Batched and served forms of the CDUGKS library (see include/cdugks.h).
#include "cdugks.h"
#include "cdugks_host.h"

using namespace cdg;

extern "C" {

int cdugks_batch_create(cdugks_ctx* const*, int, int, cdugks_batch** out) {
    if (out) *out = nullptr;
    return fail(CDUGKS_ERR_UNKNOWN, "batched form not built yet");
}
int cdugks_batch_step(cdugks_batch*, int64_t) { return fail(CDUGKS_ERR_UNKNOWN, "batched form not built yet"); }
void cdugks_batch_destroy(cdugks_batch*) {}

int cdugks_server_create(size_t, int, int, void*, cdugks_server** out) {
    if (out) *out = nullptr;
    return fail(CDUGKS_ERR_UNKNOWN, "served form not built yet");
}
int cdugks_submit(cdugks_server*, const cdugks_space*, const cdugks_velocity*, const cdugks_params*,
                  const double*, const double*, const double*, int64_t, uint64_t*) {
    return fail(CDUGKS_ERR_UNKNOWN, "served form not built yet");
}
int cdugks_poll(cdugks_server*, uint64_t, double*, double*, double*, double*, double*) {
    return fail(CDUGKS_ERR_UNKNOWN, "served form not built yet");
}
void cdugks_server_destroy(cdugks_server*) {}

}  // extern "C"
