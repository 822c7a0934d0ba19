// Serving loop (not built yet).
#include <hip/hip_runtime.h>

#include "ecc_runtime.h"

using namespace ecc;

extern "C" ecc_status ecc_server_create(ecc_context, const ecc_server_config *, ecc_server *) {
    return fail(ECC_ERR_UNSUPPORTED, "serving is not built yet");
}
extern "C" ecc_status ecc_server_submit(ecc_server, const ecc_field *, const ecc_curves *, uint64_t *) {
    return fail(ECC_ERR_UNSUPPORTED, "serving is not built yet");
}
extern "C" ecc_status ecc_server_poll(ecc_server, uint64_t, int32_t *) {
    return fail(ECC_ERR_UNSUPPORTED, "serving is not built yet");
}
extern "C" ecc_status ecc_server_drain(ecc_server) { return fail(ECC_ERR_UNSUPPORTED, "serving is not built yet"); }
extern "C" ecc_status ecc_server_destroy(ecc_server) { return ECC_OK; }
