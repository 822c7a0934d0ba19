// Batched entry point and serving loop (placeholder loop over single fields).
#include <hip/hip_runtime.h>

#include "ecc_runtime.h"

namespace ecc {
struct BatchState {};
void destroy_batch_state(ecc_context ctx) {
    delete ctx->batch;
    ctx->batch = nullptr;
}
}  // namespace ecc

using namespace ecc;

extern "C" ecc_status ecc_curves_compute_batch(ecc_context ctx, int32_t n, const ecc_field *fields,
                                               const ecc_curves *curves, void *stream) {
    clear_error();
    if (!ctx) return fail(ECC_ERR_INVALID_ARG, "context is NULL");
    if (n < 0 || (n > 0 && (!fields || !curves))) return fail(ECC_ERR_INVALID_ARG, "bad batch arrays");
    std::vector<FieldInfo> infos(n);
    for (int i = 0; i < n; ++i) {
        ecc_status s = validate_field(&fields[i], &curves[i], &infos[i], false);
        if (s != ECC_OK) return s;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    int e = (int)hipSetDevice(ctx->device);
    if (e) return hip_fail(e, "hipSetDevice");
    ecc_status s = acquire_workspace(ctx, stream);
    if (s != ECC_OK) return s;
    for (int i = 0; i < n && s == ECC_OK; ++i) s = compute_one(ctx, &fields[i], infos[i], &curves[i], stream);
    ecc_status s2 = release_workspace(ctx, stream);
    return s != ECC_OK ? s : s2;
}

extern "C" ecc_status ecc_batch_plan_tune(ecc_context ctx, int32_t n, const ecc_field *fields, void *stream) {
    (void)n; (void)fields; (void)stream;
    if (!ctx) return fail(ECC_ERR_INVALID_ARG, "context is NULL");
    return ECC_OK;
}

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
