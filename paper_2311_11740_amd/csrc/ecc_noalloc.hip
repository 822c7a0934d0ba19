// Allocation-free single-field entry point (ecc_curves_compute_noalloc).
//
// Every device buffer of the single-field path lives in one static device
// array per GPU, `scratch`, laid out as
//   [0, 256)                  merge ticket (kept at zero by the merge kernel)
//   [kOffThr, +256 KiB)       the thresholds, staged from the context's pinned buffer
//   [kOffLut, +128 KiB)       value -> level table of integer fields with thresholds
//   [kOffTotals, ...)         per-level totals, then the atomic drain's accumulators
//                             (or, for the 3D tile kernel, per-workgroup partials)
// Host code never uses the array's name as a device address: set-up reads the
// symbol's address on each device once and every launch takes that pointer.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <unordered_map>

#include "ecc_runtime.h"

namespace ecc {

constexpr size_t kScratchBytes = ECC_NOALLOC_SCRATCH_BYTES;
constexpr size_t kOffThr = 256;
constexpr size_t kOffLut = kOffThr + sizeof(float) * 65536;
constexpr size_t kOffTotals = kOffLut + sizeof(uint16_t) * 65536;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static std::unordered_map<int, unsigned char *> g_scratch;  // device -> address of `scratch` there

// Address of this device's scratch array, looked up (and its merge ticket
// zeroed) on the first call for the device; the device must be current.
ecc_status noalloc_scratch(int device, unsigned char **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch.find(device);
    if (it != g_scratch.end()) {
        *out = it->second;
        return ECC_OK;
    }
    void *p = nullptr;
    int e = (int)hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    e = (int)hipMemset(p, 0, 256);
    if (!e) e = (int)hipDeviceSynchronize();
    if (e) return hip_fail(e, "clearing the scratch ticket");
    g_scratch[device] = (unsigned char *)p;
    *out = (unsigned char *)p;
    return ECC_OK;
}

__global__ void ecc_zero_words(unsigned *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

}  // namespace ecc

using namespace ecc;

extern "C" ecc_status ecc_curves_compute_noalloc(ecc_context ctx, const ecc_field *field, const ecc_curves *curves,
                                                 void *stream) {
    clear_error();
    if (!ctx) return fail(ECC_ERR_INVALID_ARG, "context is NULL");
    FieldInfo fi;
    ecc_status s = validate_field(field, curves, &fi, false);
    if (s != ECC_OK) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    int e = (int)hipSetDevice(ctx->device);
    if (e) return hip_fail(e, "hipSetDevice");
    if (!ctx->scratch) return fail(ECC_ERR_DEVICE, "the context has no scratch array");
    const OnePlan p = plan_one(ctx, fi, curves, field->data);
    const bool use_acc = atomic_drain() && (fi.ndim == 2 || p.zmarch);
    const size_t acc_bytes = (size_t)kAccCopies * p.nch * fi.L * sizeof(int64_t);
    const size_t tot_off = kOffTotals;
    const size_t part_off = (tot_off + p.totals_bytes + 255) & ~size_t(255);
    const size_t need = part_off + (use_acc ? acc_bytes : p.partial_bytes);
    if (need > kScratchBytes)
        return fail(ECC_ERR_UNSUPPORTED,
                    "ecc_curves_compute_noalloc: this field needs " + std::to_string(need) +
                        " bytes of scratch; the allocation-free entry point has " + std::to_string(kScratchBytes));
    unsigned char *base = ctx->scratch;
    hipStream_t st = (hipStream_t)stream;
    s = acquire_workspace(ctx, stream);  // orders this call after the context's other calls (tiny-field buffer)
    if (s != ECC_OK) return s;
    // everything that must start at zero: the merge ticket and the accumulators
    hipLaunchKernelGGL(ecc_zero_words, dim3(1), dim3(64), 0, st, (unsigned *)base, 64);
    e = (int)hipGetLastError();
    if (!e && use_acc) e = launch_zero(base + part_off, acc_bytes, stream);
    if (e) return hip_fail(e, "scratch clear");
    LevelArgs lv;
    lv.L = fi.L;
    lv.mode = LM_IDENTITY;
    lv.thr = nullptr;
    lv.lut = nullptr;
    lv.u0 = 0.f;
    lv.u0d = 0.0;
    lv.inv_step = 0.f;
    lv.eps = 0.f;
    lv.eps_far = 0.f;
    lv.neg = 0u;
    if (field->thresholds || fi.super) {
        // stage through the context's pinned buffer (reused once the previous
        // staging copy has run); superlevel levels as -t (integer identity:
        // t_l = L - 1 - l), which the kernels compare -x against
        e = (int)hipEventSynchronize(ctx->stage_event);
        if (e) return hip_fail(e, "hipEventSynchronize(staging)");
        if (!fi.super)
            std::memcpy(ctx->h_stage, field->thresholds, sizeof(float) * fi.L);
        else if (field->thresholds)
            negate_thresholds(field->thresholds, fi.L, ctx->h_stage);
        else
            for (int l = 0; l < fi.L; ++l) ctx->h_stage[l] = (float)(l - (fi.L - 1));
        lv.neg = fi.super ? 0x80000000u : 0u;
        float *d_thr = (float *)(base + kOffThr);
        e = (int)hipMemcpyAsync(d_thr, ctx->h_stage, sizeof(float) * fi.L, hipMemcpyHostToDevice, st);
        if (!e) e = (int)hipEventRecord(ctx->stage_event, st);
        if (e) return hip_fail(e, "staging the thresholds");
        lv.thr = d_thr;
        if (fi.dtype == ECC_U8 || fi.dtype == ECC_U16) {
            uint16_t *lut = (uint16_t *)(base + kOffLut);
            e = launch_level_lut(d_thr, fi.L, fi.dtype == ECC_U8 ? 256 : 65536, lut, fi.super, stream);
            if (e) return hip_fail(e, "level table kernel");
            lv.mode = LM_LUT;
            lv.lut = lut;
        } else if (AffineFit fit; affine_levels(ctx->h_stage, fi.L, &fit)) {
            lv.mode = LM_AFFINE;
            lv.u0 = fit.u0;
            lv.u0d = fit.u0d;
            lv.inv_step = fit.inv_step;
            lv.eps = fit.eps;
            lv.eps_far = fit.eps_far;
            if (fi.super) lv.inv_step = -lv.inv_step;
        } else {
            lv.mode = LM_SEARCH;
        }
    }
    s = compute_core(ctx, field, fi, curves, lv, p, (int32_t *)(base + part_off), (int64_t *)(base + tot_off),
                     (unsigned *)base, stream, false, use_acc ? (int64_t *)(base + part_off) : nullptr);
    ecc_status s2 = release_workspace(ctx, stream);
    return s != ECC_OK ? s : s2;
}
