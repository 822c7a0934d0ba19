// Host runtime of libecc: context, validation, threshold cache, workspace and
// the single-field entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ecc_runtime.h"

namespace ecc {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

ecc_status fail(ecc_status s, const std::string &msg) {
    g_err = msg;
    return s;
}
void clear_error() { g_err.clear(); }

ecc_status hip_fail(int err, const char *what) {
    return fail(ECC_ERR_DEVICE,
                std::string(what) + ": " + hipGetErrorString((hipError_t)err));
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
ecc_status validate_field(const ecc_field *f, const ecc_curves *c, FieldInfo *info,
                          bool curves_on_host) {
    if (!f) return fail(ECC_ERR_INVALID_ARG, "field is NULL");
    if (!c) return fail(ECC_ERR_INVALID_ARG, "curves is NULL");
    if (f->ndim != 2 && f->ndim != 3) return fail(ECC_ERR_INVALID_ARG, "ndim must be 2 or 3");
    if (f->dtype != ECC_U8 && f->dtype != ECC_U16 && f->dtype != ECC_F32)
        return fail(ECC_ERR_INVALID_ARG, "dtype must be ECC_U8, ECC_U16 or ECC_F32");
    for (int k = 0; k < f->ndim; ++k)
        if (f->shape[k] < 1) return fail(ECC_ERR_INVALID_ARG, "every shape entry must be >= 1");
    if (!f->data) return fail(ECC_ERR_INVALID_ARG, "field data is NULL");
    if (f->n_levels < 1) return fail(ECC_ERR_INVALID_ARG, "n_levels must be >= 1");
    if (f->n_levels > kMaxLevels)
        return fail(ECC_ERR_UNSUPPORTED, "n_levels above 65535 is not supported");
    int conn = f->connectivity;
    if (conn == 0) conn = f->ndim == 2 ? 8 : 26;
    if (f->ndim == 2 && conn != 8 && conn != 4)
        return fail(ECC_ERR_INVALID_ARG, "2D connectivity must be 8 or 4");
    if (f->ndim == 3 && conn != 26 && conn != 6)
        return fail(ECC_ERR_INVALID_ARG, "3D connectivity must be 26 or 6");
    if (f->filtration != ECC_SUBLEVEL && f->filtration != ECC_SUPERLEVEL)
        return fail(ECC_ERR_INVALID_ARG, "filtration must be ECC_SUBLEVEL or ECC_SUPERLEVEL");
    const bool super = f->filtration == ECC_SUPERLEVEL;
    if (f->dtype == ECC_F32 && !f->thresholds)
        return fail(ECC_ERR_INVALID_ARG, "float32 fields need a thresholds array");
    if (f->thresholds) {
        for (int l = 0; l < f->n_levels; ++l) {
            if (std::isnan(f->thresholds[l]))
                return fail(ECC_ERR_INVALID_ARG, "thresholds must not be NaN");
            if (l > 0 && !super && f->thresholds[l] < f->thresholds[l - 1])
                return fail(ECC_ERR_INVALID_ARG, "thresholds must be non-decreasing");
            if (l > 0 && super && f->thresholds[l] > f->thresholds[l - 1])
                return fail(ECC_ERR_INVALID_ARG, "superlevel thresholds must be non-increasing");
        }
    }
    if (f->ndim == 2 && c->volume) return fail(ECC_ERR_INVALID_ARG, "volume must be NULL for 2D fields");
    if (!c->ec && !c->perimeter && !c->area && !c->volume)
        return fail(ECC_ERR_INVALID_ARG, "no output curve requested");
    for (int k = 0; k < f->ndim; ++k)
        if (f->shape[k] >= (int64_t(1) << 31)) return fail(ECC_ERR_UNSUPPORTED, "a dimension of 2^31 or more");
    int64_t cells = 1;
    for (int k = 0; k < f->ndim; ++k) {
        if (f->shape[k] > (int64_t(1) << 40) / cells)
            return fail(ECC_ERR_UNSUPPORTED, "more than 2^40 cells");
        cells *= f->shape[k];
    }
    (void)curves_on_host;
    info->ndim = f->ndim;
    info->dtype = f->dtype;
    info->d = f->ndim == 3 ? f->shape[0] : 1;
    info->h = f->shape[f->ndim - 2];
    info->w = f->shape[f->ndim - 1];
    info->cells = cells;
    info->L = f->n_levels;
    info->conn = conn;
    info->elem_bytes = f->dtype == ECC_U8 ? 1 : (f->dtype == ECC_U16 ? 2 : 4);
    info->super = super;
    return ECC_OK;
}

const float *field_thresholds(const ecc_field *f, std::vector<float> &tmp) {
    if (f->thresholds || f->filtration != ECC_SUPERLEVEL) return f->thresholds;
    const int L = f->n_levels;
    tmp.resize(L);
    for (int l = 0; l < L; ++l) tmp[l] = (float)(L - 1 - l);
    return tmp.data();
}

void negate_thresholds(const float *t, int L, float *dst) {
    for (int l = 0; l < L; ++l) dst[l] = -t[l];
}

}  // namespace ecc

using namespace ecc;

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
static ecc_status upload(void **dst, const void *src, size_t bytes) {
    int e = (int)hipMalloc(dst, bytes);
    if (e) return hip_fail(e, "hipMalloc(table)");
    e = (int)hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    if (e) return hip_fail(e, "hipMemcpy(table)");
    return ECC_OK;
}

extern "C" ecc_status ecc_create(int device, ecc_context *out) {
    clear_error();
    if (!out) return fail(ECC_ERR_INVALID_ARG, "ecc_create: out is NULL");
    *out = nullptr;
    int ndev = 0;
    int e = (int)hipGetDeviceCount(&ndev);
    if (e) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(ECC_ERR_INVALID_ARG, "ecc_create: no such device");
    e = (int)hipSetDevice(device);
    if (e) return hip_fail(e, "hipSetDevice");
    hipDeviceProp_t prop;
    e = (int)hipGetDeviceProperties(&prop, device);
    if (e) return hip_fail(e, "hipGetDeviceProperties");
    auto *ctx = new ecc_context_s();
    ctx->device = device;
    ctx->n_cu = prop.multiProcessorCount;
    ctx->max_lds = prop.sharedMemPerBlock;
    ctx->arch = prop.gcnArchName;
    // per-cell delta tables (2D) and per-vertex tables (3D)
    for (int k = 0; k < 2; ++k) {
        const int conn2 = k == 0 ? 8 : 4;
        int32_t dt[256][3];
        cell_delta_table_2d(conn2, dt);
        uint64_t packed[256];  // in the 2D kernels' index order
        for (int n = 0; n < 256; ++n) {
            const int p = pattern_of_index(n ^ kNorthFlip2D);
            packed[n] = (uint64_t)(dt[p][0] + kEcBias2) |
                        (uint64_t)(dt[p][1] + kPerBias2) << kShiftPer2 | 1ull << kShiftCnt2;
        }
        ecc_status s = upload((void **)&ctx->d_delta2[k], packed, sizeof(packed));
        if (s != ECC_OK) {
            ecc_destroy(ctx);
            return s;
        }
        std::memcpy(ctx->h_delta2[k], dt, sizeof(dt));
        const int conn3 = k == 0 ? 26 : 6;
        int32_t vt[256][4];
        vertex_table_3d(conn3, vt);
        int64_t vp[256];
        for (int m = 0; m < 256; ++m)  // four 16-bit fields, every channel scaled by 8
            vp[m] = (int64_t)vt[m][0] + (int64_t)(vt[m][1] * 4) * 65536 +
                    (int64_t)(vt[m][2] * 2) * 4294967296LL + (int64_t)vt[m][3] * 281474976710656LL;
        s = upload((void **)&ctx->d_vtab3[k], vp, sizeof(vp));
        if (s != ECC_OK) {
            ecc_destroy(ctx);
            return s;
        }
        // z-marching tables from the 2D per-cell EC deltas of the same pattern
        // (8-C for the 26-C volume, 4-C for 6-C): [0, 256) the layer term with
        // the 2D perimeter delta (4 minus 2 per edge neighbour in) and the
        // biases, [256, 512) the image delta, signs as the decomposition takes
        // them; the constant two surface units of the vertical neighbours'
        // term sit in the layer term (min image) or the image term (max image)
        uint32_t zt[512];
        const int sgn = k == 0 ? -1 : 1;
        const uint32_t two_faces = 2u << kShiftSurf3;
        for (int n = 0; n < 256; ++n) {  // in the kernels' index order, north bit complemented
            const int p = pattern_of_index(n ^ kNorthFlip2D);
            const int per = 4 - 2 * __builtin_popcount(p & 0x5A);  // N, W, E, S bits
            zt[n] = (uint32_t)(sgn * dt[p][0] + kEcBias3) + ((uint32_t)(per + 8) << kShiftSurf3) -
                    (k == 0 ? two_faces : 0u);
            zt[256 + n] = (uint32_t)(-sgn * dt[p][0]) - (k == 1 ? two_faces : 0u);
        }
        s = upload((void **)&ctx->d_zm3[k], zt, sizeof(zt));
        if (s != ECC_OK) {
            ecc_destroy(ctx);
            return s;
        }
    }
    {
        // class-count deltas, two words per pattern in the 2D kernels' index order
        int32_t ct[256][5];
        class_delta_table_2d(ct);
        uint64_t packed[512];
        for (int n = 0; n < 256; ++n) {
            const int p = pattern_of_index(n ^ kNorthFlip2D);
            packed[n] = (uint64_t)(ct[p][0] + kClsBias) | (uint64_t)(ct[p][1] + kClsBias) << kClsShift1 |
                        1ull << kClsShift2;
            packed[256 + n] = (uint64_t)(ct[p][2] + kClsBias) | (uint64_t)(ct[p][3] + kClsBias) << kClsShift1 |
                              (uint64_t)ct[p][4] << kClsShift2;
        }
        ecc_status s = upload((void **)&ctx->d_cls2, packed, sizeof(packed));
        if (s != ECC_OK) {
            ecc_destroy(ctx);
            return s;
        }
        uint16_t t3[8][256];  // 3D class transitions of the corners of an entering voxel
        class_transitions_3d(t3);
        s = upload((void **)&ctx->d_trans3, t3, sizeof(t3));
        if (s != ECC_OK) {
            ecc_destroy(ctx);
            return s;
        }
        // per-plane crease deltas + 4, in the kernels' index order: [0, 256)
        // for the yz and xz plane patterns, [256, 512) with the north bit
        // complemented for the layer pattern
        int32_t cd[256];
        crease_delta_table_2d(cd);
        uint32_t tc[512];
        for (int n = 0; n < 256; ++n) {
            tc[n] = (uint32_t)(cd[pattern_of_index(n)] + 4);
            tc[256 + n] = (uint32_t)(cd[pattern_of_index(n ^ kNorthFlip2D)] + 4);
        }
        s = upload((void **)&ctx->d_crease3, tc, sizeof(tc));
        if (s != ECC_OK) {
            ecc_destroy(ctx);
            return s;
        }
    }
    e = (int)hipEventCreateWithFlags(&ctx->ws_event, hipEventDisableTiming);
    if (e) {
        ecc_destroy(ctx);
        return hip_fail(e, "hipEventCreate");
    }
    // the merge kernel's completion ticket, zeroed here once and for all (the
    // kernel leaves it at zero): zeroing it lazily on the null stream would not
    // order the clear before a first merge queued on a non-blocking stream
    e = (int)hipMalloc(&ctx->d_counter, 256);
    if (e) {
        ecc_destroy(ctx);
        return fail(ECC_ERR_OUT_OF_MEMORY, "hipMalloc(counter) failed");
    }
    e = (int)hipMemset(ctx->d_counter, 0, 256);
    if (!e) e = (int)hipHostMalloc(&ctx->h_stage, sizeof(float) * 65536, 0);
    if (!e) e = (int)hipEventCreateWithFlags(&ctx->stage_event, hipEventDisableTiming);
    if (!e) e = (int)hipMalloc(&ctx->d_tiny, 256);
    if (!e) e = (int)hipMemset(ctx->d_tiny, 0, 256);
    if (!e) e = (int)hipDeviceSynchronize();
    if (e) {
        ecc_destroy(ctx);
        return hip_fail(e, "hipMemset(counter)");
    }
    // the allocation-free entry point's scratch array on this device
    ecc_status ss = noalloc_scratch(device, &ctx->scratch);
    if (ss != ECC_OK) {
        ecc_destroy(ctx);
        return ss;
    }
    *out = ctx;
    return ECC_OK;
}

extern "C" ecc_status ecc_destroy(ecc_context ctx) {
    clear_error();
    if (!ctx) return ECC_OK;
    hipSetDevice(ctx->device);
    hipDeviceSynchronize();
    for (int k = 0; k < 2; ++k) {
        if (ctx->d_delta2[k]) hipFree(ctx->d_delta2[k]);
        if (ctx->d_vtab3[k]) hipFree(ctx->d_vtab3[k]);
        if (ctx->d_zm3[k]) hipFree(ctx->d_zm3[k]);
    }
    if (ctx->d_cls2) hipFree(ctx->d_cls2);
    if (ctx->d_trans3) hipFree(ctx->d_trans3);
    if (ctx->d_crease3) hipFree(ctx->d_crease3);
    for (auto *t : ctx->thr_cache) free_thresholds(t);
    ctx->thr_cache.clear();
    for (auto &pe : ctx->prof_events) {
        hipEventDestroy(pe.first);
        hipEventDestroy(pe.second);
    }
    ctx->ws.release();
    if (ctx->d_counter) hipFree(ctx->d_counter);
    if (ctx->d_tiny) hipFree(ctx->d_tiny);
    if (ctx->h_stage) hipHostFree(ctx->h_stage);
    if (ctx->stage_event) hipEventDestroy(ctx->stage_event);
    if (ctx->ws_event) hipEventDestroy(ctx->ws_event);
    destroy_batch_state(ctx);
    destroy_stream_state(ctx);
    delete ctx;
    return ECC_OK;
}

extern "C" const char *ecc_last_error(void) { return g_err.c_str(); }

extern "C" const char *ecc_status_string(ecc_status s) {
    switch (s) {
    case ECC_OK: return "ECC_OK";
    case ECC_ERR_INVALID_ARG: return "ECC_ERR_INVALID_ARG";
    case ECC_ERR_UNSUPPORTED: return "ECC_ERR_UNSUPPORTED";
    case ECC_ERR_OUT_OF_MEMORY: return "ECC_ERR_OUT_OF_MEMORY";
    case ECC_ERR_DEVICE: return "ECC_ERR_DEVICE";
    case ECC_ERR_BUSY: return "ECC_ERR_BUSY";
    }
    return "unknown status";
}

namespace ecc {

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
void DevBuf::release() {
    if (ptr) hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

ecc_status DevBuf::ensure(size_t need, const char *what) {
    if (need <= bytes) return ECC_OK;
    release();
    size_t cap = std::max(need, (size_t)1 << 20);
    int e = (int)hipMalloc(&ptr, cap);
    if (e) {
        ptr = nullptr;
        return fail(ECC_ERR_OUT_OF_MEMORY, std::string("hipMalloc(") + what + ") failed");
    }
    bytes = cap;
    return ECC_OK;
}

// ---------------------------------------------------------------------------
// thresholds: device copies cached by content
// ---------------------------------------------------------------------------
void free_thresholds(ThrEntry *t) {
    if (t->d_thr) hipFree(t->d_thr);
    if (t->d_lut8) hipFree(t->d_lut8);
    if (t->d_lut16) hipFree(t->d_lut16);
    if (t->h_pinned) hipHostFree(t->h_pinned);
    if (t->ready) hipEventDestroy(t->ready);
    if (t->last_use) hipEventDestroy(t->last_use);
    delete t;
}

static bool same_thresholds(const ThrEntry *t, const float *thr, int L, bool neg) {
    return t->L == L && t->neg == neg && std::memcmp(t->host.data(), thr, sizeof(float) * L) == 0;
}

static ThrEntry *find_thresholds(ecc_context ctx, const float *thr, int L, bool neg) {
    for (auto *t : ctx->thr_cache)
        if (same_thresholds(t, thr, L, neg)) return t;
    return nullptr;
}

// Frees the least recently fetched entry outside `keep`, preferring one that
// no queued work reads any more; otherwise waits for the latest work that
// reads it (never for the whole device).
static ecc_status evict_threshold(ecc_context ctx, const std::vector<const ThrEntry *> &keep, void *stream) {
    ecc_status s = use_stream(ctx, stream);
    if (s != ECC_OK) return s;
    auto kept = [&keep](const ThrEntry *t) { return std::find(keep.begin(), keep.end(), t) != keep.end(); };
    auto idle = [](const ThrEntry *t) {
        return (!t->used || hipEventQuery(t->last_use) == hipSuccess) && hipEventQuery(t->ready) == hipSuccess;
    };
    int victim = -1;
    for (int pass = 0; pass < 2 && victim < 0; ++pass)
        for (int i = 0; i < (int)ctx->thr_cache.size(); ++i) {
            ThrEntry *t = ctx->thr_cache[i];
            if (kept(t) || (pass == 0 && !idle(t))) continue;
            if (victim < 0 || t->tick < ctx->thr_cache[victim]->tick) victim = i;
        }
    if (victim < 0) return fail(ECC_ERR_UNSUPPORTED, "threshold cache: nothing to evict");
    ThrEntry *t = ctx->thr_cache[victim];
    int e;
    if (ctx->one_stream) {  // every use of the victim was queued on this one stream
        e = (int)hipStreamSynchronize((hipStream_t)stream);
    } else {
        e = (int)hipEventSynchronize(t->ready);
        if (!e && t->used) e = (int)hipEventSynchronize(t->last_use);
    }
    if (e) return hip_fail(e, "hipEventSynchronize(thresholds)");
    free_thresholds(t);
    ctx->thr_cache.erase(ctx->thr_cache.begin() + victim);
    return ECC_OK;
}

ecc_status get_thresholds(ecc_context ctx, const float *thr, int L, bool neg, int dtype, void *stream,
                          const ThrEntry **out) {
    ThrEntry *hit = find_thresholds(ctx, thr, L, neg);
    hipStream_t st = (hipStream_t)stream;
    if (!hit) {
        if (ctx->thr_cache.size() >= kThrCacheMax) {
            ecc_status s = evict_threshold(ctx, {}, stream);
            if (s != ECC_OK) return s;
        }
        auto *t = new ThrEntry();
        t->L = L;
        t->neg = neg;
        t->host.assign(thr, thr + L);
        int e = (int)hipEventCreateWithFlags(&t->ready, hipEventDisableTiming);
        if (!e) e = (int)hipEventCreateWithFlags(&t->last_use, hipEventDisableTiming);
        if (!e) e = (int)hipHostMalloc(&t->h_pinned, sizeof(float) * L, 0);
        if (e) {
            free_thresholds(t);
            return hip_fail(e, "threshold cache entry");
        }
        if (neg)
            negate_thresholds(thr, L, t->h_pinned);
        else
            std::memcpy(t->h_pinned, thr, sizeof(float) * L);
        e = (int)hipMalloc(&t->d_thr, sizeof(float) * L);
        if (e) {
            free_thresholds(t);
            return fail(ECC_ERR_OUT_OF_MEMORY, "hipMalloc(thresholds) failed");
        }
        e = (int)hipMemcpyAsync(t->d_thr, t->h_pinned, sizeof(float) * L, hipMemcpyHostToDevice, st);
        if (!e) e = (int)hipEventRecord(t->ready, st);
        if (e) {
            free_thresholds(t);
            return hip_fail(e, "hipMemcpyAsync(thresholds)");
        }
        t->ready_stream = stream;
        AffineFit fit;
        t->affine = affine_levels(t->h_pinned, L, &fit);
        t->u0 = fit.u0;
        t->u0d = fit.u0d;
        t->inv_step = fit.inv_step;
        t->eps = fit.eps;
        t->eps_far = fit.eps_far;
        ctx->thr_cache.push_back(t);
        hit = t;
    } else if (hit->ready_stream != stream) {
        // the upload (or a level table) was queued on another stream
        int e = (int)hipStreamWaitEvent(st, hit->ready, 0);
        if (e) return hip_fail(e, "hipStreamWaitEvent(thresholds)");
    }
    hit->tick = ++ctx->thr_tick;
    // integer fields with thresholds: value -> level table, built once on the device
    const bool need8 = dtype == ECC_U8 && !hit->d_lut8, need16 = dtype == ECC_U16 && !hit->d_lut16;
    if (need8 || need16) {
        uint16_t **dst = need8 ? &hit->d_lut8 : &hit->d_lut16;
        const int nv = need8 ? 256 : 65536;
        int e = (int)hipMalloc(dst, nv * sizeof(uint16_t));
        if (e) {
            *dst = nullptr;
            return fail(ECC_ERR_OUT_OF_MEMORY, "hipMalloc(level table) failed");
        }
        e = launch_level_lut(hit->d_thr, L, nv, *dst, hit->neg, stream);
        if (!e) e = (int)hipEventRecord(hit->ready, st);
        if (e) return hip_fail(e, "level table kernel");
        hit->ready_stream = stream;
    }
    *out = hit;
    return ECC_OK;
}

// Distinct threshold arrays among `fields` (integer superlevel fields without
// thresholds count by their level count; such a field and one whose caller
// array has the same content count twice, which only overestimates).
static int count_distinct(int n, const ecc_field *const *fields, ecc_context ctx, bool uncached_only) {
    int k = 0;
    std::vector<float> tmp;
    for (int i = 0; i < n; ++i) {
        const ecc_field *f = fields[i];
        const bool neg = f->filtration == ECC_SUPERLEVEL;
        if (!f->thresholds && !neg) continue;
        bool seen = false;
        for (int j = 0; j < i && !seen; ++j) {
            const ecc_field *g = fields[j];
            if (g->n_levels != f->n_levels || (g->filtration == ECC_SUPERLEVEL) != neg) continue;
            if (!f->thresholds || !g->thresholds)
                seen = !f->thresholds && !g->thresholds;
            else
                seen = g->thresholds == f->thresholds ||
                       std::memcmp(g->thresholds, f->thresholds, sizeof(float) * f->n_levels) == 0;
        }
        if (seen) continue;
        if (uncached_only && ctx && find_thresholds(ctx, field_thresholds(f, tmp), f->n_levels, neg)) continue;
        ++k;
    }
    return k;
}

int count_distinct_thresholds(int n, const ecc_field *const *fields) {
    return count_distinct(n, fields, nullptr, false);
}

ecc_status reserve_thresholds(ecc_context ctx, int n, const ecc_field *const *fields, void *stream) {
    if (count_distinct(n, fields, nullptr, false) > (int)kThrCacheMax)
        return fail(ECC_ERR_UNSUPPORTED, "one call may use at most 256 distinct threshold arrays");
    const int n_new = count_distinct(n, fields, ctx, true);
    std::vector<const ThrEntry *> keep;  // the arrays of this call that are cached already
    std::vector<float> tmp;
    for (int i = 0; i < n; ++i)
        if (const float *a = field_thresholds(fields[i], tmp))
            if (const ThrEntry *t =
                    find_thresholds(ctx, a, fields[i]->n_levels, fields[i]->filtration == ECC_SUPERLEVEL))
                keep.push_back(t);
    while (ctx->thr_cache.size() + (size_t)n_new > kThrCacheMax) {
        ecc_status s = evict_threshold(ctx, keep, stream);
        if (s != ECC_OK) return s;
    }
    return ECC_OK;
}

ecc_status note_threshold_use(ecc_context ctx, const LevelArgs &lv, void *stream) {
    if (!lv.thr) return ECC_OK;
    ecc_status s = use_stream(ctx, stream);
    if (s != ECC_OK || ctx->one_stream) return s;  // one stream: its order covers the use
    for (auto *t : ctx->thr_cache)
        if (t->d_thr == lv.thr) {
            int e = (int)hipEventRecord(t->last_use, (hipStream_t)stream);
            if (e) return hip_fail(e, "hipEventRecord(thresholds)");
            t->used = true;
            return ECC_OK;
        }
    return ECC_OK;
}

ecc_status level_args(ecc_context ctx, const ecc_field *f, const FieldInfo &fi, void *stream,
                      LevelArgs *lv) {
    lv->L = fi.L;
    lv->thr = nullptr;
    lv->lut = nullptr;
    lv->u0 = 0.f;
    lv->u0d = 0.0;
    lv->inv_step = 0.f;
    lv->eps = 0.f;
    lv->eps_far = 0.f;
    lv->neg = 0u;
    std::vector<float> tmp;
    const float *thr = field_thresholds(f, tmp);
    if (!thr) {
        lv->mode = LM_IDENTITY;
        return ECC_OK;
    }
    const ThrEntry *te = nullptr;
    ecc_status s = get_thresholds(ctx, thr, fi.L, fi.super, fi.dtype, stream, &te);
    if (s != ECC_OK) return s;
    lv->thr = te->d_thr;
    // superlevel: the device thresholds are -t and the kernels compare -x
    // against them; the affine estimate takes the sign in its slope
    lv->neg = fi.super ? 0x80000000u : 0u;
    if (fi.dtype == ECC_U8) {
        lv->mode = LM_LUT;
        lv->lut = te->d_lut8;
    } else if (fi.dtype == ECC_U16) {
        lv->mode = LM_LUT;
        lv->lut = te->d_lut16;
    } else if (te->affine) {
        lv->mode = LM_AFFINE;
        lv->u0 = te->u0;
        lv->u0d = te->u0d;
        lv->inv_step = fi.super ? -te->inv_step : te->inv_step;
        lv->eps = te->eps;
        lv->eps_far = te->eps_far;
    } else {
        lv->mode = LM_SEARCH;
    }
    return ECC_OK;
}

// order work on `stream` after the previous use of the context's workspace
ecc_status use_stream(ecc_context ctx, void *stream) {
    if (!ctx->one_stream) return ECC_OK;
    if (!ctx->solo_set) {
        ctx->solo_set = true;
        ctx->solo_stream = stream;
        return ECC_OK;
    }
    if (stream == ctx->solo_stream) return ECC_OK;
    // a second stream: everything queued so far (on the one stream) completes
    // here, so no earlier use needs an event
    int e = (int)hipDeviceSynchronize();
    if (e) return hip_fail(e, "hipDeviceSynchronize");
    ctx->one_stream = false;
    ctx->ws_used = false;
    for (auto *t : ctx->thr_cache) t->used = false;
    return ECC_OK;
}

ecc_status acquire_workspace(ecc_context ctx, void *stream) {
    ecc_status s = use_stream(ctx, stream);
    if (s != ECC_OK) return s;
    if (ctx->ws_used && ctx->ws_stream != stream) {
        int e = (int)hipStreamWaitEvent((hipStream_t)stream, ctx->ws_event, 0);
        if (e) return hip_fail(e, "hipStreamWaitEvent");
    }
    return ECC_OK;
}

ecc_status release_workspace(ecc_context ctx, void *stream) {
    if (!ctx->one_stream) {
        int e = (int)hipEventRecord(ctx->ws_event, (hipStream_t)stream);
        if (e) return hip_fail(e, "hipEventRecord");
    }
    ctx->ws_used = true;
    ctx->ws_stream = stream;
    return ECC_OK;
}

// grow a workspace buffer; the old one may still be read by queued work
ecc_status grow(ecc_context ctx, DevBuf &b, size_t need, const char *what) {
    if (need <= b.bytes) return ECC_OK;
    // the old buffer may still be in use by work queued on any stream (earlier
    // fields of the same call included): wait for the device before freeing it
    (void)ctx;
    int e = (int)hipDeviceSynchronize();
    if (e) return hip_fail(e, "hipDeviceSynchronize");
    return b.ensure(need, what);
}

int pick_grid(ecc_context ctx, int64_t n_tiles, size_t lds_per_wg) {
    const size_t lds_cu = 160 * 1024;
    int per_cu = (int)std::min<size_t>(4, std::max<size_t>(1, lds_cu / std::max<size_t>(lds_per_wg, 1)));
    int64_t g = (int64_t)ctx->n_cu * per_cu;
    if (g > n_tiles) g = n_tiles;
    if (g >= 8) g -= g % 8;
    return (int)std::max<int64_t>(1, g);
}

bool atomic_drain() {
    static bool v = [] {
        const char *e = std::getenv("ECC_DRAIN");
        return !(e && std::strcmp(e, "partials") == 0);
    }();
    return v;
}

bool progress_prio() {
    static bool v = [] {
        const char *e = std::getenv("ECC_PRIO");
        return !(e && std::strcmp(e, "0") == 0);
    }();
    return v;
}

// Workgroups per CU for the z-marching 3D kernel: as many 4-wave workgroups
// as its register use lets share a CU (three for integer fields at aligned
// addresses without the crease channel, else two); environment
// ECC_ZM_WG_PER_CU overrides.  `data` NULL stands for an aligned address.
int zm_wg_per_cu(int dtype, int64_t w, const void *data, bool crease) {
    static int env = [] {
        const char *e = std::getenv("ECC_ZM_WG_PER_CU");
        if (!e) return 0;
        int x = std::atoi(e);
        return x < 1 ? 1 : (x > 8 ? 8 : x);
    }();
    if (env) return env;
    const int eb = dtype == ECC_U8 ? 1 : (dtype == ECC_U16 ? 2 : 4);
    const int vb = 4 * eb;  // bytes of one lane's block
    const bool aligned = (uintptr_t)data % vb == 0 && (w * eb) % vb == 0;
    return (!crease && eb < 4 && aligned) ? 3 : 2;
}

ecc_status merge_and_scan(ecc_context ctx, int grid, int nch, int L, int64_t *const outs[4],
                          void *stream) {
    ecc_status s = grow(ctx, ctx->ws.totals, (size_t)nch * L * sizeof(int64_t), "totals");
    if (s != ECC_OK) return s;
    int e = launch_merge((const int32_t *)ctx->ws.partial.ptr, grid, nch, L, outs,
                         (int64_t *)ctx->ws.totals.ptr, (unsigned *)ctx->d_counter, stream);
    if (e) return hip_fail(e, "merge kernel launch");
    return ECC_OK;
}

ecc_status acc_buffer(ecc_context ctx, int nch, int L, int64_t **acc, void *stream) {
    const size_t bytes = (size_t)kAccCopies * nch * L * sizeof(int64_t);
    if (ctx->ws.acc.bytes < bytes) {
        ecc_status s = grow(ctx, ctx->ws.acc, bytes, "accumulators");
        if (s != ECC_OK) return s;
        const int e = (int)hipMemset(ctx->ws.acc.ptr, 0, ctx->ws.acc.bytes);  // the merges keep them at zero
        if (e) return hip_fail(e, "hipMemset(accumulators)");
        ctx->acc_dirty = false;
    }
    if (ctx->acc_dirty) {
        const int e = launch_zero(ctx->ws.acc.ptr, ctx->ws.acc.bytes, stream);
        if (e) return hip_fail(e, "clearing the accumulators");
        ctx->acc_dirty = false;
    }
    *acc = (int64_t *)ctx->ws.acc.ptr;
    return ECC_OK;
}

// Workgroups of the 2D stream kernel (kWaves2D waves each): one per CU, and
// at most one per 4 (strip, row) units per wave of the field, so that fields
// of a few million cells still spread over every CU.  (Its bins of at most
// kMaxWindow levels plus thresholds and tables take under 90 KB of a CU's
// 160 KB of LDS.)
int grid_2d(ecc_context ctx, const FieldInfo &fi, int window, bool classes) {
    (void)window;
    (void)classes;
    const int vec = vec_2d(fi.dtype);
    const int64_t strips = (fi.w + 62 * vec - 1) / (62 * vec);
    int grid = (int)std::min<int64_t>((int64_t)ctx->n_cu,
                                      std::max<int64_t>(1, (strips * fi.h + 4 * kWaves2D - 1) / (4 * kWaves2D)));
    if (grid >= 8) grid -= grid % 8;
    return grid;
}

// Launch geometry of one field on the single-field path.
OnePlan plan_one(ecc_context ctx, const FieldInfo &fi, const ecc_curves *c, const void *data) {
    OnePlan p;
    const int L = fi.L;
    p.nch = fi.ndim == 2 ? 3 : 4;
    p.win = std::min(L, kMaxWindow);
    p.crease = fi.ndim == 3 && c->perimeter != nullptr;
    p.k = (fi.ndim == 2 ? (fi.conn == 8 ? 0 : 1) : (fi.conn == 26 ? 0 : 1));
    p.grid = 1;
    p.zmarch = false;
    if (fi.ndim == 2) {
        p.grid = grid_2d(ctx, fi, p.win, false);
    } else {
        // z-marching kernel: at least ~16 planes per wave; one round of as
        // many 4-wave workgroups as its register use lets share each CU
        // (fewer drains than more, smaller rounds); the crease channel, when
        // wanted, comes along in the same kernel.
        const int64_t units = (int64_t)zmarch_3d_columns(fi.h, fi.w) * fi.d;
        p.grid = (int)std::min<int64_t>((int64_t)ctx->n_cu * zm_wg_per_cu(fi.dtype, fi.w, data, p.crease),
                                        std::max<int64_t>(1, (units + 63) / 64));
        if (p.grid >= 8) p.grid -= p.grid % 8;
        // A volume too small to give every CU a z-marching workgroup (its
        // columns are 256 voxels wide) runs faster on the tile kernel.
        // ECC_3D_KERNEL=tile or =zmarch overrides the choice (read per call).
        const char *ek = std::getenv("ECC_3D_KERNEL");
        const bool force_tile = ek && std::strcmp(ek, "tile") == 0;
        const bool force_zm = ek && std::strcmp(ek, "zmarch") == 0;
        p.zmarch = !force_tile && zmarch_3d_fits(fi.h, fi.w, p.grid) && (force_zm || p.grid >= ctx->n_cu);
    }
    if (fi.ndim == 3 && !p.zmarch) {
        const int64_t n_tiles = ((fi.w + kTile3DX - 1) / kTile3DX) * ((fi.h + kTile3DY - 1) / kTile3DY) *
                                ((fi.d + kTile3DZ - 1) / kTile3DZ);
        p.grid = pick_grid(ctx, n_tiles, lds_bytes_3d(p.win, p.crease) + 16 * 1024);
    }
    p.partial_bytes = (size_t)p.grid * p.nch * L * sizeof(int32_t);
    p.totals_bytes = (size_t)p.nch * L * sizeof(int64_t);
    return p;
}

// The field kernels, then the merge and scan, into buffers the caller
// provides (at least plan.partial_bytes and plan.totals_bytes; `counter` a
// zero word that the merge leaves at zero).  Allocates nothing.
ecc_status compute_core(ecc_context ctx, const ecc_field *f, const FieldInfo &fi, const ecc_curves *c,
                        const LevelArgs &lv, const OnePlan &p, int32_t *partial, int64_t *totals,
                        unsigned *counter, void *stream, bool timing, int64_t *acc) {
    const int L = fi.L;
    int64_t *outs[4] = {c->ec, c->perimeter, c->area, fi.ndim == 3 ? c->volume : nullptr};
    // the kernels load whole blocks of 16 bytes (2D) or 4 elements (3D), clamped
    // to the end of the field: a field smaller than one block is copied into a
    // buffer that holds a whole block
    const void *data = f->data;
    const int64_t block = fi.ndim == 2 ? vec_2d(fi.dtype) : 4;
    if (fi.cells < block) {
        int e = (int)hipMemcpyAsync(ctx->d_tiny, f->data, (size_t)fi.cells * fi.elem_bytes,
                                    hipMemcpyDeviceToDevice, (hipStream_t)stream);
        if (e) return hip_fail(e, "hipMemcpyAsync(small field)");
        data = ctx->d_tiny;
    }
    const int k = p.k;
    // fields below 2^28 cells drain the boundary measure and the count as one word
    const bool pack = acc && fi.cells < kPackMaxCells;
    for (int lo = 0; lo < L; lo += p.win) {
        const int hi = std::min(L, lo + p.win);
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        ecc_status s = timing ? prof_events(ctx, &ev0, &ev1) : ECC_OK;
        if (s != ECC_OK) return s;
        if (fi.ndim == 2) {
            Launch2D a{data, fi.dtype, fi.h, fi.w, lv, lo, hi, ctx->d_delta2[k], partial, p.grid,
                       0, fi.h, false, false};
            a.ev_start = ev0;
            a.ev_stop = ev1;
            a.acc = acc;
            a.pack = pack;
            int e = launch_2d(a, stream);
            if (e) return hip_fail(e, "2D kernel launch");
        } else {
            Launch3D a{data, fi.dtype, fi.d, fi.h, fi.w, lv, lo, hi, ctx->d_vtab3[k], partial, p.grid,
                       p.zmarch ? false : p.crease, p.zmarch ? ctx->d_zm3[k] : nullptr, k == 1, 0, fi.d, false,
                       p.zmarch && p.crease ? ctx->d_crease3 : nullptr};
            a.ev_start = ev0;
            a.ev_stop = ev1;
            a.acc = acc;
            a.pack_surf = pack;
            int e = launch_3d(a, stream);
            if (e) return hip_fail(e, "3D kernel launch");
        }
    }
    int e = acc ? launch_merge_acc(acc, kAccCopies, p.nch, L, outs, totals, counter, stream, pack ? (fi.ndim == 3 ? 2 : 1) : -1)
                : launch_merge(partial, p.grid, p.nch, L, outs, totals, counter, stream);
    if (e) return hip_fail(e, "merge kernel launch");
    return ECC_OK;
}

ecc_status compute_one(ecc_context ctx, const ecc_field *f, const FieldInfo &fi,
                       const ecc_curves *c, void *stream) {
    LevelArgs lv;
    ecc_status s = level_args(ctx, f, fi, stream, &lv);
    if (s != ECC_OK) return s;
    const OnePlan p = plan_one(ctx, fi, c, f->data);
    s = grow(ctx, ctx->ws.partial, p.partial_bytes, "partials");
    if (s != ECC_OK) return s;
    s = grow(ctx, ctx->ws.totals, p.totals_bytes, "totals");
    if (s != ECC_OK) return s;
    int64_t *acc = nullptr;
    if (atomic_drain() && (fi.ndim == 2 || p.zmarch)) {
        s = acc_buffer(ctx, p.nch, fi.L, &acc, stream);
        if (s != ECC_OK) return s;
        ctx->acc_dirty = true;
    }
    s = compute_core(ctx, f, fi, c, lv, p, (int32_t *)ctx->ws.partial.ptr, (int64_t *)ctx->ws.totals.ptr,
                     (unsigned *)ctx->d_counter, stream, true, acc);
    if (acc && s == ECC_OK) ctx->acc_dirty = false;  // the merge that clears them is queued
    if (s != ECC_OK) return s;
    return note_threshold_use(ctx, lv, stream);
}

// class channels into counts[c][L], three at a time (the merge kernel scans up
// to three channels per launch)
static ecc_status merge_classes(ecc_context ctx, int grid, int nch, int L, int64_t *counts, void *stream) {
    ecc_status s = grow(ctx, ctx->ws.totals, (size_t)3 * L * sizeof(int64_t), "totals");
    if (s != ECC_OK) return s;
    const int32_t *partial = (const int32_t *)ctx->ws.partial.ptr;
    for (int c0 = 0; c0 < nch; c0 += 3) {  // the merge kernel scans up to three channels at once
        int64_t *outs[4] = {nullptr, nullptr, nullptr, nullptr};
        for (int j = 0; j < 3 && c0 + j < nch; ++j) outs[j] = counts + (int64_t)(c0 + j) * L;
        const int n = std::min(3, nch - c0);
        int e = launch_merge(partial + (size_t)c0 * L * grid, grid, n, L, outs, (int64_t *)ctx->ws.totals.ptr,
                             (unsigned *)ctx->d_counter, stream);
        if (e) return hip_fail(e, "merge kernel launch");
    }
    return ECC_OK;
}

// Class counts of a 3D field: passes over windows of as many levels as one
// workgroup's LDS holds bins for (21 int32 per level, next to the staged tile),
// one 1024-thread workgroup per CU adding into the per-XCD accumulators, then
// one merge that scans every class.
static ecc_status compute_classes_3d(ecc_context ctx, const ecc_field *f, const FieldInfo &fi, int64_t *counts,
                                     void *stream) {
    LevelArgs lv;
    ecc_status s = level_args(ctx, f, fi, stream, &lv);
    if (s != ECC_OK) return s;
    const int L = fi.L, nch = kNumClasses3D;
    const size_t fixed = lds_fixed_classes_3d() + 64 * sizeof(int32_t);
    const int win_max = ctx->max_lds > fixed ? (int)((ctx->max_lds - fixed) / (nch * sizeof(int32_t))) : 0;
    if (win_max < 1) return fail(ECC_ERR_DEVICE, "3D class counts: not enough LDS per workgroup");
    const int passes = (L + win_max - 1) / win_max;
    const int win = (L + passes - 1) / passes;
    int64_t *acc = nullptr;
    s = acc_buffer(ctx, nch, L, &acc, stream);
    if (s != ECC_OK) return s;
    ctx->acc_dirty = true;
    const int64_t n_tiles = ((fi.w + 63) / 64) * ((fi.h + 7) / 8) * ((fi.d + 15) / 16);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(ctx->n_cu, n_tiles));
    for (int lo = 0; lo < L; lo += win) {
        Launch3DClasses a{f->data, fi.dtype, fi.d, fi.h, fi.w, lv, lo, std::min(L, lo + win), ctx->d_trans3, acc, grid};
        hipEvent_t ev0, ev1;
        s = prof_events(ctx, &ev0, &ev1);
        if (s != ECC_OK) return s;
        a.ev_start = ev0;
        a.ev_stop = ev1;
        int e = launch_classes_3d(a, stream);
        if (e) return hip_fail(e, "3D class-count kernel launch");
    }
    int e = launch_merge_acc_rows(acc, nch, L, counts, stream);
    if (e) return hip_fail(e, "class merge kernel launch");
    ctx->acc_dirty = false;  // the merge that clears them is queued
    return note_threshold_use(ctx, lv, stream);
}

// Class counts of a 2D field: the single-field 2D path with the class-count
// bins (five channels).
static ecc_status compute_classes(ecc_context ctx, const ecc_field *f, const FieldInfo &fi, int64_t *counts,
                                  void *stream) {
    if (fi.ndim == 3) return compute_classes_3d(ctx, f, fi, counts, stream);
    LevelArgs lv;
    ecc_status s = level_args(ctx, f, fi, stream, &lv);
    if (s != ECC_OK) return s;
    const int L = fi.L, nch = kNumClasses2D;
    const int win = std::min(L, kMaxWindow);
    const int vec = vec_2d(fi.dtype);
    const int grid = grid_2d(ctx, fi, win, true);
    s = grow(ctx, ctx->ws.partial, (size_t)grid * nch * L * sizeof(int32_t), "partials");
    if (s != ECC_OK) return s;
    int32_t *partial = (int32_t *)ctx->ws.partial.ptr;
    const void *data = f->data;
    if (fi.cells < vec) {  // smaller than one vector load: padded copy
        int e = (int)hipMemcpyAsync(ctx->d_tiny, f->data, (size_t)fi.cells * fi.elem_bytes,
                                    hipMemcpyDeviceToDevice, (hipStream_t)stream);
        if (e) return hip_fail(e, "hipMemcpyAsync(small field)");
        data = ctx->d_tiny;
    }
    for (int lo = 0; lo < L; lo += win) {
        const int hi = std::min(L, lo + win);
        Launch2D a{data, fi.dtype, fi.h, fi.w, lv, lo, hi, ctx->d_cls2, partial, grid, 0, fi.h, false, true};
        hipEvent_t ev0, ev1;
        s = prof_events(ctx, &ev0, &ev1);
        if (s != ECC_OK) return s;
        a.ev_start = ev0;
        a.ev_stop = ev1;
        int e = launch_2d(a, stream);
        if (e) return hip_fail(e, "2D class-count kernel launch");
    }
    s = merge_classes(ctx, grid, nch, L, counts, stream);
    if (s != ECC_OK) return s;
    return note_threshold_use(ctx, lv, stream);
}

}  // namespace ecc

extern "C" ecc_status ecc_vertex_classes_compute(ecc_context ctx, const ecc_field *field, int64_t *counts,
                                                 void *stream) {
    clear_error();
    if (!ctx) return fail(ECC_ERR_INVALID_ARG, "context is NULL");
    if (!counts) return fail(ECC_ERR_INVALID_ARG, "counts is NULL");
    FieldInfo fi;
    const ecc_curves probe{counts, nullptr, nullptr, nullptr};
    ecc_status s = validate_field(field, &probe, &fi, false);
    if (s != ECC_OK) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    int e = (int)hipSetDevice(ctx->device);
    if (e) return hip_fail(e, "hipSetDevice");
    s = acquire_workspace(ctx, stream);
    if (s != ECC_OK) return s;
    s = compute_classes(ctx, field, fi, counts, stream);
    ecc_status s2 = release_workspace(ctx, stream);
    return s != ECC_OK ? s : s2;
}

extern "C" ecc_status ecc_curves_compute(ecc_context ctx, const ecc_field *field,
                                         const ecc_curves *curves, void *stream) {
    clear_error();
    if (!ctx) return fail(ECC_ERR_INVALID_ARG, "context is NULL");
    FieldInfo fi;
    ecc_status s = validate_field(field, curves, &fi, false);
    if (s != ECC_OK) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    int e = (int)hipSetDevice(ctx->device);
    if (e) return hip_fail(e, "hipSetDevice");
    s = acquire_workspace(ctx, stream);
    if (s != ECC_OK) return s;
    s = compute_one(ctx, field, fi, curves, stream);
    ecc_status s2 = release_workspace(ctx, stream);
    return s != ECC_OK ? s : s2;
}

extern "C" ecc_status ecc_validate_field(const ecc_field *field, const ecc_curves *curves) {
    clear_error();
    FieldInfo fi;
    return validate_field(field, curves, &fi, false);
}

namespace ecc {
// Timing events are created without the system-scope fence (a cache
// write-back and invalidate when the event is recorded), which would run
// inside the measured interval and hold back the work after it.  They are only
// read for elapsed times, never to order memory.
static ecc_status timing_event_pair(hipEvent_t *a, hipEvent_t *b) {
    int e = (int)hipEventCreateWithFlags(a, hipEventDisableSystemFence);
    if (e) return hip_fail(e, "hipEventCreateWithFlags");
    e = (int)hipEventCreateWithFlags(b, hipEventDisableSystemFence);
    if (e) return hip_fail(e, "hipEventCreateWithFlags");
    return ECC_OK;
}

ecc_status prof_begin(ecc_context ctx, void *stream, int *slot) {
    *slot = -1;
    if (!ctx->prof_on) return ECC_OK;
    if (ctx->prof_used == ctx->prof_events.size()) {
        hipEvent_t a, b;
        ecc_status s = timing_event_pair(&a, &b);
        if (s != ECC_OK) return s;
        ctx->prof_events.push_back({a, b});
    }
    *slot = (int)ctx->prof_used++;
    int e = (int)hipEventRecord(ctx->prof_events[*slot].first, (hipStream_t)stream);
    if (e) return hip_fail(e, "hipEventRecord");
    return ECC_OK;
}

ecc_status prof_end(ecc_context ctx, void *stream, int slot) {
    if (slot < 0) return ECC_OK;
    int e = (int)hipEventRecord(ctx->prof_events[slot].second, (hipStream_t)stream);
    if (e) return hip_fail(e, "hipEventRecord");
    return ECC_OK;
}

ecc_status prof_events(ecc_context ctx, hipEvent_t *start, hipEvent_t *stop) {
    *start = *stop = nullptr;
    if (!ctx->prof_on) return ECC_OK;
    if (ctx->prof_used == ctx->prof_events.size()) {
        hipEvent_t a, b;
        ecc_status s = timing_event_pair(&a, &b);
        if (s != ECC_OK) return s;
        ctx->prof_events.push_back({a, b});
    }
    const size_t slot = ctx->prof_used++;
    *start = ctx->prof_events[slot].first;
    *stop = ctx->prof_events[slot].second;
    return ECC_OK;
}
}  // namespace ecc

extern "C" ecc_status ecc_profile_enable(ecc_context ctx, int32_t on) {
    clear_error();
    if (!ctx) return fail(ECC_ERR_INVALID_ARG, "context is NULL");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->prof_on = on != 0;
    return ECC_OK;
}

extern "C" ecc_status ecc_profile_read(ecc_context ctx, double *total_ms, int64_t *launches, int32_t reset) {
    clear_error();
    if (!ctx || !total_ms || !launches) return fail(ECC_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    double tot = 0;
    for (size_t i = 0; i < ctx->prof_used; ++i) {
        int e = (int)hipEventSynchronize(ctx->prof_events[i].second);
        if (e) return hip_fail(e, "hipEventSynchronize");
        float ms = 0;
        e = (int)hipEventElapsedTime(&ms, ctx->prof_events[i].first, ctx->prof_events[i].second);
        if (e) return hip_fail(e, "hipEventElapsedTime");
        tot += ms;
    }
    *total_ms = tot;
    *launches = (int64_t)ctx->prof_used;
    if (reset) ctx->prof_used = 0;
    return ECC_OK;
}
