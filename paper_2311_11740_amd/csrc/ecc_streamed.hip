// Fields in host memory, streamed through the device in slabs.
//
// The analogue of the paper's low-memory mode (Computational Results: memory
// scaling; Conclusions): a field that lives in host memory (and may be larger
// than device memory) is cut along its slowest axis into slabs of whole rows
// (2D) or planes (3D).  Each slab is copied with one halo row or plane on each
// side into one of two device buffers on a copy stream, while the slab before
// it is histogrammed on the caller's stream; every slab adds to the same
// accumulators (or per-workgroup partials), so the merge and scan run once at
// the end.  A cell is counted by the slab that owns it, and its neighbours
// come from the halo, so the curves are those of the whole field.
//
// Pinned host memory is copied to the device directly.  Pageable memory is
// first copied by host threads into one of two pinned bounce buffers (while
// the previous bounce buffer's DMA and the slab before run), which is what
// lets the copy engine run at the pinned rate.  The buffers, the copy stream,
// the events and the copy threads live in the context and are reused by the
// next call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "ecc_copier.h"
#include "ecc_internal.h"
#include "ecc_runtime.h"

namespace ecc {

struct StreamState {
    DevBuf buf[2];  // device slab buffers
    DevBuf curves;  // device curves of the call
    char *bounce[2] = {nullptr, nullptr};  // pinned bounce buffers for pageable fields
    size_t bounce_bytes = 0;
    hipStream_t copy = nullptr;
    // copied: a slab landed in buf[b]; computed: the kernels that read buf[b]
    // are done; drained: the DMA out of bounce[b] is done
    hipEvent_t copied[2] = {nullptr, nullptr}, computed[2] = {nullptr, nullptr}, drained[2] = {nullptr, nullptr};
    Copier copier;
};

void destroy_stream_state(ecc_context ctx) {
    StreamState *st = ctx->streamed;
    if (!st) return;
    if (st->copy) {
        hipStreamSynchronize(st->copy);
        hipStreamDestroy(st->copy);
    }
    for (int k = 0; k < 2; ++k) {
        if (st->copied[k]) hipEventDestroy(st->copied[k]);
        if (st->computed[k]) hipEventDestroy(st->computed[k]);
        if (st->drained[k]) hipEventDestroy(st->drained[k]);
        if (st->bounce[k]) hipHostFree(st->bounce[k]);
        st->buf[k].release();
    }
    st->curves.release();
    delete st;
    ctx->streamed = nullptr;
}

namespace {

ecc_status stream_state(ecc_context ctx, StreamState **out) {
    if (!ctx->streamed) {
        auto *st = new StreamState();
        int e = (int)hipStreamCreateWithFlags(&st->copy, hipStreamNonBlocking);
        for (int b = 0; b < 2 && !e; ++b) {
            e = (int)hipEventCreateWithFlags(&st->copied[b], hipEventDisableTiming);
            if (!e) e = (int)hipEventCreateWithFlags(&st->computed[b], hipEventDisableTiming);
            if (!e) e = (int)hipEventCreateWithFlags(&st->drained[b], hipEventDisableTiming);
        }
        ctx->streamed = st;
        if (e) {
            destroy_stream_state(ctx);
            return hip_fail(e, "streamed-path stream/events");
        }
    }
    *out = ctx->streamed;
    return ECC_OK;
}

// whether host memory at p is pinned (page-locked and known to the runtime)
bool host_pinned(const void *p) {
    hipPointerAttribute_t attr;
    const hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeHost;
}

ecc_status stream_field(ecc_context ctx, const ecc_field *f, const FieldInfo &fi, const ecc_curves *c,
                        size_t slab_bytes, void *stream) {
    const bool is3 = fi.ndim == 3;
    const int64_t unit_bytes = (is3 ? fi.h * fi.w : fi.w) * fi.elem_bytes;  // one row or plane
    const int64_t n_units = is3 ? fi.d : fi.h;
    if (slab_bytes == 0) slab_bytes = (size_t)256 << 20;
    const int64_t per_slab = (int64_t)(slab_bytes / (size_t)unit_bytes) - 2;  // rows or planes owned
    if (per_slab < 1)
        return fail(ECC_ERR_INVALID_ARG, "slab_bytes must hold at least three rows (2D) or planes (3D)");
    const int64_t R = std::min(per_slab, n_units);
    const bool crease = is3 && c->perimeter != nullptr;
    const int L = fi.L;
    const int nch = is3 ? 4 : 3;
    const int win = std::min(L, kMaxWindow);
    const int k = is3 ? (fi.conn == 26 ? 0 : 1) : (fi.conn == 8 ? 0 : 1);
    // one launch geometry for every slab (the partials of a workgroup add up)
    int grid;
    if (is3) {
        const int64_t units = (int64_t)zmarch_3d_columns(fi.h, fi.w) * R;
        // (the slab buffers are device allocations: aligned)
        grid = (int)std::min<int64_t>((int64_t)ctx->n_cu * zm_wg_per_cu(fi.dtype, fi.w, nullptr, crease),
                                      std::max<int64_t>(1, (units + 63) / 64));
        if (grid >= 8) grid -= grid % 8;
        if (!zmarch_3d_fits(fi.h, fi.w, grid))
            return fail(ECC_ERR_UNSUPPORTED, "streamed 3D fields: planes too large for the z-marching kernel");
    } else {
        FieldInfo slab = fi;
        slab.h = R;
        grid = grid_2d(ctx, slab, win, false);
    }
    StreamState *st = nullptr;
    ecc_status s = stream_state(ctx, &st);
    if (s != ECC_OK) return s;
    LevelArgs lv;
    s = level_args(ctx, f, fi, stream, &lv);
    if (s != ECC_OK) return s;
    // slab + halo at offset kPad, with kPad bytes after it: the kernels' vector
    // loads are clamped to the last whole vector of the field they are given
    // (here: up to the end of the buffer's units), which for a slab of fewer
    // cells than one vector starts up to 64 bytes before the slab
    constexpr size_t kPad = 256;
    const size_t slab_copy = (size_t)(R + 2) * (size_t)unit_bytes;
    const size_t buf_bytes = slab_copy + 2 * kPad;
    const bool acc_drain = atomic_drain();
    int32_t *partial = nullptr;
    int64_t *acc = nullptr;
    for (int b = 0; b < 2; ++b) {
        s = grow(ctx, st->buf[b], buf_bytes, "slab buffer");
        if (s != ECC_OK) return s;
    }
    s = grow(ctx, st->curves, (size_t)nch * L * sizeof(int64_t), "curves");
    if (s == ECC_OK) s = grow(ctx, ctx->ws.totals, (size_t)nch * L * sizeof(int64_t), "totals");
    if (s != ECC_OK) return s;
    if (acc_drain) {
        s = acc_buffer(ctx, nch, L, &acc, stream);
        ctx->acc_dirty = s == ECC_OK;
    } else {
        s = grow(ctx, ctx->ws.partial, (size_t)grid * nch * L * sizeof(int32_t), "partials");
        partial = (int32_t *)ctx->ws.partial.ptr;
    }
    if (s != ECC_OK) return s;
    const bool pinned = host_pinned(f->data);
    if (!pinned && st->bounce_bytes < slab_copy) {
        // rare: wait for the DMA that may still read the old bounce buffers
        int e = (int)hipStreamSynchronize(st->copy);
        for (int b = 0; b < 2 && !e; ++b) {
            if (st->bounce[b]) hipHostFree(st->bounce[b]);
            st->bounce[b] = nullptr;
        }
        st->bounce_bytes = 0;
        for (int b = 0; b < 2 && !e; ++b) e = (int)hipHostMalloc(&st->bounce[b], slab_copy, 0);
        if (e) return fail(ECC_ERR_OUT_OF_MEMORY, "hipHostMalloc(bounce buffers) failed");
        st->bounce_bytes = slab_copy;
    }
    hipStream_t cs = (hipStream_t)stream;
    // the copy stream starts after the work already queued on the caller's stream
    int e = (int)hipEventRecord(st->computed[0], cs);
    if (!e) e = (int)hipEventRecord(st->computed[1], cs);
    if (e) return hip_fail(e, "hipEventRecord");

    const char *host = (const char *)f->data;
    int slab = 0;
    for (int64_t a = 0; a < n_units; a += R, ++slab) {
        const int64_t b = std::min(n_units, a + R);
        const int64_t u0 = a > 0 ? a - 1 : 0, u1 = std::min(n_units, b + 1);  // units in the buffer
        const int bi = slab & 1;
        const size_t n = (size_t)(u1 - u0) * (size_t)unit_bytes;
        char *dev = (char *)st->buf[bi].ptr + kPad;
        const char *src = host + u0 * unit_bytes;
        if (!pinned) {
            // stage the slab in a pinned bounce buffer once its previous DMA is done
            e = (int)hipEventSynchronize(st->drained[bi]);
            if (e) return hip_fail(e, "hipEventSynchronize");
            st->copier.copy(st->bounce[bi], src, n);
            src = st->bounce[bi];
        }
        e = (int)hipStreamWaitEvent(st->copy, st->computed[bi], 0);
        if (!e) e = (int)hipMemcpyAsync(dev, src, n, hipMemcpyHostToDevice, st->copy);
        if (!e) e = (int)hipEventRecord(st->copied[bi], st->copy);
        if (!e && !pinned) e = (int)hipEventRecord(st->drained[bi], st->copy);
        if (!e) e = (int)hipStreamWaitEvent(cs, st->copied[bi], 0);
        if (e) return hip_fail(e, "slab copy");
        // the buffer seen as the field's units [0, u1) (units below u0 are never read)
        const void *data_v = dev - u0 * unit_bytes;
        for (int lo = 0; lo < L; lo += win) {
            const int hi = std::min(L, lo + win);
            if (is3) {
                Launch3D la{data_v, fi.dtype, u1, fi.h, fi.w, lv, lo, hi, ctx->d_vtab3[k], partial, grid, false,
                            ctx->d_zm3[k], k == 1, a, b, slab > 0, crease ? ctx->d_crease3 : nullptr};
                la.acc = acc;
                la.pack_surf = acc && fi.cells < kPackMaxCells;
                e = launch_3d(la, stream);
            } else {
                Launch2D la{data_v, fi.dtype, u1, fi.w, lv, lo, hi, ctx->d_delta2[k], partial, grid,
                            a, b, slab > 0, false};
                la.acc = acc;
                la.pack = acc && fi.cells < kPackMaxCells;
                e = launch_2d(la, stream);
            }
            if (e) return hip_fail(e, "slab kernel launch");
        }
        e = (int)hipEventRecord(st->computed[bi], cs);
        if (e) return hip_fail(e, "hipEventRecord");
    }
    int64_t *dc = (int64_t *)st->curves.ptr;
    int64_t *host_out[4] = {c->ec, c->perimeter, c->area, is3 ? c->volume : nullptr};
    int64_t *outs[4];
    for (int ch = 0; ch < 4; ++ch) outs[ch] = host_out[ch] ? dc + (size_t)ch * L : nullptr;
    e = acc ? launch_merge_acc(acc, kAccCopies, nch, L, outs, (int64_t *)ctx->ws.totals.ptr,
                               (unsigned *)ctx->d_counter, stream, acc && fi.cells < kPackMaxCells ? (is3 ? 2 : 1) : -1)
            : launch_merge(partial, grid, nch, L, outs, (int64_t *)ctx->ws.totals.ptr, (unsigned *)ctx->d_counter,
                           stream);
    if (e) return hip_fail(e, "merge kernel launch");
    if (acc) ctx->acc_dirty = false;
    for (int ch = 0; ch < 4; ++ch) {
        if (!host_out[ch]) continue;
        e = (int)hipMemcpyAsync(host_out[ch], outs[ch], (size_t)L * sizeof(int64_t), hipMemcpyDeviceToHost, cs);
        if (e) return hip_fail(e, "curve copy");
    }
    e = (int)hipStreamSynchronize(cs);
    if (e) return hip_fail(e, "hipStreamSynchronize");
    return ECC_OK;
}

}  // namespace

}  // namespace ecc

using namespace ecc;

extern "C" ecc_status ecc_curves_compute_streamed(ecc_context ctx, const ecc_field *field,
                                                  const ecc_curves *curves, size_t slab_bytes, void *stream) {
    clear_error();
    if (!ctx) return fail(ECC_ERR_INVALID_ARG, "context is NULL");
    FieldInfo fi;
    ecc_status s = validate_field(field, curves, &fi, true);
    if (s != ECC_OK) return s;
    std::lock_guard<std::mutex> lk(ctx->mu);
    int e = (int)hipSetDevice(ctx->device);
    if (e) return hip_fail(e, "hipSetDevice");
    s = acquire_workspace(ctx, stream);
    if (s != ECC_OK) return s;
    s = stream_field(ctx, field, fi, curves, slab_bytes, stream);
    ecc_status s2 = release_workspace(ctx, stream);
    return s != ECC_OK ? s : s2;
}
