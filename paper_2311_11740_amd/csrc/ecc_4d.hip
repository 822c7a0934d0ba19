// 4D fields: ecc_curves_compute_4d.
//
// The field is a stack of a volumes (slices); its curves follow from 3D
// curves of the slices and of the images of consecutive slices (min images
// for the closure, max images for the face-adjacency complex), see the
// slab kernel in ecc_k3d.hip.  The host cuts every slice and image into items
// of whole tiles of one shape (chosen for the d x h x w slice), deals them to
// workgroups, and queues the slab kernel and the finishing kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "ecc_runtime.h"

using namespace ecc;

extern "C" ecc_status ecc_curves_compute_4d(ecc_context ctx, const ecc_field4 *field, int64_t *ec,
                                            int64_t *boundary, int64_t *volume, void *stream) {
    clear_error();
    if (!ctx) return fail(ECC_ERR_INVALID_ARG, "context is NULL");
    if (!field) return fail(ECC_ERR_INVALID_ARG, "field is NULL");
    if (!ec && !boundary && !volume) return fail(ECC_ERR_INVALID_ARG, "no output curve requested");
    for (int k = 0; k < 4; ++k)
        if (field->shape[k] < 1) return fail(ECC_ERR_INVALID_ARG, "every shape entry must be >= 1");
    int conn = field->connectivity;
    if (conn == 0) conn = 80;
    if (conn != 80 && conn != 8) return fail(ECC_ERR_INVALID_ARG, "4D connectivity must be 80 or 8");
    const int64_t a = field->shape[0], d = field->shape[1], h = field->shape[2], w = field->shape[3];
    int64_t cells = 1;
    for (int k = 0; k < 4; ++k) {
        if (field->shape[k] > (int64_t(1) << 31) / cells) return fail(ECC_ERR_UNSUPPORTED, "more than 2^31 cells");
        cells *= field->shape[k];
    }
    // the slices stacked as one volume: dtype, data, levels, thresholds and
    // filtration checked (and level arguments built) as for a 3D field
    ecc_field f3{};
    f3.ndim = 3;
    f3.dtype = field->dtype;
    f3.shape[0] = a * d;
    f3.shape[1] = h;
    f3.shape[2] = w;
    f3.data = field->data;
    f3.n_levels = field->n_levels;
    f3.connectivity = 26;
    f3.thresholds = field->thresholds;
    f3.filtration = field->filtration;
    int64_t probe = 0;
    const ecc_curves c3{&probe, nullptr, nullptr, nullptr};
    FieldInfo fi;
    ecc_status s = validate_field(&f3, &c3, &fi, false);
    if (s != ECC_OK) return s;
    if (fi.L > kBatchMaxLevels) return fail(ECC_ERR_UNSUPPORTED, "4D fields take at most 4096 levels");
    const bool faces = conn == 8;
    const int L = fi.L;

    std::lock_guard<std::mutex> lk(ctx->mu);
    int e = (int)hipSetDevice(ctx->device);
    if (e) return hip_fail(e, "hipSetDevice");
    s = acquire_workspace(ctx, stream);
    if (s != ECC_OK) return s;
    auto done = [&](ecc_status st) {
        const ecc_status s2 = release_workspace(ctx, stream);
        return st != ECC_OK ? st : s2;
    };
    LevelArgs lv;
    s = level_args(ctx, &f3, fi, stream, &lv);
    if (s != ECC_OK) return done(s);

    // items: (virtual volume, tile range); slices v < a, then the images
    const TileShape ts = tile_shape_3d(d, h, w);
    const int64_t tiles_x = (w + ts.tx - 1) / ts.tx, tiles_y = (h + ts.ty - 1) / ts.ty;
    const int64_t n_vol = a + (faces ? std::max<int64_t>(a - 1, 0) : a + 1);
    if (n_vol * tiles_x * tiles_y * ((d + ts.tz - 1) / ts.tz) > (int64_t(1) << 30))
        return done(fail(ECC_ERR_UNSUPPORTED, "too many 4D work items"));
    std::vector<BatchItem> sorted;
    std::vector<int32_t> first;
    const int grid = schedule_4d(ctx->n_cu, L, n_vol, d, h, w, ts, sorted, first);

    s = grow(ctx, ctx->ws.items, sizeof(BatchItem) * sorted.size(), "4D work items");
    if (s == ECC_OK) s = grow(ctx, ctx->ws.first, sizeof(int32_t) * first.size(), "4D work split");
    if (s == ECC_OK) s = grow(ctx, ctx->ws.totals, (size_t)3 * L * sizeof(int64_t), "totals");
    int64_t *acc = nullptr;
    if (s == ECC_OK) s = acc_buffer(ctx, 6, L, &acc, stream);
    if (s != ECC_OK) return done(s);
    hipStream_t st = (hipStream_t)stream;
    // pageable sources: the copies are staged before the calls return
    e = (int)hipMemcpyAsync(ctx->ws.items.ptr, sorted.data(), sizeof(BatchItem) * sorted.size(),
                            hipMemcpyHostToDevice, st);
    if (!e)
        e = (int)hipMemcpyAsync(ctx->ws.first.ptr, first.data(), sizeof(int32_t) * first.size(),
                                hipMemcpyHostToDevice, st);
    if (e) return done(hip_fail(e, "hipMemcpyAsync(4D schedule)"));

    Launch4D g{};
    g.data = field->data;
    g.dtype = field->dtype;
    g.a = a;
    g.d = d;
    g.h = h;
    g.w = w;
    g.lv = lv;
    g.faces = faces;
    g.items = (const BatchItem *)ctx->ws.items.ptr;
    g.wg_first = (const int32_t *)ctx->ws.first.ptr;
    g.grid = grid;
    g.vtab = ctx->d_vtab3[faces ? 1 : 0];
    g.acc = acc;
    g.totals = (int64_t *)ctx->ws.totals.ptr;
    g.out[0] = ec;
    g.out[1] = boundary;
    g.out[2] = volume;
    g.tx = ts.tx;
    g.ty = ts.ty;
    g.tz = ts.tz;
    g.tiles_x = (int)tiles_x;
    g.tiles_y = (int)tiles_y;
    ctx->acc_dirty = true;
    e = launch_4d(g, stream);
    if (e) return done(hip_fail(e, "4D kernel launch"));
    ctx->acc_dirty = false;  // the finishing kernel that clears them is queued
    return done(note_threshold_use(ctx, lv, stream));
}
