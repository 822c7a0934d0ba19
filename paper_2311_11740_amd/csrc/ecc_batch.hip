// Batched entry point and its autotuner.
//
// A batch call groups its fields by kernel class: 2D fields with at most
// kBatchMaxLevels levels and kBatchMaxCells cells go to the persistent 2D
// batched kernel, volumes with at most kBatchMaxLevels levels and
// kBatch3DMaxCells voxels to the persistent 3D batched kernel (one launch per
// (dimension, dtype, level mode) group); every other field (more levels,
// large volumes, fewer cells than one vector load) runs through the
// single-field path on the same stream after them.
//
// The plan of a batch (work items, their assignment to workgroups, per-field
// histograms and tickets, the captured graph) depends only on the shapes,
// dtypes, level counts, connectivities and level modes of the fields, so it is
// cached under that key and reused; a call only rewrites the per-field
// descriptors (data and output pointers, level arguments) with one
// host-to-device copy and replays the graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <functional>
#include <map>
#include <queue>
#include <string>
#include <tuple>
#include <vector>

#include "ecc_runtime.h"

namespace ecc {

struct BatchGroup {
    int ndim = 2, dtype = 0, lm = 0;
    std::vector<int> fields;  // descriptor slots
    int grid = 0, max_L = 0, n_items = 0;
    BatchItem *d_items = nullptr;
    int32_t *d_wg_first = nullptr;
};

struct BatchPlan {
    std::string key;
    int item_cells = 0, wg_per_cu = 0;
    std::vector<BatchGroup> groups;
    std::vector<int> kind;     // field index -> 2 or 3 (batched kernel), 0 = single-field path
    std::vector<int> slot_of;  // field index -> slot in its kind's descriptors
    std::vector<int> others;   // fields on the single-field path
    int n_desc = 0, n_desc3 = 0;
    std::vector<int32_t> n_items_of;  // per field index
    std::vector<int64_t> hist_off;    // per field index, in int32 elements
    BatchField2D *d_desc = nullptr, *h_desc = nullptr;
    BatchField3D *d_desc3 = nullptr, *h_desc3 = nullptr;
    int32_t *d_hist = nullptr;
    uint32_t *d_done = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t copy_done = nullptr, last_use = nullptr;
    bool copy_pending = false, used = false;
    uint64_t last_tick = 0;
};

struct BatchState {
    std::vector<BatchPlan *> plans;
    std::map<std::string, std::pair<int, int>> tuned;  // key -> (item cells, workgroups per CU)
    hipStream_t capture = nullptr;
    uint64_t tick = 0;
    uint64_t *d_luts = nullptr;  // [2][256] packed 2D per-cell deltas, 8-C then 4-C
    int64_t *d_vt3 = nullptr;    // [2][256] 3D per-octant tables, 26-C then 6-C
};

constexpr size_t kMaxPlans = 8;
constexpr int kDefaultItemCells = 64 * 1024;
constexpr int kDefaultWgPerCu = 4;

static void free_plan(BatchPlan *p) {
    if (!p) return;
    for (auto &g : p->groups) {
        if (g.d_items) hipFree(g.d_items);
        if (g.d_wg_first) hipFree(g.d_wg_first);
    }
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    if (p->d_desc) hipFree(p->d_desc);
    if (p->h_desc) hipHostFree(p->h_desc);
    if (p->d_desc3) hipFree(p->d_desc3);
    if (p->h_desc3) hipHostFree(p->h_desc3);
    if (p->d_hist) hipFree(p->d_hist);
    if (p->d_done) hipFree(p->d_done);
    if (p->copy_done) hipEventDestroy(p->copy_done);
    if (p->last_use) hipEventDestroy(p->last_use);
    delete p;
}

void destroy_batch_state(ecc_context ctx) {
    BatchState *b = ctx->batch;
    if (!b) return;
    for (auto *p : b->plans) free_plan(p);
    if (b->capture) hipStreamDestroy(b->capture);
    if (b->d_luts) hipFree(b->d_luts);
    if (b->d_vt3) hipFree(b->d_vt3);
    delete b;
    ctx->batch = nullptr;
}

static ecc_status batch_state(ecc_context ctx, BatchState **out) {
    if (!ctx->batch) {
        auto *b = new BatchState();
        int e = (int)hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
        if (e) {
            delete b;
            return hip_fail(e, "hipStreamCreate");
        }
        e = (int)hipMalloc(&b->d_luts, 2 * 256 * sizeof(uint64_t));
        if (!e) e = (int)hipMalloc(&b->d_vt3, 2 * 256 * sizeof(int64_t));
        if (e) {
            if (b->d_luts) hipFree(b->d_luts);
            hipStreamDestroy(b->capture);
            delete b;
            return fail(ECC_ERR_OUT_OF_MEMORY, "hipMalloc(batch tables) failed");
        }
        for (int k = 0; k < 2 && !e; ++k) {
            e = (int)hipMemcpy(b->d_luts + 256 * k, ctx->d_delta2[k], 256 * sizeof(uint64_t),
                               hipMemcpyDeviceToDevice);
            if (!e)
                e = (int)hipMemcpy(b->d_vt3 + 256 * k, ctx->d_vtab3[k], 256 * sizeof(int64_t),
                                   hipMemcpyDeviceToDevice);
        }
        if (e) {
            hipFree(b->d_luts);
            hipFree(b->d_vt3);
            hipStreamDestroy(b->capture);
            delete b;
            return hip_fail(e, "hipMemcpy(batch tables)");
        }
        ctx->batch = b;
    }
    *out = ctx->batch;
    return ECC_OK;
}

// the batched kernel that takes a field (2 or 3), or 0
int batch_kind(const FieldInfo &fi) {
    if (fi.L > kBatchMaxLevels) return 0;
    if (fi.ndim == 2) return fi.cells <= kBatchMaxCells && fi.cells >= vec_2d(fi.dtype) ? 2 : 0;
    return fi.cells <= kBatch3DMaxCells ? 3 : 0;
}

bool batchable(const FieldInfo &fi) { return batch_kind(fi) != 0; }

static std::string plan_key(int n, const FieldInfo *fi, const LevelArgs *lv) {
    std::string k;
    k.reserve((size_t)n * 40 + 16);
    auto put = [&k](int64_t v) { k.append(reinterpret_cast<const char *>(&v), sizeof(v)); };
    put(n);
    for (int i = 0; i < n; ++i) {
        put(fi[i].ndim | fi[i].dtype << 4 | (int64_t)fi[i].conn << 8 | (int64_t)lv[i].mode << 16 |
            (int64_t)fi[i].L << 24);
        put(fi[i].d);
        put(fi[i].h);
        put(fi[i].w);
    }
    return k;
}

// descriptors of a field (everything but the plan's histogram, ticket and item count)
void fill_desc_2d(BatchField2D &d, const ecc_field &f, const ecc_curves &c, const FieldInfo &fi,
                  const LevelArgs &lv) {
    std::memset(&d, 0, sizeof(d));
    d.data = f.data;
    d.h = fi.h;
    d.w = fi.w;
    d.out[0] = c.ec;
    d.out[1] = c.perimeter;
    d.out[2] = c.area;
    d.thr = lv.thr;
    d.lut = lv.lut;
    d.L = fi.L;
    d.conn_idx = fi.conn == 8 ? 0 : 1;
    d.inv_step = lv.inv_step;
    d.neg = lv.neg;
    d.cpass = pass_constant(lv.u0d, 0);
    d.eps = lv.eps;
}

void fill_desc_3d(BatchField3D &d, const ecc_field &f, const ecc_curves &c, const FieldInfo &fi,
                  const LevelArgs &lv) {
    std::memset(&d, 0, sizeof(d));
    d.data = f.data;
    d.d = fi.d;
    d.h = fi.h;
    d.w = fi.w;
    d.out[0] = c.ec;
    d.out[1] = c.perimeter;
    d.out[2] = c.area;
    d.out[3] = c.volume;
    d.thr = lv.thr;
    d.lut = lv.lut;
    d.L = fi.L;
    d.conn_idx = fi.conn == 26 ? 0 : 1;
    d.neg = lv.neg;
    d.u0 = lv.u0;
    d.inv_step = lv.inv_step;
    d.eps = lv.eps;
    const TileShape ts = tile_shape_3d(fi.d, fi.h, fi.w);
    d.tx = ts.tx;
    d.ty = ts.ty;
    d.tz = ts.tz;
    d.tiles_x = (int32_t)((fi.w + ts.tx - 1) / ts.tx);
    d.tiles_y = (int32_t)((fi.h + ts.ty - 1) / ts.ty);
}

static int launch_group(const BatchState *bs, const BatchPlan *p, const BatchGroup &g, void *stream) {
    if (g.ndim == 2)
        return launch_batch_2d(g.dtype, g.lm, p->d_desc, g.d_items, g.d_wg_first, g.grid, bs->d_luts, g.max_L,
                               stream);
    return launch_batch_3d(g.dtype, g.lm, p->d_desc3, g.d_items, g.d_wg_first, g.grid, bs->d_vt3, g.max_L, stream);
}

// A cached plan: batchable fields grouped by (dimension, dtype, level mode), each group
// scheduled as above, device copies of the schedules, per-field histograms
// and tickets, and the group launches captured as a graph.
static ecc_status build_plan(ecc_context ctx, BatchState *bs, int n, const FieldInfo *fi, const LevelArgs *lv,
                             const std::string &key, int item_cells, int wg_per_cu, BatchPlan **out) {
    auto *p = new BatchPlan();
    p->key = key;
    p->item_cells = item_cells;
    p->wg_per_cu = wg_per_cu;
    p->slot_of.assign(n, -1);
    p->kind.assign(n, 0);
    std::map<std::tuple<int, int, int>, int> group_of;
    for (int i = 0; i < n; ++i) {
        const int kd = batch_kind(fi[i]);
        if (!kd) {
            p->others.push_back(i);
            continue;
        }
        const auto gk = std::make_tuple(kd, fi[i].dtype, lv[i].mode);
        auto it = group_of.find(gk);
        if (it == group_of.end()) {
            it = group_of.emplace(gk, (int)p->groups.size()).first;
            p->groups.emplace_back();
            p->groups.back().ndim = kd;
            p->groups.back().dtype = fi[i].dtype;
            p->groups.back().lm = lv[i].mode;
        }
        p->kind[i] = kd;
        p->slot_of[i] = kd == 2 ? p->n_desc++ : p->n_desc3++;
        p->groups[it->second].fields.push_back(i);
    }
    p->n_items_of.assign(n, 0);
    p->hist_off.assign(n, 0);
    int64_t hist_total = 0;
    for (int i = 0; i < n; ++i)
        if (p->kind[i]) {
            p->hist_off[i] = hist_total;
            hist_total += (p->kind[i] == 2 ? 3 : 4) * (int64_t)fi[i].L;
        }
    auto cleanup = [&](ecc_status s) {
        free_plan(p);
        return s;
    };
    for (auto &g : p->groups) {
        std::vector<SchedField> sf;
        for (int i : g.fields) {
            g.max_L = std::max(g.max_L, fi[i].L);
            sf.push_back(SchedField{p->slot_of[i], fi[i].h, fi[i].w, fi[i].d});
        }
        std::vector<BatchItem> sorted;
        std::vector<int32_t> first;
        std::vector<int32_t> n_items;
        if (g.ndim == 2)
            g.grid = schedule_batch_2d(ctx->n_cu, g.dtype, g.lm, g.max_L, sf, item_cells, wg_per_cu, sorted, first,
                                       n_items);
        else
            g.grid = schedule_batch_3d(ctx->n_cu, g.max_L, sf, item_cells, wg_per_cu, sorted, first, n_items);
        g.n_items = (int)sorted.size();
        for (size_t j = 0; j < g.fields.size(); ++j) p->n_items_of[g.fields[j]] = n_items[j];
        int e = (int)hipMalloc(&g.d_items, sizeof(BatchItem) * std::max<size_t>(1, sorted.size()));
        if (e) return cleanup(fail(ECC_ERR_OUT_OF_MEMORY, "hipMalloc(batch items) failed"));
        e = (int)hipMalloc(&g.d_wg_first, sizeof(int32_t) * first.size());
        if (e) return cleanup(fail(ECC_ERR_OUT_OF_MEMORY, "hipMalloc(batch schedule) failed"));
        e = (int)hipMemcpy(g.d_items, sorted.data(), sizeof(BatchItem) * sorted.size(), hipMemcpyHostToDevice);
        if (!e) e = (int)hipMemcpy(g.d_wg_first, first.data(), sizeof(int32_t) * first.size(), hipMemcpyHostToDevice);
        if (e) return cleanup(hip_fail(e, "hipMemcpy(batch plan)"));
    }
    if (p->n_desc > 0) {
        int e = (int)hipMalloc(&p->d_desc, sizeof(BatchField2D) * p->n_desc);
        if (e) return cleanup(fail(ECC_ERR_OUT_OF_MEMORY, "hipMalloc(batch descriptors) failed"));
        e = (int)hipHostMalloc(&p->h_desc, sizeof(BatchField2D) * p->n_desc, 0);
        if (e) return cleanup(hip_fail(e, "hipHostMalloc(batch descriptors)"));
    }
    if (p->n_desc3 > 0) {
        int e = (int)hipMalloc(&p->d_desc3, sizeof(BatchField3D) * p->n_desc3);
        if (e) return cleanup(fail(ECC_ERR_OUT_OF_MEMORY, "hipMalloc(batch descriptors) failed"));
        e = (int)hipHostMalloc(&p->h_desc3, sizeof(BatchField3D) * p->n_desc3, 0);
        if (e) return cleanup(hip_fail(e, "hipHostMalloc(batch descriptors)"));
    }
    if (p->n_desc + p->n_desc3 > 0) {
        int e = (int)hipMalloc(&p->d_hist, sizeof(int32_t) * std::max<int64_t>(1, hist_total));
        if (e) return cleanup(fail(ECC_ERR_OUT_OF_MEMORY, "hipMalloc(batch histograms) failed"));
        e = (int)hipMalloc(&p->d_done, sizeof(uint32_t) * n);
        if (e) return cleanup(fail(ECC_ERR_OUT_OF_MEMORY, "hipMalloc(batch tickets) failed"));
        // the kernels leave both at zero after every launch
        e = (int)hipMemset(p->d_hist, 0, sizeof(int32_t) * std::max<int64_t>(1, hist_total));
        if (!e) e = (int)hipMemset(p->d_done, 0, sizeof(uint32_t) * n);
        if (!e) e = (int)hipDeviceSynchronize();
        if (e) return cleanup(hip_fail(e, "hipMemset(batch workspace)"));
    }
    int e = (int)hipEventCreateWithFlags(&p->copy_done, hipEventDisableTiming);
    if (!e) e = (int)hipEventCreateWithFlags(&p->last_use, hipEventDisableTiming);
    if (e) return cleanup(hip_fail(e, "hipEventCreate"));
    // capture the group launches into a graph; on failure the call launches them directly
    if (!p->groups.empty()) {
        bool ok = hipStreamBeginCapture(bs->capture, hipStreamCaptureModeRelaxed) == hipSuccess;
        bool launched = ok;
        for (auto &g : p->groups)
            if (launched) launched = launch_group(bs, p, g, bs->capture) == 0;
        if (ok) ok = hipStreamEndCapture(bs->capture, &p->graph) == hipSuccess && launched;
        if (ok) ok = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) == hipSuccess;
        if (!ok) {
            if (p->exec) hipGraphExecDestroy(p->exec);
            if (p->graph) hipGraphDestroy(p->graph);
            p->exec = nullptr;
            p->graph = nullptr;
            (void)hipGetLastError();
        }
    }
    *out = p;
    return ECC_OK;
}

static ecc_status find_or_build_plan(ecc_context ctx, BatchState *bs, int n, const FieldInfo *fi,
                                     const LevelArgs *lv, int force_item_cells, int force_wpc, BatchPlan **out) {
    const std::string key = plan_key(n, fi, lv);
    const bool forced = force_item_cells > 0;
    if (!forced)
        for (auto *p : bs->plans)
            if (p->key == key) {
                p->last_tick = ++bs->tick;
                *out = p;
                return ECC_OK;
            }
    int cells = kDefaultItemCells, wpc = kDefaultWgPerCu;
    auto t = bs->tuned.find(key);
    if (t != bs->tuned.end()) {
        cells = t->second.first;
        wpc = t->second.second;
    }
    if (forced) {
        cells = force_item_cells;
        wpc = force_wpc;
    }
    BatchPlan *p = nullptr;
    ecc_status s = build_plan(ctx, bs, n, fi, lv, key, cells, wpc, &p);
    if (s != ECC_OK) return s;
    p->last_tick = ++bs->tick;
    if (!forced) {
        if (bs->plans.size() >= kMaxPlans) {  // evict the least recently used plan
            auto lru = std::min_element(bs->plans.begin(), bs->plans.end(),
                                        [](BatchPlan *a, BatchPlan *b) { return a->last_tick < b->last_tick; });
            int e = (int)hipEventSynchronize((*lru)->last_use);
            if (e) {
                free_plan(p);
                return hip_fail(e, "hipEventSynchronize");
            }
            free_plan(*lru);
            bs->plans.erase(lru);
        }
        bs->plans.push_back(p);
    }
    *out = p;
    return ECC_OK;
}

// Queue one run of a plan on `stream`: descriptors, the graph (or the group
// launches), then the fields of the single-field path.
static ecc_status run_plan(ecc_context ctx, BatchState *bs, BatchPlan *p, int n, const ecc_field *fields,
                           const ecc_curves *curves, const FieldInfo *fi, const LevelArgs *lv, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    int e;
    if (p->used) {  // after the previous run of this plan (its histograms and tickets)
        e = (int)hipStreamWaitEvent(st, p->last_use, 0);
        if (e) return hip_fail(e, "hipStreamWaitEvent");
    }
    if (p->n_desc + p->n_desc3 > 0) {
        if (p->copy_pending) {  // the pinned descriptors may still be in flight
            e = (int)hipEventSynchronize(p->copy_done);
            if (e) return hip_fail(e, "hipEventSynchronize");
        }
        for (int i = 0; i < n; ++i) {
            const int sl = p->slot_of[i];
            if (p->kind[i] == 2) {
                BatchField2D &d = p->h_desc[sl];
                fill_desc_2d(d, fields[i], curves[i], fi[i], lv[i]);
                d.hist = p->d_hist + p->hist_off[i];
                d.done = p->d_done + i;
                d.n_items = p->n_items_of[i];
            } else if (p->kind[i] == 3) {
                BatchField3D &d = p->h_desc3[sl];
                fill_desc_3d(d, fields[i], curves[i], fi[i], lv[i]);
                d.hist = p->d_hist + p->hist_off[i];
                d.done = p->d_done + i;
                d.n_items = p->n_items_of[i];
            }
        }
        e = 0;
        if (p->n_desc)
            e = (int)hipMemcpyAsync(p->d_desc, p->h_desc, sizeof(BatchField2D) * p->n_desc, hipMemcpyHostToDevice,
                                    st);
        if (!e && p->n_desc3)
            e = (int)hipMemcpyAsync(p->d_desc3, p->h_desc3, sizeof(BatchField3D) * p->n_desc3,
                                    hipMemcpyHostToDevice, st);
        if (e) return hip_fail(e, "hipMemcpyAsync(batch descriptors)");
        e = (int)hipEventRecord(p->copy_done, st);
        if (e) return hip_fail(e, "hipEventRecord");
        p->copy_pending = true;
        int slot = -1;
        ecc_status s = prof_begin(ctx, stream, &slot);
        if (s != ECC_OK) return s;
        if (p->exec) {
            e = (int)hipGraphLaunch(p->exec, st);
            if (e) return hip_fail(e, "hipGraphLaunch");
        } else {
            for (auto &g : p->groups) {
                e = launch_group(bs, p, g, stream);
                if (e) return hip_fail(e, "batched kernel launch");
            }
        }
        s = prof_end(ctx, stream, slot);
        if (s != ECC_OK) return s;
        for (int i = 0; i < n; ++i) {  // the graph reads these threshold arrays
            if (!p->kind[i] || !lv[i].thr) continue;
            bool seen = false;
            for (int j = 0; j < i && !seen; ++j) seen = p->kind[j] && lv[j].thr == lv[i].thr;
            if (!seen) {
                s = note_threshold_use(ctx, lv[i], stream);
                if (s != ECC_OK) return s;
            }
        }
    }
    if (!p->others.empty()) {
        ecc_status s = acquire_workspace(ctx, stream);
        if (s != ECC_OK) return s;
        for (int i : p->others) {
            s = compute_one(ctx, &fields[i], fi[i], &curves[i], stream);
            if (s != ECC_OK) break;
        }
        ecc_status s2 = release_workspace(ctx, stream);
        if (s != ECC_OK) return s;
        if (s2 != ECC_OK) return s2;
    }
    e = (int)hipEventRecord(p->last_use, st);
    if (e) return hip_fail(e, "hipEventRecord");
    p->used = true;
    return ECC_OK;
}

// validation and level arguments of every field (thresholds uploaded once per
// distinct array)
static ecc_status prepare(ecc_context ctx, int n, const ecc_field *fields, const ecc_curves *curves,
                          void *stream, std::vector<FieldInfo> &fi, std::vector<LevelArgs> &lv) {
    fi.resize(n);
    lv.resize(n);
    for (int i = 0; i < n; ++i) {
        ecc_status s = validate_field(&fields[i], &curves[i], &fi[i], false);
        if (s != ECC_OK) return s;
    }
    std::vector<const ecc_field *> fp(n);
    for (int i = 0; i < n; ++i) fp[i] = &fields[i];
    ecc_status s = reserve_thresholds(ctx, n, fp.data(), stream);
    if (s != ECC_OK) return s;
    for (int i = 0; i < n; ++i) {
        s = level_args(ctx, &fields[i], fi[i], stream, &lv[i]);
        if (s != ECC_OK) return s;
    }
    return ECC_OK;
}

}  // namespace ecc

using namespace ecc;

extern "C" ecc_status ecc_curves_compute_batch(ecc_context ctx, int32_t n, const ecc_field *fields,
                                               const ecc_curves *curves, void *stream) {
    clear_error();
    if (!ctx) return fail(ECC_ERR_INVALID_ARG, "context is NULL");
    if (n < 0 || (n > 0 && (!fields || !curves))) return fail(ECC_ERR_INVALID_ARG, "bad batch arrays");
    if (n == 0) return ECC_OK;
    for (int i = 0; i < n; ++i) {  // host-only checks before any device work
        FieldInfo f;
        ecc_status s = validate_field(&fields[i], &curves[i], &f, false);
        if (s != ECC_OK) return s;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    int e = (int)hipSetDevice(ctx->device);
    if (e) return hip_fail(e, "hipSetDevice");
    std::vector<FieldInfo> fi;
    std::vector<LevelArgs> lv;
    ecc_status s = prepare(ctx, n, fields, curves, stream, fi, lv);
    if (s != ECC_OK) return s;
    BatchState *bs = nullptr;
    s = batch_state(ctx, &bs);
    if (s != ECC_OK) return s;
    BatchPlan *p = nullptr;
    s = find_or_build_plan(ctx, bs, n, fi.data(), lv.data(), 0, 0, &p);
    if (s != ECC_OK) return s;
    return run_plan(ctx, bs, p, n, fields, curves, fi.data(), lv.data(), stream);
}

extern "C" ecc_status ecc_batch_plan_tune(ecc_context ctx, int32_t n, const ecc_field *fields, void *stream) {
    clear_error();
    if (!ctx) return fail(ECC_ERR_INVALID_ARG, "context is NULL");
    if (n < 0 || (n > 0 && !fields)) return fail(ECC_ERR_INVALID_ARG, "bad batch arrays");
    if (n == 0) return ECC_OK;
    // trial runs write no curves; validation sees one (unused) output so that
    // it accepts the request
    std::vector<ecc_curves> none(n), probe(n);
    std::memset(none.data(), 0, sizeof(ecc_curves) * n);
    std::memset(probe.data(), 0, sizeof(ecc_curves) * n);
    static int64_t dummy;
    for (int i = 0; i < n; ++i) {
        probe[i].ec = &dummy;
        FieldInfo f;
        ecc_status s = validate_field(&fields[i], &probe[i], &f, false);
        if (s != ECC_OK) return s;
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    int e = (int)hipSetDevice(ctx->device);
    if (e) return hip_fail(e, "hipSetDevice");
    std::vector<FieldInfo> fi;
    std::vector<LevelArgs> lv;
    ecc_status s = prepare(ctx, n, fields, probe.data(), stream, fi, lv);
    if (s != ECC_OK) return s;
    BatchState *bs = nullptr;
    s = batch_state(ctx, &bs);
    if (s != ECC_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t t0, t1;
    e = (int)hipEventCreate(&t0);
    if (e) return hip_fail(e, "hipEventCreate");
    e = (int)hipEventCreate(&t1);
    if (e) {
        hipEventDestroy(t0);
        return hip_fail(e, "hipEventCreate");
    }
    const bool prof = ctx->prof_on;
    ctx->prof_on = false;  // trial runs are not reported
    const int cells_c[] = {16 * 1024, 32 * 1024, 64 * 1024, 128 * 1024, 256 * 1024};
    const int wpc_c[] = {2, 4, 8};
    float best = 1e30f;
    std::pair<int, int> best_cfg(kDefaultItemCells, kDefaultWgPerCu);
    for (int cells : cells_c)
        for (int wpc : wpc_c) {
            BatchPlan *p = nullptr;
            s = find_or_build_plan(ctx, bs, n, fi.data(), lv.data(), cells, wpc, &p);
            if (s != ECC_OK) break;
            float ms = 1e30f;
            for (int rep = 0; rep < 3 && s == ECC_OK; ++rep) {
                e = (int)hipEventRecord(t0, st);
                if (!e) s = run_plan(ctx, bs, p, n, fields, none.data(), fi.data(), lv.data(), stream);
                if (!e && s == ECC_OK) e = (int)hipEventRecord(t1, st);
                if (!e && s == ECC_OK) e = (int)hipEventSynchronize(t1);
                float t = 0.f;
                if (!e && s == ECC_OK) e = (int)hipEventElapsedTime(&t, t0, t1);
                if (e && s == ECC_OK) s = hip_fail(e, "timing a trial run");
                if (rep > 0 && s == ECC_OK) ms = std::min(ms, t);  // first run warms up
            }
            const int e2 = (int)hipStreamSynchronize(st);
            free_plan(p);
            if (s != ECC_OK) break;
            if (e2) {
                s = hip_fail(e2, "hipStreamSynchronize");
                break;
            }
            if (ms < best) {
                best = ms;
                best_cfg = {cells, wpc};
            }
        }
    ctx->prof_on = prof;
    hipEventDestroy(t0);
    hipEventDestroy(t1);
    if (s != ECC_OK) return s;
    const std::string key = plan_key(n, fi.data(), lv.data());
    bs->tuned[key] = best_cfg;
    for (auto it = bs->plans.begin(); it != bs->plans.end(); ++it)  // rebuild with the tuned geometry
        if ((*it)->key == key) {
            hipEventSynchronize((*it)->last_use);
            free_plan(*it);
            bs->plans.erase(it);
            break;
        }
    return ECC_OK;
}
