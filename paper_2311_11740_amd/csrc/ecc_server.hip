// Serving loop: continuous batching of EC-curve requests.
//
// Memory.  At creation the server takes one device arena of the HBM budget, a
// pinned host arena of the same layout for staging and results, and a fixed number of
// slots (each with a per-level histogram and ticket for the batched kernel).
// A request is admitted when a slot is free and the arena has room for its
// field and curves (first fit); otherwise the submit returns ECC_ERR_BUSY.
// An admitted request keeps its device copy of the field and its curves
// resident until its results are back on the host, then releases them.
//
// Work.  The submitting thread stages the field in its pinned range (large
// fields with several copy threads).  A worker thread copies staged fields to
// the device on a copy stream and launches every request whose copy has
// landed, all at once: the 2D fields and the small volumes the batched
// kernels take go into one launch of those kernels (as many as are ready, up
// to max_batch), the others (large volumes, more than 4096 levels) run the
// single-field path on a second compute stream; results come back to pinned
// memory and then to the caller's arrays.  Requests submitted while earlier
// ones are on the GPU are copied meanwhile and join the next launch, so
// copies and kernels of different requests overlap.  The worker holds the
// server's lock only to take new requests and to retire finished ones.
#include <hip/hip_runtime.h>

#include <chrono>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "ecc_copier.h"
#include "ecc_runtime.h"

namespace ecc {

// first-fit allocator of byte ranges in [0, size), 256-byte granules
class Arena {
  public:
    void init(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t n, size_t *off) {
        n = round(n);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                *off = it->first;
                const size_t rest = it->second - n, at = it->first + n;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t n) {
        n = round(n);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    static size_t round(size_t n) { return (n + 255) & ~size_t(255); }

  private:
    std::map<size_t, size_t> free_;
};


enum ReqState { kReserving, kStaged, kCopying, kReady, kRunning, kComplete, kFailed };

struct Request {
    uint64_t ticket = 0;
    ecc_field field{};   // data points into the device arena once admitted
    FieldInfo fi{};
    std::vector<float> thr;
    ecc_curves host_out{};
    int nch = 0;
    size_t field_bytes = 0, total_bytes = 0, off = 0;
    int slot = -1;
    std::atomic<int> state{kReserving};  // written by the worker, read by poll
    ecc_status err = ECC_OK;
    hipEvent_t ev_h2d = nullptr;
    int launch = -1;  // index of the completion event in the server's ring
};

}  // namespace ecc

using namespace ecc;

struct ecc_server_s {
    ecc_context ctx = nullptr;
    ecc_server_config cfg{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    hipStream_t s_copy = nullptr, s_2d = nullptr, s_other = nullptr;
    char *d_arena = nullptr, *h_arena = nullptr;
    Arena dev;
    std::vector<int> free_slots;
    int32_t *d_hist = nullptr;  // [slots][4][kBatchMaxLevels]
    uint32_t *d_done = nullptr;  // [slots]
    uint64_t *d_luts = nullptr;  // [2][256]
    int64_t *d_vt3 = nullptr;    // [2][256]
    // per-launch schedule buffers (device + pinned), reused once their launch is done
    struct Launch {
        BatchField2D *d_desc = nullptr, *h_desc = nullptr;
        BatchField3D *d_desc3 = nullptr, *h_desc3 = nullptr;
        BatchItem *d_items = nullptr, *h_items = nullptr;
        int32_t *d_first = nullptr, *h_first = nullptr;
        size_t cap_desc = 0, cap_desc3 = 0, cap_items = 0, cap_first = 0;
        hipEvent_t done = nullptr;
        bool busy = false;
    };
    std::vector<Launch> ring;
    std::unordered_map<uint64_t, Request *> reqs;
    std::deque<Request *> staged, copying, ready;
    Copier copier;
    std::vector<Request *> running;
    uint64_t next_ticket = 1;
    int64_t inflight = 0;
};

namespace {

constexpr int kRing = 4;

ecc_status grow_pair(void **d, void **h, size_t *cap, size_t need) {
    if (need <= *cap) return ECC_OK;
    size_t n = std::max(need, *cap * 2);
    if (*d) hipFree(*d);
    if (*h) hipHostFree(*h);
    *d = *h = nullptr;
    *cap = 0;
    int e = (int)hipMalloc(d, n);
    if (e) return fail(ECC_ERR_OUT_OF_MEMORY, "hipMalloc(serving schedule) failed");
    e = (int)hipHostMalloc(h, n, 0);
    if (e) return hip_fail(e, "hipHostMalloc(serving schedule)");
    *cap = n;
    return ECC_OK;
}

// a finished request's curves, from its pinned slot into the caller's arrays
void copy_results(ecc_server srv, Request *r) {
    const char *res = srv->h_arena + r->off + Arena::round(r->field_bytes);
    int64_t *dst[4] = {r->host_out.ec, r->host_out.perimeter, r->host_out.area, r->host_out.volume};
    int k = 0;
    for (int c = 0; c < 4; ++c)
        if (dst[c]) {
            std::memcpy(dst[c], res + (size_t)k * r->fi.L * 8, (size_t)r->fi.L * 8);
            ++k;
        }
}

// release a request's memory and slot and report it done; srv->mu held
void retire(ecc_server srv, Request *r, ecc_status err) {
    srv->dev.release(r->off, r->total_bytes);
    srv->free_slots.push_back(r->slot);
    if (r->ev_h2d) hipEventDestroy(r->ev_h2d);
    r->ev_h2d = nullptr;
    r->err = err;
    r->state = err == ECC_OK ? kComplete : kFailed;
    --srv->inflight;
}

// device curves of a request (channels packed in ec, perimeter, area, volume order)
int64_t *dev_curves(ecc_server srv, Request *r) {
    return reinterpret_cast<int64_t *>(srv->d_arena + r->off + Arena::round(r->field_bytes));
}

ecc_curves dev_curve_ptrs(ecc_server srv, Request *r) {
    ecc_curves c{};
    int64_t *base = dev_curves(srv, r);
    int64_t **dst[4] = {&c.ec, &c.perimeter, &c.area, &c.volume};
    int64_t *want[4] = {r->host_out.ec, r->host_out.perimeter, r->host_out.area, r->host_out.volume};
    int k = 0;
    for (int ch = 0; ch < 4; ++ch)
        if (want[ch]) *dst[ch] = base + (size_t)(k++) * r->fi.L;
    return c;
}

// queue the D2H copy of a request's curves into its pinned slot
ecc_status copy_back(ecc_server srv, Request *r, hipStream_t s) {
    const size_t off = r->off + Arena::round(r->field_bytes);
    int e = (int)hipMemcpyAsync(srv->h_arena + off, srv->d_arena + off, (size_t)r->nch * r->fi.L * 8,
                                hipMemcpyDeviceToHost, s);
    return e ? hip_fail(e, "hipMemcpyAsync(results)") : ECC_OK;
}

int free_launch(ecc_server srv) {
    for (int i = 0; i < (int)srv->ring.size(); ++i)
        if (!srv->ring[i].busy) return i;
    return -1;
}

// Launch every ready request (worker thread, without srv->mu: the ready,
// running and launch lists belong to the worker).  Requests that fail to
// launch go to `failed`.
ecc_status launch_ready(ecc_server srv, std::vector<std::pair<Request *, ecc_status>> &failed) {
    ecc_context ctx = srv->ctx;
    std::vector<Request *> batch2d, other;
    const int li = free_launch(srv);
    std::deque<Request *> keep;
    // a launch takes at most as many distinct threshold arrays (by content) as
    // the context's cache holds at once; requests beyond wait for the next one
    std::vector<const ecc_field *> thr_fields;
    int n_thr = 0;
    for (Request *r : srv->ready) {
        bool take = batchable(r->fi) && li >= 0 && (int)batch2d.size() < srv->cfg.max_batch;
        if (take && (r->field.thresholds || r->fi.super)) {  // a threshold array (or implied superlevel one)
            thr_fields.push_back(&r->field);
            const int k = count_distinct_thresholds((int)thr_fields.size(), thr_fields.data());
            if (k > (int)kThrCacheMax) {
                thr_fields.pop_back();
                take = false;
            } else {
                n_thr = k;
            }
        }
        if (take)
            batch2d.push_back(r);
        else if (!batchable(r->fi))
            other.push_back(r);
        else
            keep.push_back(r);  // waits for the next launch
    }
    (void)n_thr;
    if (batch2d.empty() && other.empty()) return ECC_OK;
    srv->ready.swap(keep);
    std::lock_guard<std::mutex> lk(ctx->mu);
    ecc_status s = ECC_OK;
    if (!batch2d.empty()) {
        auto &L = srv->ring[li];
        std::vector<LevelArgs> lv(batch2d.size());
        s = reserve_thresholds(ctx, (int)thr_fields.size(), thr_fields.data(), srv->s_2d);
        for (size_t i = 0; i < batch2d.size() && s == ECC_OK; ++i)
            s = level_args(ctx, &batch2d[i]->field, batch2d[i]->fi, srv->s_2d, &lv[i]);
        // group by (dimension, dtype, level mode); one schedule per group,
        // items appended; a request's descriptor slot counts within its dimension
        std::map<std::tuple<int, int, int>, std::vector<int>> groups;
        std::vector<int> slot(batch2d.size());
        int n2 = 0, n3 = 0;
        for (size_t i = 0; i < batch2d.size(); ++i) {
            const int kd = batch_kind(batch2d[i]->fi);
            slot[i] = kd == 2 ? n2++ : n3++;
            groups[std::make_tuple(kd, batch2d[i]->fi.dtype, lv[i].mode)].push_back((int)i);
        }
        std::vector<BatchItem> all_items;
        std::vector<int32_t> all_first;
        struct G {
            int kind, dtype, lm, max_L, grid;
            size_t item0, first0;
        };
        std::vector<G> gl;
        std::vector<int32_t> n_items_of(batch2d.size(), 0);
        for (auto &kv : groups) {
            const int kd = std::get<0>(kv.first), dt = std::get<1>(kv.first), lm = std::get<2>(kv.first);
            std::vector<SchedField> sf;
            int max_L = 0;
            for (int i : kv.second) {
                const FieldInfo &f = batch2d[i]->fi;
                sf.push_back(SchedField{slot[i], f.h, f.w, f.d});
                max_L = std::max(max_L, f.L);
            }
            std::vector<BatchItem> items;
            std::vector<int32_t> first, n_items;
            const int grid = kd == 2 ? schedule_batch_2d(ctx->n_cu, dt, lm, max_L, sf, 64 * 1024, 4, items, first,
                                                         n_items)
                                     : schedule_batch_3d(ctx->n_cu, max_L, sf, 64 * 1024, 4, items, first, n_items);
            for (size_t j = 0; j < kv.second.size(); ++j) n_items_of[kv.second[j]] = n_items[j];
            gl.push_back(G{kd, dt, lm, max_L, grid, all_items.size(), all_first.size()});
            all_items.insert(all_items.end(), items.begin(), items.end());
            all_first.insert(all_first.end(), first.begin(), first.end());
        }
        if (s == ECC_OK && n2)
            s = grow_pair((void **)&L.d_desc, (void **)&L.h_desc, &L.cap_desc, sizeof(BatchField2D) * n2);
        if (s == ECC_OK && n3)
            s = grow_pair((void **)&L.d_desc3, (void **)&L.h_desc3, &L.cap_desc3, sizeof(BatchField3D) * n3);
        if (s == ECC_OK) s = grow_pair((void **)&L.d_items, (void **)&L.h_items, &L.cap_items,
                                       sizeof(BatchItem) * std::max<size_t>(1, all_items.size()));
        if (s == ECC_OK) s = grow_pair((void **)&L.d_first, (void **)&L.h_first, &L.cap_first,
                                       sizeof(int32_t) * std::max<size_t>(1, all_first.size()));
        if (s == ECC_OK) {
            for (size_t i = 0; i < batch2d.size(); ++i) {
                Request *r = batch2d[i];
                const ecc_curves c = dev_curve_ptrs(srv, r);
                int32_t *hist = srv->d_hist + (size_t)r->slot * 4 * kBatchMaxLevels;
                if (batch_kind(r->fi) == 2) {
                    BatchField2D &d = L.h_desc[slot[i]];
                    fill_desc_2d(d, r->field, c, r->fi, lv[i]);
                    d.hist = hist;
                    d.done = srv->d_done + r->slot;
                    d.n_items = n_items_of[i];
                } else {
                    BatchField3D &d = L.h_desc3[slot[i]];
                    fill_desc_3d(d, r->field, c, r->fi, lv[i]);
                    d.hist = hist;
                    d.done = srv->d_done + r->slot;
                    d.n_items = n_items_of[i];
                }
            }
            std::memcpy(L.h_items, all_items.data(), sizeof(BatchItem) * all_items.size());
            std::memcpy(L.h_first, all_first.data(), sizeof(int32_t) * all_first.size());
            int e = 0;
            if (n2)
                e = (int)hipMemcpyAsync(L.d_desc, L.h_desc, sizeof(BatchField2D) * n2, hipMemcpyHostToDevice,
                                        srv->s_2d);
            if (!e && n3)
                e = (int)hipMemcpyAsync(L.d_desc3, L.h_desc3, sizeof(BatchField3D) * n3, hipMemcpyHostToDevice,
                                        srv->s_2d);
            if (!e) e = (int)hipMemcpyAsync(L.d_items, L.h_items, sizeof(BatchItem) * all_items.size(),
                                            hipMemcpyHostToDevice, srv->s_2d);
            if (!e) e = (int)hipMemcpyAsync(L.d_first, L.h_first, sizeof(int32_t) * all_first.size(),
                                            hipMemcpyHostToDevice, srv->s_2d);
            for (size_t g = 0; g < gl.size() && !e; ++g)
                e = gl[g].kind == 2
                        ? launch_batch_2d(gl[g].dtype, gl[g].lm, L.d_desc, L.d_items + gl[g].item0,
                                          L.d_first + gl[g].first0, gl[g].grid, srv->d_luts, gl[g].max_L, srv->s_2d)
                        : launch_batch_3d(gl[g].dtype, gl[g].lm, L.d_desc3, L.d_items + gl[g].item0,
                                          L.d_first + gl[g].first0, gl[g].grid, srv->d_vt3, gl[g].max_L, srv->s_2d);
            if (e) s = hip_fail(e, "serving batched launch");
            for (size_t i = 0; i < batch2d.size() && s == ECC_OK; ++i) {  // the launch reads these arrays
                bool seen = false;
                for (size_t j = 0; j < i && !seen; ++j) seen = lv[j].thr == lv[i].thr;
                if (!seen) s = note_threshold_use(ctx, lv[i], srv->s_2d);
            }
        }
        for (Request *r : batch2d)
            if (s == ECC_OK) s = copy_back(srv, r, srv->s_2d);
        if (s == ECC_OK) {
            int e = (int)hipEventRecord(L.done, srv->s_2d);
            if (e) s = hip_fail(e, "hipEventRecord");
        }
        for (Request *r : batch2d) {
            if (s == ECC_OK) {
                r->state = kRunning;
                r->launch = li;
                srv->running.push_back(r);
            } else {
                failed.push_back({r, s});
            }
        }
        if (s == ECC_OK) L.busy = true;
    }
    for (Request *r : other) {
        // the single-field path, one request after the other on its own stream
        ecc_status so = acquire_workspace(ctx, srv->s_other);
        const ecc_curves c = dev_curve_ptrs(srv, r);
        if (so == ECC_OK) so = compute_one(ctx, &r->field, r->fi, &c, srv->s_other);
        const ecc_status s2 = release_workspace(ctx, srv->s_other);
        if (so == ECC_OK) so = s2;
        if (so == ECC_OK) so = copy_back(srv, r, srv->s_other);
        if (so == ECC_OK && !r->ev_h2d) {
            int e = (int)hipEventCreateWithFlags(&r->ev_h2d, hipEventDisableTiming);
            if (e) so = hip_fail(e, "hipEventCreate");
        }
        if (so == ECC_OK) {
            int e = (int)hipEventRecord(r->ev_h2d, srv->s_other);  // reused as the completion event
            if (e) so = hip_fail(e, "hipEventRecord");
        }
        if (so == ECC_OK) {
            r->state = kRunning;
            r->launch = -1;
            srv->running.push_back(r);
        } else {
            failed.push_back({r, so});
        }
    }
    return ECC_OK;
}

// One pass over all requests (worker thread); returns whether anything
// changed.  srv->mu is taken only to take new requests and to retire
// finished ones, so submit and poll never wait for the GPU calls.
bool advance(ecc_server srv) {
    bool moved = false;
    std::deque<Request *> fresh;
    std::vector<std::pair<Request *, ecc_status>> done;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        fresh.swap(srv->staged);
    }
    // copies of staged requests
    for (Request *r : fresh) {
        int e = (int)hipEventCreateWithFlags(&r->ev_h2d, hipEventDisableTiming);
        if (!e) e = (int)hipMemcpyAsync(srv->d_arena + r->off, srv->h_arena + r->off, r->field_bytes,
                                        hipMemcpyHostToDevice, srv->s_copy);
        if (!e) e = (int)hipEventRecord(r->ev_h2d, srv->s_copy);
        if (e) {
            done.push_back({r, hip_fail(e, "serving copy")});
        } else {
            r->state = kCopying;
            srv->copying.push_back(r);
        }
        moved = true;
    }
    // copies that have landed
    for (auto it = srv->copying.begin(); it != srv->copying.end();) {
        if (hipEventQuery((*it)->ev_h2d) == hipSuccess) {
            (*it)->state = kReady;
            srv->ready.push_back(*it);
            it = srv->copying.erase(it);
            moved = true;
        } else {
            ++it;
        }
    }
    if (!srv->ready.empty()) {
        const size_t before = srv->ready.size();
        launch_ready(srv, done);
        moved |= srv->ready.size() != before;
    }
    // finished launches: results to the callers' arrays
    std::vector<bool> ring_done(srv->ring.size(), false);
    for (size_t i = 0; i < srv->ring.size(); ++i)
        ring_done[i] = srv->ring[i].busy && hipEventQuery(srv->ring[i].done) == hipSuccess;
    for (auto it = srv->running.begin(); it != srv->running.end();) {
        Request *r = *it;
        const bool fin = r->launch >= 0 ? ring_done[r->launch] : hipEventQuery(r->ev_h2d) == hipSuccess;
        if (fin) {
            copy_results(srv, r);
            done.push_back({r, ECC_OK});
            it = srv->running.erase(it);
            moved = true;
        } else {
            ++it;
        }
    }
    for (size_t i = 0; i < srv->ring.size(); ++i)
        if (ring_done[i]) srv->ring[i].busy = false;
    if (!done.empty()) {
        std::lock_guard<std::mutex> lk(srv->mu);
        for (auto &d : done) retire(srv, d.first, d.second);
        srv->cv_done.notify_all();
    }
    return moved;
}

void worker_main(ecc_server srv) {
    hipSetDevice(srv->ctx->device);
    for (;;) {
        const bool moved = advance(srv);
        const bool busy = !srv->copying.empty() || !srv->ready.empty() || !srv->running.empty();
        std::unique_lock<std::mutex> lk(srv->mu);
        if (srv->stop && !busy && srv->staged.empty()) break;
        if (!moved && srv->staged.empty()) {
            if (busy)  // GPU work in flight: check again shortly
                srv->cv_work.wait_for(lk, std::chrono::microseconds(20));
            else
                srv->cv_work.wait(lk, [srv] { return srv->stop || !srv->staged.empty(); });
        }
    }
}

void release_server(ecc_server srv) {
    for (auto &L : srv->ring) {
        if (L.d_desc) hipFree(L.d_desc);
        if (L.h_desc) hipHostFree(L.h_desc);
        if (L.d_desc3) hipFree(L.d_desc3);
        if (L.h_desc3) hipHostFree(L.h_desc3);
        if (L.d_items) hipFree(L.d_items);
        if (L.h_items) hipHostFree(L.h_items);
        if (L.d_first) hipFree(L.d_first);
        if (L.h_first) hipHostFree(L.h_first);
        if (L.done) hipEventDestroy(L.done);
    }
    for (auto &kv : srv->reqs) {
        if (kv.second->ev_h2d) hipEventDestroy(kv.second->ev_h2d);
        delete kv.second;
    }
    if (srv->d_arena) hipFree(srv->d_arena);
    if (srv->h_arena) hipHostFree(srv->h_arena);
    if (srv->d_hist) hipFree(srv->d_hist);
    if (srv->d_done) hipFree(srv->d_done);
    if (srv->d_luts) hipFree(srv->d_luts);
    if (srv->d_vt3) hipFree(srv->d_vt3);
    if (srv->s_copy) hipStreamDestroy(srv->s_copy);
    if (srv->s_2d) hipStreamDestroy(srv->s_2d);
    if (srv->s_other) hipStreamDestroy(srv->s_other);
    delete srv;
}

}  // namespace

extern "C" ecc_status ecc_server_create(ecc_context ctx, const ecc_server_config *cfg, ecc_server *out) {
    clear_error();
    if (!ctx || !cfg || !out) return fail(ECC_ERR_INVALID_ARG, "NULL argument");
    if (cfg->hbm_budget_bytes < 4096 || cfg->max_slots < 1 || cfg->max_slots > 65536 || cfg->max_batch < 1)
        return fail(ECC_ERR_INVALID_ARG, "server config: budget >= 4096 bytes, 1 <= max_slots <= 65536, "
                                         "max_batch >= 1");
    auto *srv = new ecc_server_s();
    srv->ctx = ctx;
    srv->cfg = *cfg;
    srv->cfg.max_batch = std::min(cfg->max_batch, cfg->max_slots);
    int e = (int)hipSetDevice(ctx->device);
    auto bail = [&](ecc_status s) {
        release_server(srv);
        return s;
    };
    if (e) return bail(hip_fail(e, "hipSetDevice"));
    const size_t budget = Arena::round(cfg->hbm_budget_bytes);
    e = (int)hipMalloc(&srv->d_arena, budget);
    if (e) return bail(fail(ECC_ERR_OUT_OF_MEMORY, "hipMalloc(serving arena) failed"));
    e = (int)hipHostMalloc(&srv->h_arena, budget, 0);
    if (e) return bail(hip_fail(e, "hipHostMalloc(serving staging)"));
    srv->dev.init(budget);
    const size_t hist = (size_t)cfg->max_slots * 4 * kBatchMaxLevels * sizeof(int32_t);
    e = (int)hipMalloc(&srv->d_hist, hist);
    if (!e) e = (int)hipMalloc(&srv->d_done, (size_t)cfg->max_slots * sizeof(uint32_t));
    if (e) return bail(fail(ECC_ERR_OUT_OF_MEMORY, "hipMalloc(serving histograms) failed"));
    // zero once; the batched kernel leaves every slot's histogram and ticket at zero
    e = (int)hipMemset(srv->d_hist, 0, hist);
    if (!e) e = (int)hipMemset(srv->d_done, 0, (size_t)cfg->max_slots * sizeof(uint32_t));
    if (!e) e = (int)hipMalloc(&srv->d_luts, 2 * 256 * sizeof(uint64_t));
    if (!e) e = (int)hipMalloc(&srv->d_vt3, 2 * 256 * sizeof(int64_t));
    for (int k = 0; k < 2 && !e; ++k) {
        e = (int)hipMemcpy(srv->d_luts + 256 * k, ctx->d_delta2[k], 256 * sizeof(uint64_t), hipMemcpyDeviceToDevice);
        if (!e)
            e = (int)hipMemcpy(srv->d_vt3 + 256 * k, ctx->d_vtab3[k], 256 * sizeof(int64_t), hipMemcpyDeviceToDevice);
    }
    if (!e) e = (int)hipDeviceSynchronize();
    if (e) return bail(hip_fail(e, "serving set-up"));
    e = (int)hipStreamCreateWithFlags(&srv->s_copy, hipStreamNonBlocking);
    if (!e) e = (int)hipStreamCreateWithFlags(&srv->s_2d, hipStreamNonBlocking);
    if (!e) e = (int)hipStreamCreateWithFlags(&srv->s_other, hipStreamNonBlocking);
    if (e) return bail(hip_fail(e, "hipStreamCreate"));
    srv->ring.resize(kRing);
    for (auto &L : srv->ring) {
        e = (int)hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
        if (e) return bail(hip_fail(e, "hipEventCreate"));
    }
    {
        // the single-field path's workspace, grown now for up to 4096 levels,
        // so that a request does not wait for the device to grow it later
        std::lock_guard<std::mutex> lk(ctx->mu);
        ecc_status s = grow(ctx, ctx->ws.partial, (size_t)4 * 4096 * 4 * ctx->n_cu * sizeof(int32_t), "partials");
        if (s == ECC_OK) s = grow(ctx, ctx->ws.totals, (size_t)4 * 4096 * sizeof(int64_t), "totals");
        if (s != ECC_OK) return bail(s);
    }
    for (int i = cfg->max_slots - 1; i >= 0; --i) srv->free_slots.push_back(i);
    srv->worker = std::thread(worker_main, srv);
    *out = srv;
    return ECC_OK;
}

extern "C" ecc_status ecc_server_submit(ecc_server srv, const ecc_field *field, const ecc_curves *host_curves,
                                        uint64_t *ticket) {
    clear_error();
    if (!srv || !field || !host_curves || !ticket) return fail(ECC_ERR_INVALID_ARG, "NULL argument");
    FieldInfo fi;
    ecc_status s = validate_field(field, host_curves, &fi, true);
    if (s != ECC_OK) return s;
    if (!field->data) return fail(ECC_ERR_INVALID_ARG, "field data is NULL");
    int nch = 0;
    for (const int64_t *p : {host_curves->ec, host_curves->perimeter, host_curves->area, host_curves->volume})
        nch += p ? 1 : 0;
    auto *r = new Request();
    r->fi = fi;
    r->field = *field;
    r->host_out = *host_curves;
    r->nch = nch;
    r->field_bytes = (size_t)fi.cells * fi.elem_bytes;
    r->total_bytes = Arena::round(r->field_bytes) + (size_t)nch * fi.L * 8;
    if (Arena::round(r->total_bytes) > Arena::round(srv->cfg.hbm_budget_bytes)) {
        delete r;
        return fail(ECC_ERR_INVALID_ARG, "request larger than the server's memory budget");
    }
    if (field->thresholds) {
        r->thr.assign(field->thresholds, field->thresholds + fi.L);
        r->field.thresholds = r->thr.data();
    }
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) {
            delete r;
            return fail(ECC_ERR_INVALID_ARG, "server is shutting down");
        }
        if (srv->free_slots.empty() || !srv->dev.alloc(r->total_bytes, &r->off)) {
            delete r;
            return fail(ECC_ERR_BUSY, "no free slot or memory; retry after a poll");
        }
        r->slot = srv->free_slots.back();
        srv->free_slots.pop_back();
        r->ticket = srv->next_ticket++;
        r->field.data = srv->d_arena + r->off;
        srv->reqs[r->ticket] = r;
        ++srv->inflight;
    }
    // stage the field in its pinned range outside the lock (the range is ours);
    // large fields are copied by several threads
    srv->copier.copy(srv->h_arena + r->off, static_cast<const char *>(field->data), r->field_bytes);
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        r->state = kStaged;
        srv->staged.push_back(r);
    }
    srv->cv_work.notify_one();
    *ticket = r->ticket;
    return ECC_OK;
}

extern "C" ecc_status ecc_server_poll(ecc_server srv, uint64_t ticket, int32_t *done) {
    clear_error();
    if (!srv || !done) return fail(ECC_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return fail(ECC_ERR_INVALID_ARG, "unknown ticket");
    Request *r = it->second;
    if (r->state == kComplete || r->state == kFailed) {
        const ecc_status s = r->err;
        srv->reqs.erase(it);
        delete r;
        *done = 1;
        return s == ECC_OK ? ECC_OK : fail(s, "request failed");
    }
    *done = 0;
    return ECC_OK;
}

extern "C" ecc_status ecc_server_drain(ecc_server srv) {
    clear_error();
    if (!srv) return fail(ECC_ERR_INVALID_ARG, "NULL argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_work.notify_one();
    srv->cv_done.wait(lk, [srv] { return srv->inflight == 0; });
    return ECC_OK;
}

extern "C" ecc_status ecc_server_destroy(ecc_server srv) {
    clear_error();
    if (!srv) return ECC_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_one();
    if (srv->worker.joinable()) srv->worker.join();
    hipSetDevice(srv->ctx->device);
    hipDeviceSynchronize();
    release_server(srv);
    return ECC_OK;
}
