// Host-side context and helpers of libecc (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "ecc_internal.h"
#include "ecc_levels.h"
#include "ecc_schedule.h"

namespace ecc {

constexpr int kMaxLevels = 65535;   // level indices are staged as u16 (L = never)
constexpr int kMaxWindow = 4096;    // levels histogrammed per pass (LDS budget)
constexpr size_t kThrCacheMax = 256;  // distinct threshold arrays kept on the device

struct FieldInfo {
    int ndim, dtype;
    int64_t d, h, w, cells;
    int L, conn;
    int elem_bytes;
    bool super;  // superlevel filtration
};

struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    ecc_status ensure(size_t need, const char *what);
    void release();
};

// A threshold array cached on the device (by content).  `ready` follows the
// last upload or level-table build, queued on `ready_stream`: work on any
// other stream waits for it before reading the arrays.  `last_use` follows
// the latest queued work that reads them, so that evicting the entry waits
// for that work only.
struct ThrEntry {
    int L = 0;
    std::vector<float> host;  // the caller's thresholds (the cache key, with `neg`)
    bool neg = false;         // superlevel: the device holds -t, the level tables map -v
    float *h_pinned = nullptr;
    float *d_thr = nullptr;
    uint16_t *d_lut8 = nullptr;
    uint16_t *d_lut16 = nullptr;
    bool affine = false;
    float u0 = 0.f, inv_step = 0.f, eps = 0.f, eps_far = 0.f;
    double u0d = 0.0;
    hipEvent_t ready = nullptr, last_use = nullptr;
    void *ready_stream = nullptr;
    bool used = false;
    uint64_t tick = 0;  // last fetch, for LRU eviction
};

struct Workspace {
    DevBuf partial, totals, acc;
    DevBuf items, first;  // 4D work items and their split over workgroups
    void release() {
        partial.release();
        totals.release();
        acc.release();
        items.release();
        first.release();
    }
};

struct BatchState;   // ecc_batch.hip
struct StreamState;  // ecc_streamed.hip

}  // namespace ecc

struct ecc_context_s {
    int device = 0;
    int n_cu = 0;
    std::string arch;
    std::mutex mu;
    uint64_t *d_delta2[2] = {nullptr, nullptr};  // 2D per-cell deltas, 8-C and 4-C
    int32_t h_delta2[2][256][3];
    int64_t *d_vtab3[2] = {nullptr, nullptr};    // 3D per-vertex table, 26-C and 6-C
    uint32_t *d_zm3[2] = {nullptr, nullptr};     // 3D z-marching tables, 26-C and 6-C
    uint64_t *d_cls2 = nullptr;                  // 2D per-cell class-count deltas, 2 x 256 words
    uint16_t *d_trans3 = nullptr;                // 3D class transitions per corner and octant mask, [8][256]
    size_t max_lds = 0;                          // LDS bytes one workgroup may use
    uint32_t *d_crease3 = nullptr;               // 3D crease by z-marching: per-plane deltas + 4
    std::vector<ecc::ThrEntry *> thr_cache;
    uint64_t thr_tick = 0;
    ecc::Workspace ws;
    hipEvent_t ws_event = nullptr;
    void *ws_stream = nullptr;
    bool ws_used = false;
    // While every call has queued its work on one stream (`solo_stream`),
    // stream order alone keeps the workspace and the cached thresholds safe
    // and no events are recorded per call (each record costs the device a
    // fence between kernels).  The first call on another stream waits for the
    // device once; from then on calls order their streams with events.
    bool one_stream = true;
    bool solo_set = false;
    void *solo_stream = nullptr;
    ecc::BatchState *batch = nullptr;
    ecc::StreamState *streamed = nullptr;  // ecc_streamed.hip
    // the atomic drain's accumulators (ws.acc) hold sums of a call whose merge
    // was never queued (an error path): they are cleared before the next use
    bool acc_dirty = false;
    void *d_counter = nullptr;  // merge kernel's completion ticket (kept at zero)
    void *d_tiny = nullptr;     // 256 B: padded copy of fields smaller than one vector load
    // allocation-free entry point: this device's scratch array, and a pinned
    // staging buffer for thresholds (65536 floats) reused once `stage_event`
    // (recorded after its last copy) has completed
    unsigned char *scratch = nullptr;
    float *h_stage = nullptr;
    hipEvent_t stage_event = nullptr;
    // kernel timing (ecc_profile_enable)
    bool prof_on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;
    size_t prof_used = 0;
};

namespace ecc {
ecc_status hip_fail(int err, const char *what);
ecc_status validate_field(const ecc_field *f, const ecc_curves *c, FieldInfo *info, bool curves_on_host);
void free_thresholds(ThrEntry *t);
ecc_status level_args(ecc_context ctx, const ecc_field *f, const FieldInfo &fi, void *stream, LevelArgs *lv);
// The thresholds that define the field's levels: the caller's array, or for an
// integer field with NULL thresholds under the superlevel filtration the
// implied t_l = L - 1 - l (written into `tmp`); NULL for identity sublevel
// levels.
const float *field_thresholds(const ecc_field *f, std::vector<float> &tmp);
// Superlevel thresholds as the device uses them: dst[l] = -t[l] (non-decreasing),
// so that the level of x is the sublevel level of -x.
void negate_thresholds(const float *t, int L, float *dst);
// Makes room in the threshold cache for the distinct (by content) arrays of
// `fields` that are not cached yet, so that fetching them all evicts none of
// them; fails when they are more than the cache holds.
ecc_status reserve_thresholds(ecc_context ctx, int n, const ecc_field *const *fields, void *stream);
// the distinct threshold arrays (by content) among `fields`
int count_distinct_thresholds(int n, const ecc_field *const *fields);
// records on `stream` that the work queued so far reads lv's threshold arrays
ecc_status note_threshold_use(ecc_context ctx, const LevelArgs &lv, void *stream);
// to be called before a call queues work on `stream` (see one_stream)
ecc_status use_stream(ecc_context ctx, void *stream);
ecc_status acquire_workspace(ecc_context ctx, void *stream);
ecc_status release_workspace(ecc_context ctx, void *stream);
ecc_status grow(ecc_context ctx, DevBuf &b, size_t need, const char *what);
ecc_status compute_one(ecc_context ctx, const ecc_field *f, const FieldInfo &fi, const ecc_curves *c, void *stream);
// launch geometry and buffer sizes of the single-field path
struct OnePlan {
    int grid, nch, win, k;
    bool zmarch, crease;
    size_t partial_bytes, totals_bytes;
};
OnePlan plan_one(ecc_context ctx, const FieldInfo &fi, const ecc_curves *c, const void *data);
ecc_status compute_core(ecc_context ctx, const ecc_field *f, const FieldInfo &fi, const ecc_curves *c,
                        const LevelArgs &lv, const OnePlan &p, int32_t *partial, int64_t *totals,
                        unsigned *counter, void *stream, bool timing, int64_t *acc = nullptr);
// address of the allocation-free entry point's scratch array on `device`
// (looked up once per device; the device must be current)
ecc_status noalloc_scratch(int device, unsigned char **out);
int pick_grid(ecc_context ctx, int64_t n_tiles, size_t lds_per_wg);
// workgroups of the 2D stream kernel for a field
int grid_2d(ecc_context ctx, const FieldInfo &fi, int window, bool classes);
// workgroups per CU of the 3D z-marching kernel for a field (ECC_ZM_WG_PER_CU
// overrides)
int zm_wg_per_cu(int dtype, int64_t w, const void *data, bool crease);
ecc_status merge_and_scan(ecc_context ctx, int grid, int nch, int L, int64_t *const outs[4], void *stream);
void destroy_batch_state(ecc_context ctx);
void destroy_stream_state(ecc_context ctx);
// the atomic drain's accumulators for nch channels of L levels (zero), grown
// and cleared as needed (may synchronise the device when it grows)
ecc_status acc_buffer(ecc_context ctx, int nch, int L, int64_t **acc, void *stream);
// the batched kernel that takes a field: 2, 3, or 0 for the single-field path
int batch_kind(const FieldInfo &fi);
bool batchable(const FieldInfo &fi);  // batch_kind(fi) != 0
// a field's batched-kernel descriptor without its histogram, ticket and item count
void fill_desc_2d(BatchField2D &d, const ecc_field &f, const ecc_curves &c, const FieldInfo &fi, const LevelArgs &lv);
void fill_desc_3d(BatchField3D &d, const ecc_field &f, const ecc_curves &c, const FieldInfo &fi, const LevelArgs &lv);
// records the start event of a timed launch on `stream` (no-op unless profiling)
ecc_status prof_begin(ecc_context ctx, void *stream, int *slot);
ecc_status prof_end(ecc_context ctx, void *stream, int slot);
// a pair of timing events for the launches of one field-reading pass, which
// the dispatches record themselves (kernel start and end, no launch overhead);
// both NULL unless profiling
ecc_status prof_events(ecc_context ctx, hipEvent_t *start, hipEvent_t *stop);
}  // namespace ecc
