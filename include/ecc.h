/*
 * ecc.h - Euler-characteristic curves of 2D/3D scalar fields on MI355X (gfx950).
 *
 * C ABI of libecc.so.  The operation is the one of Laky & Zavala, "A Fast and
 * Scalable Computational Topology Framework for the Euler Characteristic":
 *
 *   - a field of intensities (Methodology: pixels/voxels are the top cells of a
 *     cubical complex; Algorithms 1 and 3 take a w x h or w x h x d field),
 *   - a sublevel filtration over levels (Eq. (2): at level c a cell is active
 *     when its value <= c; including a cell includes its edges and vertices),
 *   - a connectivity (8/4 in 2D, 26 in 3D; Table 1, Table 2),
 *
 * in; and, for every level, the Euler characteristic chi = V - E + F - C of
 * Eq. (1) together with the perimeter, area and volume descriptors of Tables 1
 * and 2, out.  The curves are exact integers (int64).
 *
 * Conventions for every entry point:
 *   - Every function returns an ecc_status; nothing throws across the ABI.  On
 *     failure ecc_last_error() returns a message for the calling thread.
 *   - Arguments are validated before any work is queued; on a validation
 *     error nothing is written to any output.
 *   - Device work is queued on the caller's HIP stream (an hipStream_t passed
 *     as void*, NULL = the default stream) and is asynchronous: outputs are
 *     valid once that stream has completed the work.  Field data and output
 *     curves are DEVICE pointers owned by the caller and must stay valid until
 *     then.  Threshold arrays are HOST pointers, read during the call only.
 *   - One ecc_context may be used from several threads; calls on it are
 *     serialised internally.  Work queued on different streams through one
 *     context is ordered by the context (its workspace is reused).
 */
#ifndef ECC_H
#define ECC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ECC_OK = 0,
    ECC_ERR_INVALID_ARG = 1,   /* a documented precondition does not hold            */
    ECC_ERR_UNSUPPORTED = 2,   /* valid request outside what this build supports     */
    ECC_ERR_OUT_OF_MEMORY = 3, /* device or host allocation failed                   */
    ECC_ERR_DEVICE = 4,        /* a HIP runtime call failed                          */
    ECC_ERR_BUSY = 5           /* serving admission is full; retry later             */
} ecc_status;

typedef enum { ECC_U8 = 1, ECC_U16 = 2, ECC_F32 = 3 } ecc_dtype;

/* Direction of the filtration (ecc_field.filtration).
 *   ECC_SUBLEVEL    sets {x : f(x) <= c} over rising c, Eq. (2); the default (0).
 *   ECC_SUPERLEVEL  sets {x : f(x) >= c} over falling c: the mirror of Eq. (2),
 *                   the sublevel filtration of -f at -c. */
typedef enum { ECC_SUBLEVEL = 0, ECC_SUPERLEVEL = 1 } ecc_filtration;

typedef struct ecc_context_s *ecc_context;

/*
 * A field and its filtration.
 *   ndim          2 or 3.
 *   dtype         ECC_U8, ECC_U16 or ECC_F32.
 *   shape         2D {h, w}; 3D {d, h, w}; C order (last axis contiguous), each >= 1.
 *                 Cells number h*w (or d*h*w) <= 2^40.
 *   data          DEVICE pointer to the cells, caller-owned.
 *   n_levels      L >= 1: number of filtration levels, 0 .. L-1.
 *   thresholds    HOST pointer to L non-decreasing, non-NaN float32 values, or NULL.
 *                 With thresholds, a cell is active at level l when
 *                 float32(value) <= thresholds[l] (Eq. (2)).  NULL means the
 *                 integer levels t_l = l the paper uses (values are the level
 *                 index, Algorithm 1's increments at data[k]); NULL is allowed
 *                 for ECC_U8 / ECC_U16 only.
 *                 A cell that is active at no level (integer value >= L, float
 *                 value above the last threshold, NaN) never enters; this is
 *                 the paper's M+1 sentinel, not an error.  Cells outside the
 *                 field never enter either (the collar of the Methodology).
 *   connectivity  2D: 8 (vertex adjacency, the paper's default) or 4;
 *                 3D: 26 (the paper's default) or 6 (derived: the same
 *                 construction as Table 1's 4-C column one dimension up).
 *                 0 selects the default.
 *   filtration    ECC_SUBLEVEL (0: everything above) or ECC_SUPERLEVEL.  With
 *                 ECC_SUPERLEVEL the thresholds must be non-increasing (and
 *                 non-NaN) and a cell is active at level l when
 *                 float32(value) >= thresholds[l]; NULL thresholds (integer
 *                 fields) mean t_l = L - 1 - l, so level l holds the values
 *                 >= L - 1 - l and every value enters (values >= L - 1 at
 *                 level 0).  NaN never enters; +inf enters at level 0.  The
 *                 curves equal those of the sublevel filtration of -value with
 *                 thresholds -t_l, bit for bit.  Every entry point takes it.
 */
typedef struct {
    int32_t ndim;
    int32_t dtype;
    int64_t shape[3];
    const void *data;
    int32_t n_levels;
    int32_t connectivity;
    const float *thresholds;
    int32_t filtration;
} ecc_field;

/*
 * Output curves: DEVICE pointers to int64 arrays of length n_levels, caller-owned;
 * NULL = channel not wanted (at least one must be non-NULL).
 *   ec         Euler characteristic at each level (Eq. (1)).
 *   perimeter  2D: unit lattice edges with exactly one active pixel (Table 1).
 *              3D: crease measure, sum over lattice edges of kappa of the 4 voxels
 *              around it (1 for one or three active, 2 for two diagonal); the
 *              reading of Table 2's Perimeter column.
 *   area       2D: active pixels.  3D: unit faces with exactly one active voxel
 *              (Table 2 Area column).
 *   volume     3D only (must be NULL in 2D): active voxels.
 */
typedef struct {
    int64_t *ec;
    int64_t *perimeter;
    int64_t *area;
    int64_t *volume;
} ecc_curves;

/* Create a context on HIP device `device`: uploads the contribution tables,
 * queries the device.  *out receives the handle. */
ecc_status ecc_create(int device, ecc_context *out);

/* Wait for the context's queued work and free everything it owns. */
ecc_status ecc_destroy(ecc_context ctx);

/* Message of the last failing call on this thread ("" if none).  Valid until the
 * thread's next call into the library. */
const char *ecc_last_error(void);

/* Name of a status code. */
const char *ecc_status_string(ecc_status s);

/*
 * Check a request against every precondition of ecc_curves_compute without
 * queuing any work (host-only; touches neither the field data nor the curves).
 * Returns ECC_OK or the status ecc_curves_compute would return for it.
 */
ecc_status ecc_validate_field(const ecc_field *field, const ecc_curves *curves);

/*
 * EC, perimeter, area and volume curves of one field (one pass over the field:
 * level index, vertex-contribution deltas, per-workgroup histograms, merge and
 * prefix scan over levels).
 */
ecc_status ecc_curves_compute(ecc_context ctx, const ecc_field *field, const ecc_curves *curves,
                              void *stream);

/*
 * ecc_curves_compute for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, validation, asynchrony and results as ecc_curves_compute,
 * but every device buffer of the call (the merge ticket, the staged
 * thresholds, the value -> level table of integer fields with thresholds, the
 * per-level totals and the per-workgroup partials) lives in one static device
 * array of ECC_NOALLOC_SCRATCH_BYTES per GPU, held from the first context
 * created on that GPU until the process ends; the call makes no hipMalloc,
 * hipFree or other allocating call.
 *   - Thresholds are copied into the context's pinned staging buffer (made by
 *     ecc_create); the call first waits on the host until the previous
 *     staging copy of this context has run.
 *   - Every call of this entry point on one GPU (any context, stream or
 *     thread of the process) shares the array and keeps the last call's
 *     contents: calls that overlap on the device race; order them (one
 *     stream, or events).  The merge ticket is cleared by each call.
 *   - Limit: the accumulators (16 x channels x n_levels x 8 bytes; 2D fields
 *     and large 3D volumes) or, for small 3D volumes, per-workgroup partials
 *     (workgroups x 4 x n_levels x 4 bytes), plus totals (channels x n_levels
 *     x 8 bytes) plus 384 KiB must fit in ECC_NOALLOC_SCRATCH_BYTES: every 2D
 *     field and every large volume fits (65535 levels take 34 MiB), a small
 *     volume with tens of thousands of levels may not; those requests return
 *     ECC_ERR_UNSUPPORTED before any work is queued.
 *   - Kernel timing (ecc_profile_enable) does not record these launches.
 */
#define ECC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
ecc_status ecc_curves_compute_noalloc(ecc_context ctx, const ecc_field *field, const ecc_curves *curves,
                                      void *stream);

/*
 * Curves of a field that lives in HOST memory, streamed through the device in
 * slabs (the GPU counterpart of the paper's low-memory mode, Computational
 * Results on memory scaling and the Conclusions): the field is cut along its
 * slowest axis (rows in 2D, planes in 3D) into slabs that fit slab_bytes with
 * one halo row or plane on each side; each slab is copied on an internal stream
 * into one of two device buffers while the slab before it is histogrammed on
 * `stream`, and every slab adds to the same per-workgroup partials.  The curves
 * equal those of ecc_curves_compute on the same field.
 *
 * field:  as for ecc_curves_compute, except that data is a HOST pointer
 *         (pageable or pinned), read during the call only.
 * curves: HOST pointers, n_levels int64 each, NULL = channel not wanted.
 * slab_bytes: device bytes per slab buffer (two are allocated for the call and
 *         freed before it returns); 0 = 256 MiB.  Must hold three rows (2D) or
 *         planes (3D), else ECC_ERR_INVALID_ARG.
 * Blocking: returns once the curves are written (synchronises `stream`).  The
 * device memory used is two slab buffers plus the partials, whatever the
 * field's size.
 */
ecc_status ecc_curves_compute_streamed(ecc_context ctx, const ecc_field *field, const ecc_curves *curves,
                                       size_t slab_bytes, void *stream);

/*
 * The same for n fields of any mix of shapes, dtypes, level counts and
 * connectivities (the paper's dispatch of many small images, Discussion of the
 * microscopy case, and of many small volumes, its molecular-dynamics case).
 * fields[i] and curves[i] follow the single-field contract.  2D fields with at
 * most 4096 levels, and volumes with at most 4096 levels and 2^22 voxels, go
 * into one persistent launch per (dimension, dtype, level mode) group,
 * replayed from a captured graph; other fields (larger volumes, more levels)
 * run through the single-field path on the same stream after them.
 * The launch geometry comes from the context's tuning cache (see
 * ecc_batch_plan_tune), else defaults.
 * The threshold arrays of one call are uploaded once per distinct content; a
 * call may use at most 256 distinct arrays (ECC_ERR_UNSUPPORTED beyond, before
 * any work is queued).
 */
ecc_status ecc_curves_compute_batch(ecc_context ctx, int32_t n, const ecc_field *fields,
                                    const ecc_curves *curves, void *stream);

/*
 * A 4D field (the Conclusions name 4D data, such as hyperspectral images over
 * time, as the next step; the definitions of the Methodology carry over).
 *   dtype, data, n_levels, thresholds, filtration: as in ecc_field, with
 *                 n_levels at most 4096.
 *   shape         {a, d, h, w}, C order (w contiguous), each >= 1, at most
 *                 2^31 cells.
 *   connectivity  80 (the closure of the active hypercubes, the paper's
 *                 construction one dimension up; the default, also 0) or 8
 *                 (the complex of fully active blocks, as 4-C / 6-C).
 */
typedef struct {
    int32_t dtype;
    int64_t shape[4];
    const void *data;
    int32_t n_levels;
    int32_t connectivity;
    const float *thresholds;
    int32_t filtration;
} ecc_field4;

/*
 * Curves of a 4D field: ec (Eq. (1) over the cells of dimensions 0..4 of the
 * complex at each level), boundary (unit 3-faces with exactly one active
 * hypercube, the 4D counterpart of the perimeter and surface columns) and
 * volume (active hypercubes).  DEVICE int64 arrays of n_levels, caller-owned;
 * NULL = not wanted (at least one given).  Asynchronous on `stream`.
 * Errors: ECC_ERR_INVALID_ARG for a broken rule above or of ecc_field,
 * ECC_ERR_UNSUPPORTED for more than 4096 levels or 2^31 cells; nothing is
 * queued then.
 */
ecc_status ecc_curves_compute_4d(ecc_context ctx, const ecc_field4 *field, int64_t *ec, int64_t *boundary,
                                 int64_t *volume, void *stream);

/*
 * Autotuner: times the batched launch over candidate tile shapes and work splits
 * for this mix of fields (data must be valid device memory; the outputs of the
 * trial runs are discarded) and stores the fastest in the context's cache, keyed by
 * the exact mix (every field's shape, dtype, level count, level mode and
 * connectivity, in order): later calls with the same mix use it.  Synchronises
 * `stream`.  Optional.
 */
ecc_status ecc_batch_plan_tune(ecc_context ctx, int32_t n, const ecc_field *fields, void *stream);

/*
 * Host copies of the per-vertex contribution tables the kernels use, built from
 * the cell counts of Tables 1 and 2 (for tests):
 *   2D: out[16][4] = {4*EC(conn), 2*perimeter, 4*area, 0} per 2x2 mask, mask bit k
 *       = pixel (i-1,j-1), (i-1,j), (i,j-1), (i,j) for k = 0..3 around vertex (i,j).
 *   3D: out[256][4] = {8*EC(conn), 2*crease, 4*surface, 8*volume} per 2x2x2 mask,
 *       mask bit (dx + 2*dy + 4*dz) = voxel at offset (dz,dy,dx) in {0,1}^3.
 */
ecc_status ecc_vertex_table(int32_t ndim, int32_t connectivity, int32_t *out);

/*
 * Vertex class counts per level (the vertex-contribution map behind Table 1,
 * Table 2 and Eq. 4, the quantity the curves are weighted sums of).
 * The lattice vertices are the corners of the cells ((h+1) x (w+1) in 2D,
 * (d+1) x (h+1) x (w+1) in 3D); at level l the neighbourhood of a vertex (its
 * 2^n cells with level <= l, cells outside the field never in) falls in one
 * class; empty neighbourhoods are not counted.
 *   2D, 5 classes (the rows of Table 1):
 *     counts[0*L + l]  one pixel
 *     counts[1*L + l]  two pixels sharing an edge
 *     counts[2*L + l]  two pixels on a diagonal
 *     counts[3*L + l]  three pixels
 *     counts[4*L + l]  four pixels
 *   Any per-vertex descriptor of Table 1 at either connectivity is a fixed
 *   weighting of these, e.g. 4*EC(8-C) = one - 2*diagonal - three,
 *   4*EC(4-C) = one + 2*diagonal - three,
 *   2*perimeter = 2*one + 2*adjacent + 4*diagonal + 2*three.
 *   3D, 21 classes (the non-empty rows of Table 2): the orbits of the 2x2x2
 *   octant masks under the cube's 48 symmetries, numbered by (number of
 *   voxels, smallest mask in the orbit); ecc_vertex_class_table gives the
 *   class of every mask.  counts[c*L + l] as in 2D.
 *
 * field: as for ecc_curves_compute; the connectivity is checked but does not
 *        matter.
 * counts: DEVICE pointer, caller-owned, 5 * n_levels (2D) or 21 * n_levels (3D)
 *        int64, class-major as above; written only by the queued work.
 * Asynchronous on `stream`; same validation and error behaviour as
 * ecc_curves_compute (nothing is queued on error).
 */
ecc_status ecc_vertex_classes_compute(ecc_context ctx, const ecc_field *field, int64_t *counts, void *stream);

/*
 * Class of each vertex mask as ecc_vertex_classes_compute counts it, -1 for
 * the empty mask (for tests).  ndim 2: 16 masks, bits as for ecc_vertex_table,
 * classes 0..4; ndim 3: 256 masks, bit dx + 2*dy + 4*dz, classes 0..20.
 * out: HOST, 16 or 256 int32.
 */
ecc_status ecc_vertex_class_table(int32_t ndim, int32_t *out);

/*
 * Kernel timing for measurement.  While enabled, the context records a pair of
 * HIP events around the launches of each field-reading pass (the kernels that
 * read the field from HBM: one, or in 3D with the crease channel two; not the
 * merge and scan kernels that follow) on the stream the launches go to.  ecc_profile_read waits for the
 * recorded events, returns the summed elapsed milliseconds and the number of
 * launches, and forgets them when `reset` is non-zero.  Enabling it adds two
 * event records per launch and nothing else.
 */
ecc_status ecc_profile_enable(ecc_context ctx, int32_t on);
ecc_status ecc_profile_read(ecc_context ctx, double *total_ms, int64_t *launches, int32_t reset);

/* ---------------------------------------------------------------------------
 * Serving: a request loop with continuous batching (the paper's real-time use,
 * Discussion: many small images per second).
 *
 * At creation the server reserves a device arena of hbm_budget_bytes, a pinned
 * host arena of the same size for staging and results and max_slots slots, and
 * starts a worker thread on the context's device.  A request is admitted when a
 * slot is free and its field plus curves fit in the arena (first fit); its field
 * is staged in pinned memory during the submit, copied to the device on a copy
 * stream, and computed as soon as it has landed:
 * all ready requests the batched kernels take (2D fields and volumes of at
 * most 2^22 voxels with at most 4096 levels; up to max_batch, and at most 256
 * distinct threshold arrays; the rest join the next launch) in one launch of
 * the batched kernels, others (larger volumes, more than 4096 levels) through
 * the single-field path on a second stream.  Requests submitted while earlier ones run join the next launch.
 * Results go back to pinned memory and then to the caller's host arrays, and
 * the request's slot and memory are released.
 * ------------------------------------------------------------------------- */
typedef struct ecc_server_s *ecc_server;

typedef struct {
    size_t hbm_budget_bytes; /* device bytes for resident request fields + curves */
    int32_t max_slots;       /* requests resident at once (1..65536)              */
    int32_t max_batch;       /* requests per batched launch (<= max_slots)        */
} ecc_server_config;

/* Allocates the arenas (device and pinned host, hbm_budget_bytes each) and
 * starts the worker.  ECC_ERR_INVALID_ARG for a config outside the ranges
 * above; ECC_ERR_OUT_OF_MEMORY when the arenas cannot be allocated. */
ecc_status ecc_server_create(ecc_context ctx, const ecc_server_config *cfg, ecc_server *out);
/*
 * A request: field->data is a HOST pointer (copied into the pinned staging
 * arena before this returns, so the caller may reuse it); host_curves are HOST
 * arrays of length n_levels (NULL = not wanted, as in ecc_curves) that must
 * stay valid until the request is reported done.  Thresholds are copied.
 * ECC_ERR_BUSY when no slot is free or the arena has no room right now (retry
 * after a poll); ECC_ERR_INVALID_ARG when the request is malformed or larger
 * than the whole budget.  Thread-safe.
 */
ecc_status ecc_server_submit(ecc_server srv, const ecc_field *field, const ecc_curves *host_curves,
                             uint64_t *ticket);
/* *done = 1 once the request's host curves are written (the ticket is then
 * forgotten: polling it again is ECC_ERR_INVALID_ARG), 0 while pending.  A
 * request that failed reports *done = 1 and returns its error status. */
ecc_status ecc_server_poll(ecc_server srv, uint64_t ticket, int32_t *done);
/* Block until every submitted request has completed. */
ecc_status ecc_server_drain(ecc_server srv);
/* Drain, stop the worker and free the server and its arenas. */
ecc_status ecc_server_destroy(ecc_server srv);

#ifdef __cplusplus
}
#endif
#endif /* ECC_H */
