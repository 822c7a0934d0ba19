/*
 * All-levels oracle (O2) for EC, perimeter, area and volume curves.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only
 * tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg load the
 * shared library built from it.  It shares no code, header, table or constant
 * with the HIP library.
 *
 * What it computes (Laky & Zavala, Methodology section):
 *   - level index of a cell: the first filtration level l with value <= t_l
 *     (sublevel filtration, Eq. (2)); with identity levels t_l = l.  Cells
 *     outside the field and cells that never satisfy the test (values above
 *     the last threshold, NaN) are never active, the role of the paper's M+1
 *     sentinel in Algorithms 1 and 4.  Superlevel filtration (the mirror of
 *     Eq. (2)): the first l with value >= t_l over non-increasing t; with
 *     integer levels t_l = L - 1 - l.  Everything after the level index is
 *     the same for both directions.
 *   - The complex at level l is the closure of the active closed cells (text
 *     after Eq. (2)).  A lattice k-cell belongs to it exactly when one of the
 *     top cells containing it is active, i.e. from level min(level index of
 *     those top cells) on.  So the EC curve of Eq. (1) is the running sum over
 *     levels of sum_k (-1)^k (number of k-cells entering at that level).  This
 *     is the definition of chi counted for all levels at once, O(N + L).
 *   - 4-connected (2D) / 6-connected (3D) EC: the complex whose vertices are
 *     active cells, whose edges are face-adjacent active pairs, whose squares
 *     are fully active axis-plane 2x2 blocks and whose cubes are fully active
 *     2x2x2 blocks; such an element enters at the max level index of its
 *     cells.  Table 1's 4-C column is this complex's per-vertex share.
 *   - perimeter (2D) / surface (3D): unit lattice edges / faces with exactly
 *     one active neighbour; between levels min and max of its two cells.
 *   - area (2D) / volume (3D): number of active cells.
 *   - crease (3D "perimeter", Table 2 Perimeter column read as): sum over
 *     lattice edges of kappa(4 cells around the edge), kappa = 1 for one or
 *     three active, 2 for two diagonally opposite, else 0.
 *
 * Parallelisation: optional OpenMP over the slowest lattice axis with one
 * histogram per thread, summed at the end (no reordering of the arithmetic
 * beyond integer addition, which is exact).
 */
#include "ecc_oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* dtype codes accepted by this oracle */
#define OR_U8 1
#define OR_U16 2
#define OR_F32 3

/* return codes */
#define OR_OK 0
#define OR_BAD 1
#define OR_NOMEM 3

/* channels of a histogram row */
#define CH_EC 0
#define CH_PERIM 1
#define CH_AREA 2
#define CH_VOL 3
#define NCH 4

static double value_at(const void *data, int dtype, int64_t i) {
    switch (dtype) {
    case OR_U8: return (double)((const uint8_t *)data)[i];
    case OR_U16: return (double)((const uint16_t *)data)[i];
    default: return (double)((const float *)data)[i];
    }
}

/* first level l with float32(x) <= t[l] (superlevel: float32(x) >= t[l]);
 * L when none (also for NaN) */
static int32_t level_of(const void *data, int dtype, int64_t i, int32_t L, const float *t, int super) {
    if (t == NULL) {
        double v = value_at(data, dtype, i);
        if (super) /* integer levels t_l = L - 1 - l: first l with v >= L - 1 - l */
            return v >= (double)(L - 1) ? 0 : (int32_t)((double)(L - 1) - v);
        /* identity levels for integer fields: t_l = l */
        return v < (double)L ? (int32_t)v : L;
    }
    float x = (float)value_at(data, dtype, i);
    int32_t lo = 0, hi = L;
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (super ? (x >= t[mid]) : (x <= t[mid]))
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

static inline int32_t min2(int32_t a, int32_t b) { return a < b ? a : b; }
static inline int32_t max2(int32_t a, int32_t b) { return a > b ? a : b; }

/* histogram row accessors: hist[(level) * NCH + ch], level in [0, L] */
#define ADD(h, lvl, ch, v) ((h)[(int64_t)(lvl) * NCH + (ch)] += (v))

/* crease weight of four cells around an edge given cyclically */
static int kappa4(int a0, int a1, int a2, int a3) {
    int n = a0 + a1 + a2 + a3;
    if (n == 1 || n == 3) return 1;
    if (n == 2 && a0 == a2) return 2;
    return 0;
}

/* emit the changes of kappa over the levels of the 4 cells around an edge */
static void crease_events(int64_t *h, int32_t L, int32_t l0, int32_t l1, int32_t l2, int32_t l3) {
    int32_t lv[4] = {l0, l1, l2, l3};
    int prev = 0;
    int32_t last = -1;
    for (;;) {
        /* next distinct level above `last` */
        int32_t nxt = L;
        for (int k = 0; k < 4; ++k)
            if (lv[k] > last && lv[k] < nxt) nxt = lv[k];
        if (nxt >= L) break;
        int k0 = l0 <= nxt, k1 = l1 <= nxt, k2 = l2 <= nxt, k3 = l3 <= nxt;
        int cur = kappa4(k0, k1, k2, k3);
        ADD(h, nxt, CH_PERIM, cur - prev);
        prev = cur;
        last = nxt;
    }
}

/* ------------------------------------------------------------------------ */
/* 2D                                                                        */
/* ------------------------------------------------------------------------ */
static void run_2d(const int32_t *lam, int64_t h, int64_t w, int32_t L, int conn,
                   int64_t *hist_all, int n_threads) {
    const int64_t W = w + 2; /* padded row length; lam is (h+2) x (w+2) */
#define LAM(i, j) lam[((int64_t)(i) + 1) * W + ((int64_t)(j) + 1)]
#ifdef _OPENMP
#pragma omp parallel for num_threads(n_threads) schedule(static)
#endif
    for (int64_t i = 0; i <= h; ++i) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        int64_t *H = hist_all + (int64_t)tid * (L + 1) * NCH;
        for (int64_t j = 0; j <= w; ++j) {
            /* the four pixels around lattice vertex (i, j) */
            int32_t a = LAM(i - 1, j - 1), b = LAM(i - 1, j), c = LAM(i, j - 1), d = LAM(i, j);
            if (conn == 8) {
                /* vertex enters with its first pixel */
                ADD(H, min2(min2(a, b), min2(c, d)), CH_EC, 1);
                /* horizontal edge (i, j)-(i, j+1): pixels (i-1, j), (i, j) */
                if (j < w) ADD(H, min2(b, d), CH_EC, -1);
                /* vertical edge (i, j)-(i+1, j): pixels (i, j-1), (i, j) */
                if (i < h) ADD(H, min2(c, d), CH_EC, -1);
                /* face (i, j) */
                if (i < h && j < w) ADD(H, d, CH_EC, 1);
            } else {
                /* V-construction: pixel (i, j) is a vertex */
                if (i < h && j < w) {
                    ADD(H, d, CH_EC, 1);
                    if (j + 1 < w) ADD(H, max2(d, LAM(i, j + 1)), CH_EC, -1);
                    if (i + 1 < h) ADD(H, max2(d, LAM(i + 1, j)), CH_EC, -1);
                    if (i + 1 < h && j + 1 < w)
                        ADD(H, max2(max2(d, LAM(i, j + 1)), max2(LAM(i + 1, j), LAM(i + 1, j + 1))),
                            CH_EC, 1);
                }
            }
            /* perimeter: lattice edges with exactly one active pixel */
            if (j < w) {
                ADD(H, min2(b, d), CH_PERIM, 1);
                ADD(H, max2(b, d), CH_PERIM, -1);
            }
            if (i < h) {
                ADD(H, min2(c, d), CH_PERIM, 1);
                ADD(H, max2(c, d), CH_PERIM, -1);
            }
            if (i < h && j < w) ADD(H, d, CH_AREA, 1);
        }
    }
#undef LAM
}

/* ------------------------------------------------------------------------ */
/* 3D                                                                        */
/* ------------------------------------------------------------------------ */
static void run_3d(const int32_t *lam, int64_t d, int64_t h, int64_t w, int32_t L, int conn,
                   int want_crease, int64_t *hist_all, int n_threads) {
    const int64_t W = w + 2, HW = (h + 2) * (w + 2);
#define LAM(k, i, j) lam[((int64_t)(k) + 1) * HW + ((int64_t)(i) + 1) * W + ((int64_t)(j) + 1)]
#ifdef _OPENMP
#pragma omp parallel for num_threads(n_threads) schedule(static)
#endif
    for (int64_t k = 0; k <= d; ++k) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        int64_t *H = hist_all + (int64_t)tid * (L + 1) * NCH;
        for (int64_t i = 0; i <= h; ++i) {
            for (int64_t j = 0; j <= w; ++j) {
                /* the 8 voxels around lattice vertex (k, i, j); cXYZ with
                 * X = z offset, Y = y offset, Z = x offset (0 -> -1, 1 -> 0) */
                int32_t c000 = LAM(k - 1, i - 1, j - 1), c001 = LAM(k - 1, i - 1, j);
                int32_t c010 = LAM(k - 1, i, j - 1), c011 = LAM(k - 1, i, j);
                int32_t c100 = LAM(k, i - 1, j - 1), c101 = LAM(k, i - 1, j);
                int32_t c110 = LAM(k, i, j - 1), c111 = LAM(k, i, j);
                int in_x = j < w, in_y = i < h, in_z = k < d;
                if (conn == 26) {
                    /* vertex */
                    int32_t m = min2(min2(min2(c000, c001), min2(c010, c011)),
                                     min2(min2(c100, c101), min2(c110, c111)));
                    ADD(H, m, CH_EC, 1);
                    /* edges from (k,i,j): along x uses voxels with x index j */
                    if (in_x) ADD(H, min2(min2(c001, c011), min2(c101, c111)), CH_EC, -1);
                    if (in_y) ADD(H, min2(min2(c010, c011), min2(c110, c111)), CH_EC, -1);
                    if (in_z) ADD(H, min2(min2(c100, c101), min2(c110, c111)), CH_EC, -1);
                    /* faces: xy-face uses voxels (k-1, i, j) and (k, i, j) */
                    if (in_x && in_y) ADD(H, min2(c011, c111), CH_EC, 1);
                    if (in_x && in_z) ADD(H, min2(c101, c111), CH_EC, 1);
                    if (in_y && in_z) ADD(H, min2(c110, c111), CH_EC, 1);
                    /* cube */
                    if (in_x && in_y && in_z) ADD(H, c111, CH_EC, -1);
                } else if (in_x && in_y && in_z) {
                    /* V-construction anchored at voxel (k, i, j) = c111 */
                    int32_t px = LAM(k, i, j + 1), py = LAM(k, i + 1, j), pz = LAM(k + 1, i, j);
                    int32_t pxy = LAM(k, i + 1, j + 1), pxz = LAM(k + 1, i, j + 1);
                    int32_t pyz = LAM(k + 1, i + 1, j), pxyz = LAM(k + 1, i + 1, j + 1);
                    int okx = j + 1 < w, oky = i + 1 < h, okz = k + 1 < d;
                    ADD(H, c111, CH_EC, 1);
                    if (okx) ADD(H, max2(c111, px), CH_EC, -1);
                    if (oky) ADD(H, max2(c111, py), CH_EC, -1);
                    if (okz) ADD(H, max2(c111, pz), CH_EC, -1);
                    if (okx && oky) ADD(H, max2(max2(c111, px), max2(py, pxy)), CH_EC, 1);
                    if (okx && okz) ADD(H, max2(max2(c111, px), max2(pz, pxz)), CH_EC, 1);
                    if (oky && okz) ADD(H, max2(max2(c111, py), max2(pz, pyz)), CH_EC, 1);
                    if (okx && oky && okz)
                        ADD(H,
                            max2(max2(max2(c111, px), max2(py, pxy)),
                                 max2(max2(pz, pxz), max2(pyz, pxyz))),
                            CH_EC, -1);
                }
                /* surface: faces between the voxel (k,i,j) and its lower
                 * neighbour along each axis (border faces included) */
                if (in_x && in_y) { /* xy-face between (k-1,i,j) and (k,i,j) */
                    ADD(H, min2(c011, c111), CH_AREA, 1);
                    ADD(H, max2(c011, c111), CH_AREA, -1);
                }
                if (in_x && in_z) { /* xz-face between (k,i-1,j) and (k,i,j) */
                    ADD(H, min2(c101, c111), CH_AREA, 1);
                    ADD(H, max2(c101, c111), CH_AREA, -1);
                }
                if (in_y && in_z) { /* yz-face between (k,i,j-1) and (k,i,j) */
                    ADD(H, min2(c110, c111), CH_AREA, 1);
                    ADD(H, max2(c110, c111), CH_AREA, -1);
                }
                if (want_crease) {
                    /* edge along x at lattice (k, i): voxels vary in (z, y) */
                    if (in_x) crease_events(H, L, c001, c011, c111, c101);
                    /* edge along y: voxels vary in (z, x) */
                    if (in_y) crease_events(H, L, c010, c011, c111, c110);
                    /* edge along z: voxels vary in (y, x) */
                    if (in_z) crease_events(H, L, c100, c101, c111, c110);
                }
                if (in_x && in_y && in_z) ADD(H, c111, CH_VOL, 1);
            }
        }
    }
#undef LAM
}

/*
 * Public entry.  Host pointers only.  shape is {h, w} (2D) or {d, h, w} (3D),
 * C order, last axis contiguous.  thresholds: NULL for identity levels
 * (integer dtypes only) or n_levels non-decreasing float32 values
 * (non-increasing with superlevel != 0).  Output pointers of length n_levels
 * may be NULL when not wanted; volume and crease are 3D only (perimeter holds
 * the crease in 3D, area the surface).
 * Returns 0 on success, 1 on bad arguments, 3 when memory runs out.
 */
int ecc_oracle_o2(int ndim, const int64_t *shape, int dtype, const void *data,
                  int32_t n_levels, const float *thresholds, int32_t connectivity, int32_t superlevel,
                  int64_t *ec, int64_t *perimeter, int64_t *area, int64_t *volume,
                  int n_threads) {
    if (ndim != 2 && ndim != 3) return OR_BAD;
    if (dtype != OR_U8 && dtype != OR_U16 && dtype != OR_F32) return OR_BAD;
    if (n_levels < 1 || data == NULL) return OR_BAD;
    if (dtype == OR_F32 && thresholds == NULL) return OR_BAD;
    if (ndim == 2 && connectivity != 8 && connectivity != 4) return OR_BAD;
    if (ndim == 3 && connectivity != 26 && connectivity != 6) return OR_BAD;
    if (ndim == 2 && volume != NULL) return OR_BAD;
    if (superlevel != 0 && superlevel != 1) return OR_BAD;
    if (thresholds)
        for (int32_t l = 0; l < n_levels; ++l) {
            if (isnan(thresholds[l])) return OR_BAD;
            if (l > 0 && !superlevel && thresholds[l] < thresholds[l - 1]) return OR_BAD;
            if (l > 0 && superlevel && thresholds[l] > thresholds[l - 1]) return OR_BAD;
        }
    int64_t d = ndim == 3 ? shape[0] : 1;
    int64_t h = shape[ndim - 2], w = shape[ndim - 1];
    if (d < 1 || h < 1 || w < 1) return OR_BAD;
    if (n_threads < 1) n_threads = 1;
#ifndef _OPENMP
    n_threads = 1;
#endif
    const int32_t L = n_levels;

    /* level index of every cell, with a never-active ring around the field */
    int64_t pd = ndim == 3 ? d + 2 : 1, ph = h + 2, pw = w + 2;
    int32_t *lam = (int32_t *)malloc(sizeof(int32_t) * (size_t)(pd * ph * pw));
    if (!lam) return OR_NOMEM;
    for (int64_t t = 0; t < pd * ph * pw; ++t) lam[t] = L;
#ifdef _OPENMP
#pragma omp parallel for num_threads(n_threads) schedule(static)
#endif
    for (int64_t k = 0; k < d; ++k)
        for (int64_t i = 0; i < h; ++i)
            for (int64_t j = 0; j < w; ++j) {
                int64_t src = (k * h + i) * w + j;
                int64_t dst = ndim == 3 ? ((k + 1) * ph + (i + 1)) * pw + (j + 1) : (i + 1) * pw + (j + 1);
                lam[dst] = level_of(data, dtype, src, L, thresholds, superlevel);
            }

    int64_t *hist = (int64_t *)calloc((size_t)n_threads * (size_t)(L + 1) * NCH, sizeof(int64_t));
    if (!hist) {
        free(lam);
        return OR_NOMEM;
    }
    if (ndim == 2)
        run_2d(lam, h, w, L, connectivity, hist, n_threads);
    else
        run_3d(lam, d, h, w, L, connectivity, perimeter != NULL, hist, n_threads);
    free(lam);

    /* sum the per-thread histograms and take running sums over levels; the
     * row at index L (never active) is dropped */
    int64_t run[NCH] = {0, 0, 0, 0};
    for (int32_t l = 0; l < L; ++l) {
        for (int c = 0; c < NCH; ++c) {
            int64_t s = 0;
            for (int t = 0; t < n_threads; ++t) s += hist[((int64_t)t * (L + 1) + l) * NCH + c];
            run[c] += s;
        }
        if (ec) ec[l] = run[CH_EC];
        if (perimeter) perimeter[l] = run[CH_PERIM];
        if (ndim == 2) {
            if (area) area[l] = run[CH_AREA];
        } else {
            if (area) area[l] = run[CH_AREA];
            if (volume) volume[l] = run[CH_VOL];
        }
    }
    free(hist);
    return OR_OK;
}

int ecc_oracle_compute(const ecc_oracle_field *field, const ecc_oracle_curves *curves, int32_t n_threads) {
    if (field == NULL || curves == NULL) return OR_BAD;
    if (!curves->ec && !curves->perimeter && !curves->area && !curves->volume) return OR_BAD;
    if (field->ndim != 2 && field->ndim != 3) return OR_BAD;
    int32_t conn = field->connectivity;
    if (conn == 0) conn = field->ndim == 2 ? 8 : 26;
    return ecc_oracle_o2(field->ndim, field->shape, field->dtype, field->data, field->n_levels,
                         field->thresholds, conn, field->filtration, curves->ec, curves->perimeter,
                         curves->area, curves->volume, n_threads);
}
