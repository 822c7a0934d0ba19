// Internal declarations shared by the host runtime, the table builders and the
// kernel launchers of libecc.
#pragma once

#include <cstdint>
#include <string>

#include "../../include/ecc.h"

namespace ecc {

// ---- errors ---------------------------------------------------------------
ecc_status fail(ecc_status s, const std::string &msg);
void clear_error();

// ---- tables (ecc_tables.cpp) -----------------------------------------------
void vertex_table_2d(int connectivity, int32_t out[16][4]);
void vertex_table_3d(int connectivity, int32_t out[256][4]);
void cell_delta_table_2d(int connectivity, int32_t delta[256][3]);
// class of a 2D quadrant mask (bit a*2+b: pixel (i-1+a, j-1+b) of vertex
// (i, j)): -1 empty, 0 one pixel, 1 two adjacent, 2 two diagonal, 3 three, 4 four
int vertex_class_2d(int mask);
// per-cell change of the five class counts when the pixel enters, by the
// "entered before" pattern of its 8 neighbours (bit k = neighbour k)
void class_delta_table_2d(int32_t delta[256][5]);
// change of the summed kappa of the four 2x2 blocks at a pixel's corners when
// the pixel enters, by "entered before" pattern (-4..4); the 3D crease delta of
// a voxel is the sum of this over its three axis planes
void crease_delta_table_2d(int32_t delta[256]);
// class of a 3D octant mask (bit dx + 2dy + 4dz): -1 empty, else 0..20, the
// orbits under the cube's 48 symmetries ordered by (voxels, smallest mask)
int octant_class_3d(int mask);
constexpr int kNumClasses3D = 21;
// The kernels index per-cell tables by a permuted pattern: index bit i (i < 4)
// is neighbour 2i and bit 4+i neighbour 2i+1 of kNbr2.  Returns the kNbr2-order
// pattern of kernel index n.
int pattern_of_index(int n);
// The 2D kernels (ecc2d_stream, ecc2d_batch) and the z-marching 3D kernel
// (its layer and image patterns) form that index with the north bit
// complemented (the north relation enters as the complemented south relation
// of the row above): their tables hold at index n the entry of
// pattern_of_index(n ^ kNorthFlip2D).
constexpr int kNorthFlip2D = 1 << 4;
extern const int kNbr2[8][2];

// ---- histogram word layouts ---------------------------------------------------
// 2D bin word (uint64): [ ec+3 : 21 bits | perimeter+4 : 23 bits | count : 20 bits ].
// The per-cell biases make every field non-negative; a bin is decoded with the
// count n: ec = f0 - 3n, perimeter = f1 - 4n, area = n.  Valid while a
// workgroup adds at most kFlush2D cells between drains (ec field <= 4n < 2^21).
constexpr int kEcBias2 = 3, kPerBias2 = 4;
constexpr int kShiftPer2 = 21, kShiftCnt2 = 44;
constexpr int64_t kFlush2D = (1 << 19) - 1;
// 2D class-count bins (two uint64 words per level), for the counts of lattice
// vertices by quadrant class (one pixel, two adjacent, two diagonal, three,
// four).  Per-cell class deltas lie in [-4, 4] (four: [0, 4]):
//   word 0: [ one+4 : 21 | adjacent+4 : 21 | count : 22 ]
//   word 1: [ diagonal+4 : 21 | three+4 : 21 | four : 22 ]
// decoded with the count n (class c = field - 4n, four as is).  Valid while a
// workgroup adds at most kFlushCls cells between drains (8n < 2^21).
constexpr int kClsBias = 4, kClsShift1 = 21, kClsShift2 = 42;
constexpr int64_t kFlushCls = (1 << 18) - 1;
constexpr int kNumClasses2D = 5;
// 3D bin word (uint64): [ ec+7 : 22 bits | surface+6 : 22 bits | count : 20 bits ],
// crease in a second uint32 word as crease+12.  Valid while at most kFlush3D
// cells are added between drains: ec+7 <= 14 and surface+6 <= 12 per cell keep
// both fields below 2^22 (14 * 299000 < 2^22), the count below 2^20 and the
// crease word (<= 24 per cell) below 2^32.
constexpr int kEcBias3 = 7, kSurfBias3 = 6, kCreaseBias3 = 12;
constexpr int kShiftSurf3 = 22, kShiftCnt3 = 44;
constexpr int64_t kFlush3D = 299000;

// ---- level index of a value ---------------------------------------------------
enum LevelMode : int {
    LM_IDENTITY = 0,  // integer value v: level v if v < L, else never (L)
    LM_LUT = 1,       // integer value v: level lut[v] (built from thresholds on the device)
    LM_AFFINE = 2,    // float: thresholds close to t0 + l*step; guess, then exact correction
    LM_SEARCH = 3,    // float: binary search over the thresholds
};

struct LevelArgs {
    int32_t L;
    int32_t mode;
    const float *thr;     // device, L floats (LM_AFFINE / LM_SEARCH)
    const uint16_t *lut;  // device, 256 or 65536 entries (LM_LUT)
    float u0, inv_step;   // LM_AFFINE: u = fma(x, inv_step, u0) ~ (x - t_0) / step
    double u0d;           // LM_AFFINE: u0 before rounding to float
    float eps;            // LM_AFFINE: where the estimate is farther than eps from a
                          // level boundary it is the exact level; elsewhere the level is
                          // settled against the thresholds (level form, and bin form of
                          // the pass window at level 0)
    float eps_far;        // LM_AFFINE: the same for the bin form of any pass window
    uint32_t neg;         // 0, or the sign bit for the superlevel filtration: thr holds
                          // -t, every threshold comparison takes -x (x ^ neg), and
                          // inv_step already carries the sign (fma(x, -s, u0) =
                          // fma(-x, s, u0) exactly); level tables are built for -v
};

// bin of the first level of a pass window in the 2D kernels' LDS histograms
// (the bins below it are per-lane bins for cells below the window)
constexpr int kBinOff = 64;

// thresholds kept in LDS by the kernels when L is at most this
constexpr int kThrLds = 4096;

// ---- kernel launch descriptors ---------------------------------------------------
struct Launch2D {
    const void *data;
    int dtype;
    int64_t h, w;
    LevelArgs lv;
    int32_t lo, hi;             // level window [lo, hi) histogrammed by this pass
    const uint64_t *delta_lut;  // device, 256 packed per-cell deltas
    int32_t *partial;           // device, [3][L][grid]
    int grid;
    int64_t row_lo, row_hi;     // rows whose cells this launch emits (halo rows are read)
    bool accumulate;            // add to the partials instead of overwriting them
    bool classes;               // class counts: delta_lut holds 2 x 256 words, partial is [5][L][grid]
    // timing (hipEvent_t or NULL): the first launch's start and the last
    // launch's end are recorded by the dispatches themselves
    void *ev_start = nullptr, *ev_stop = nullptr;
    // atomic drain (curves only): int64 accumulators [kAccCopies][3][L] instead of partials
    int64_t *acc = nullptr;
    bool pack = false;  // packed perimeter and count (acc only, fields below kPackMaxCells)
};

size_t lds_bytes_2d(int window, bool classes);
// whether the field kernels lower a wave's priority as it progresses
// (default; environment ECC_PRIO=0 turns it off)
bool progress_prio();

// cells per lane along the contiguous axis (16 bytes of input per lane)
inline int vec_2d(int dtype) { return dtype == 1 ? 16 : (dtype == 2 ? 8 : 4); }
// how the 2D kernels load a row block of this field (kLoadElement = 0,
// kLoadVector = 1, kLoadAligned = 2)
int load_mode_2d(const void *data, int64_t h, int64_t w, int elem_bytes);

struct Launch3D {
    const void *data;
    int dtype;
    int64_t d, h, w;
    LevelArgs lv;
    int32_t lo, hi;
    const int64_t *vtab;  // device, 256 packed per-vertex contributions (x8 scale)
    int32_t *partial;     // device, [4][L][grid]
    int grid;
    bool want_crease;
    // z-marching kernel (no crease channel): its two per-pattern tables, else NULL
    const uint32_t *zm_tables;
    bool conn6;
    // z-marching kernel only: the planes [z_lo, z_hi) whose voxels this launch
    // emits (planes z_lo - 1 and z_hi are read when inside the field), and
    // whether to add to the partials instead of overwriting them
    int64_t z_lo, z_hi;
    bool accumulate;
    // z-marching kernel: the per-plane crease table when the crease channel
    // is wanted (it then comes along in the same launch), else NULL
    const uint32_t *crease_table;
    // timing, as in Launch2D
    void *ev_start = nullptr, *ev_stop = nullptr;
    // atomic drain (z-marching kernel): int64 accumulators [kAccCopies][4][L]
    int64_t *acc = nullptr;
    // surface and voxel count drained as one word into channel 2 (see
    // kPackSurf3); the merge must be told the same
    bool pack_surf = false;
};
// Packed drain of fields below 2^28 cells: the boundary channel of the
// accumulators (2D perimeter, channel 1; 3D surface, channel 2) takes
// (m + kPackBias n) + (n << kPackShift) in one atomic, m the boundary measure
// and n the cell count of the bin, and the count channel after it is left
// unused.  A cell changes the boundary by -4..4 (2D) or -6..6 (3D), so every
// sum over workgroups and copies stays exact: m + 6n <= 12n < 2^36, n < 2^28.
constexpr int kPackShift = 36, kPackBias = 6;
constexpr int64_t kPackMaxCells = (int64_t)1 << 28;

// 3D vertex class counts (ecc_k3d_cls.hip): one pass over the levels [lo, hi)
// of a volume; each workgroup adds its bins into the accumulator copy of its
// XCD.
struct Launch3DClasses {
    const void *data;
    int dtype;
    int64_t d, h, w;
    LevelArgs lv;
    int32_t lo, hi;
    const uint16_t *trans;  // device, [8][256]: corner c, block mask -> new class | old class << 8 (0xFF empty)
    int64_t *acc;           // device, [kAccCopies][kNumClasses3D][L] int64
    int grid;
    void *ev_start = nullptr, *ev_stop = nullptr;
};
int launch_classes_3d(const Launch3DClasses &a, void *stream);
// LDS of the class-count kernel besides its W x kNumClasses3D int32 bins
size_t lds_fixed_classes_3d();
// per-corner class transitions of the class-count kernel, [8][256] (host)
void class_transitions_3d(uint16_t out[8][256]);

// ---- batched 2D launch ----------------------------------------------------------
// One descriptor per field of the batch (device memory, rewritten every call).
struct BatchField2D {
    const void *data;
    int64_t h, w;
    int64_t *out[3];      // ec, perimeter, area (NULL = not wanted)
    int32_t *hist;        // [3][L] per-level deltas; zero between launches
    uint32_t *done;       // items of this field finished; zero between launches
    const float *thr;     // LM_AFFINE / LM_SEARCH thresholds (device)
    const uint16_t *lut;  // LM_LUT level table (device)
    int32_t L, n_items, conn_idx;        // conn_idx 0 = 8-C, 1 = 4-C
    uint32_t neg;                        // LevelArgs::neg
    float inv_step, cpass, eps, pad1;    // LM_AFFINE (cpass of the pass over all L <= 4096 levels)
};
// A work item: (strip, row) units [u0, u1) of one field, strip-major.
struct BatchItem {
    int32_t field, u0, u1, pad;
};
// A volume of a 3D batched launch, cut into tiles of tx x ty x tz voxels
// chosen per volume (tile_shape_3d), whose levels plus a one-voxel halo fit
// in kBatch3DTileElems LDS slots.
struct BatchField3D {
    const void *data;
    int64_t d, h, w;
    int64_t *out[4];      // ec, perimeter (crease), area (surface), volume; NULL = not wanted
    int32_t *hist;        // [4][L] per-level deltas; zero between launches
    uint32_t *done;       // items of this field finished; zero between launches
    const float *thr;     // LM_AFFINE / LM_SEARCH thresholds (device)
    const uint16_t *lut;  // LM_LUT level table (device)
    int32_t L, n_items, conn_idx;  // conn_idx 0 = 26-C, 1 = 6-C
    uint32_t neg;                  // LevelArgs::neg
    float u0, inv_step, eps;       // LM_AFFINE
    int32_t tiles_x, tiles_y;      // tiles along x and y
    int32_t tx, ty, tz;            // tile shape
    int32_t pad;
};
constexpr int kBatch3DTileElems = 12288;
// Largest field and level count the batched kernels take (others go through
// the single-field path); volumes above kBatch3DMaxCells give the single-field
// kernels enough work on their own.
constexpr int64_t kBatchMaxCells = int64_t(1) << 28;
constexpr int64_t kBatch3DMaxCells = int64_t(1) << 22;
constexpr int kBatchMaxLevels = 4096;
// Items of workgroup g are items[wg_first[g] .. wg_first[g+1]).
int launch_batch_2d(int dtype, int lm, const BatchField2D *fields, const BatchItem *items,
                    const int32_t *wg_first, int grid, const uint64_t *luts, int max_L, void *stream);
// vt3: [2][256] per-octant tables, 26-C then 6-C
int launch_batch_3d(int dtype, int lm, const BatchField3D *fields, const BatchItem *items,
                    const int32_t *wg_first, int grid, const int64_t *vt3, int max_L, void *stream);

// A 4D field's launch: the slab kernel over (virtual volume, tile range)
// items, then the kernel that combines the passes and scans.
struct Launch4D {
    const void *data;
    int dtype;
    int64_t a, d, h, w;
    LevelArgs lv;
    bool faces;  // face-adjacency complex (8-C) instead of the closure (80-C)
    const BatchItem *items;
    const int32_t *wg_first;
    int grid;
    const int64_t *vtab;  // 3D per-octant table: 26-C (closure) or 6-C (faces)
    int64_t *acc;         // [kAccCopies][6][L], zero; left at zero
    int64_t *totals;      // [3][L] scratch
    int64_t *out[3];      // ec, boundary, volume (NULL = not wanted)
    int tx, ty, tz, tiles_x, tiles_y;
};
int launch_4d(const Launch4D &g, void *stream);

// device-side launchers (ecc_k2d.hip, ecc_k3d.hip, ecc_kmerge.hip); return a hipError_t as int
int launch_2d(const Launch2D &a, void *stream);
int launch_3d(const Launch3D &a, void *stream);
// partials [nch][L][grid] int32 -> per-level totals -> running sums into the
// caller's curves (channels with a NULL output are skipped); `counter` is a
// zero-initialised device word that the kernel leaves at zero
int launch_merge(const int32_t *partial, int grid, int nch, int L, int64_t *const out[4],
                 int64_t *totals, unsigned *counter, void *stream);
int launch_level_lut(const float *thr, int L, int n_values, uint16_t *lut, bool neg, void *stream);
// zero `bytes` (a multiple of 16) of device memory at p with a fill kernel
int launch_zero(void *p, size_t bytes, void *stream);
// copies of the atomic drain's accumulators, [kAccCopies][nch][L] int64: one
// per XCD of the MI355X (a workgroup takes copy XCC_ID mod kAccCopies; the
// adds are device-scope atomics, so copies shared by XCDs stay exact)
constexpr int kAccCopies = 8;
// accumulators [copies][nch][L] -> totals -> running sums into the curves;
// leaves the accumulators at zero.  `totals` (device, at least nch x L int64,
// or NULL) holds the chunk totals when L is above 1024 and the merge runs as
// two kernels
int launch_merge_acc(int64_t *acc, int copies, int nch, int L, int64_t *const out[4], int64_t *totals,
                     unsigned *counter, void *stream, int pack_ch = -1);
// the same for up to 64 channels of at most 4096 levels, into rows[ch][L]
int launch_merge_acc_rows(int64_t *acc, int nch, int L, int64_t *rows, void *stream);
// whether the curve kernels (2D stream, 3D z-marching) drain their bins with
// atomics into per-XCD accumulators (default) instead of writing per-workgroup
// partials for a merge kernel to sum (environment ECC_DRAIN=partials)
bool atomic_drain();

// tile geometry used by the single-field kernels
constexpr int kWavesPerWG = 4;
// Waves per workgroup of the single-field 2D kernel: one 1024-thread
// workgroup per CU whose 16 waves share one LDS histogram, so that one drain
// per CU (not four) adds its bins into the accumulators.
constexpr int kWaves2D = 16;
constexpr int kTile3DX = 64, kTile3DY = 4, kTile3DZ = 16;
// z-marching 3D kernel: strips of 64 lanes x 4 cells, blocks of kZmTY rows
constexpr int kZmTY = 4, kZmStripX = 256, kZmCellsPerUnit = kZmStripX * kZmTY;
int zmarch_3d_columns(int64_t h, int64_t w);
// whether one z-plane per wave keeps the workgroup bins within kFlush3D
bool zmarch_3d_fits(int64_t h, int64_t w, int grid);
size_t lds_bytes_3d(int window, bool want_crease);

}  // namespace ecc
