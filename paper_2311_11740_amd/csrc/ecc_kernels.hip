// HIP kernels for gfx950: EC / perimeter / area / volume curves of one field.
//
// Method (Laky & Zavala, Methodology): every lattice vertex contributes a
// fixed share of the EC, perimeter, area and volume that depends only on which
// of the 2^n cells around it are active (Tables 1 and 2).  Over a sublevel
// filtration (Eq. (2)) a vertex's share only changes when one of its cells
// enters, so the curves are running sums over levels of a histogram of changes
// (the change-tracking idea the paper adopts, O(N + levels)).  Here each change
// is charged to the cell that causes it: when cell p enters (cells ordered by
// level, ties by position), each vertex at a corner of p moves from its mask
// without p to its mask with p.  The sum of those differences, the cell's
// delta, depends only on which of p's neighbours entered before p.
//
// Kernel layout:
//   * one workgroup = 256 threads = 4 wave64s; persistent grid, each
//     workgroup takes a contiguous range of tiles (XCD-aware numbering so
//     neighbouring tiles share an L2);
//   * a tile plus a one-cell halo is read from HBM (coalesced along the
//     contiguous axis), mapped to level indices once, and staged in LDS as u16;
//   * each thread marches a column of the tile, keeping its 3x3 (2D) or 3x3x3
//     (3D) window of levels in registers, forms the "entered before p" pattern
//     and adds the cell's packed delta to an LDS histogram with one 64-bit
//     atomic (fields biased to stay non-negative, see ecc_internal.h);
//   * histograms are drained into a per-workgroup slice of a partials buffer
//     (no global atomics), merged by ecc_reduce and prefix-summed by ecc_scan.
#include <hip/hip_runtime.h>

#include "ecc_internal.h"

namespace ecc {

// ---------------------------------------------------------------------------
// level index: first l with value <= t_l (Eq. (2)); L = never active
// ---------------------------------------------------------------------------
template <int LM>
__device__ __forceinline__ uint32_t level_of_float(float x, const LevelArgs &a, const float *thr) {
    const int L = a.L;
    if (!(x == x)) return (uint32_t)L;  // NaN never enters
    int g;
    if constexpr (LM == LM_AFFINE) {
        const float u = (x - a.t0) * a.inv_step;
        if (u < -1.0f) return 0u;
        if (u >= (float)L + 1.0f) return (uint32_t)L;
        const float fu = floorf(u);
        const float fr = u - fu;
        g = (int)fu + 1;
        if (g > L) g = L;
        if (fr >= a.eps && fr <= 1.0f - a.eps) return (uint32_t)g;
        // close to a threshold: settle against the caller's values so that
        // t[g-1] < x <= t[g] (with t[-1] = -inf, t[L] = +inf)
        if (g < 0) g = 0;
        while (g > 0 && x <= thr[g - 1]) --g;
        while (g < L && !(x <= thr[g])) ++g;
    } else {
        int lo = 0, hi = L;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (x <= thr[mid])
                hi = mid;
            else
                lo = mid + 1;
        }
        g = lo;
    }
    return (uint32_t)g;
}

template <typename T, int LM>
__device__ __forceinline__ uint32_t level_of(T v, const LevelArgs &a, const float *thr) {
    if constexpr (LM == LM_IDENTITY) {
        const uint32_t u = (uint32_t)v;
        return u < (uint32_t)a.L ? u : (uint32_t)a.L;
    } else if constexpr (LM == LM_LUT) {
        return a.lut[(uint32_t)v];
    } else {
        return level_of_float<LM>((float)v, a, thr);
    }
}

__device__ __forceinline__ int xcd_order(int bid, int G) {
    // workgroups are dispatched round-robin over the 8 XCDs; renumber them so
    // that each XCD holds a contiguous block of workgroup ids (neighbouring
    // rows and tiles then share an L2)
    return (G & 7) == 0 ? (bid & 7) * (G >> 3) + (bid >> 3) : bid;
}

// ---------------------------------------------------------------------------
// 2D: row streaming
// ---------------------------------------------------------------------------
// One wave owns a strip of 64*VEC columns (VEC cells per lane, 16 bytes of
// input per lane and row) and walks down a run of rows, keeping the level
// indices of three rows (above, current, below) in registers.  The cells left
// and right of a lane's run come from the neighbouring lanes (ds_bpermute);
// lanes 0 and 63 read the strip's halo columns themselves.  Raw rows are
// fetched PF rows ahead into a register ring so that several 1 KiB row loads
// per wave are in flight.
template <typename T>
struct Elem;
template <>
struct Elem<uint8_t> {
    static constexpr int VEC = 16;
    __device__ static uint32_t get(const uint32_t (&w)[4], int i) { return (w[i >> 2] >> (8 * (i & 3))) & 0xFFu; }
};
template <>
struct Elem<uint16_t> {
    static constexpr int VEC = 8;
    __device__ static uint32_t get(const uint32_t (&w)[4], int i) { return (w[i >> 1] >> (16 * (i & 1))) & 0xFFFFu; }
};
template <>
struct Elem<float> {
    static constexpr int VEC = 4;
    __device__ static uint32_t get(const uint32_t (&w)[4], int i) { return w[i]; }
};

template <typename T>
__device__ __forceinline__ T as_value(uint32_t bits) {
    if constexpr (sizeof(T) == 4)
        return __uint_as_float(bits);
    else
        return (T)bits;
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct RawRow {
    uint32_t w[4];  // 16 bytes: VEC raw elements of this lane
    uint32_t halo;  // lane 0: element left of the strip; lane 63: right of it
    bool valid;     // row inside the field
};

template <typename T, bool ALIGNED>
__device__ __forceinline__ void fetch_row(const T *__restrict__ data, int64_t r, int64_t h, int64_t w,
                                          int64_t xs, int64_t x0, int lane, RawRow &raw) {
    constexpr int VEC = Elem<T>::VEC;
    raw.valid = r >= 0 && r < h;
    if (!raw.valid) return;
    const T *row = data + r * w;
    if (ALIGNED && x0 + VEC <= w) {
        const u32x4 q = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(row + x0));
        raw.w[0] = q.x; raw.w[1] = q.y; raw.w[2] = q.z; raw.w[3] = q.w;
    } else {
        raw.w[0] = raw.w[1] = raw.w[2] = raw.w[3] = 0;
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
            if (x0 + i < w) {
                uint32_t bits;
                if constexpr (sizeof(T) == 4)
                    bits = __float_as_uint(row[x0 + i]);
                else
                    bits = (uint32_t)row[x0 + i];
                constexpr int per = 4 / sizeof(T);
                raw.w[i / per] |= bits << (8 * sizeof(T) * (i % per));
            }
        }
    }
    raw.halo = 0;
    if (lane == 0 && xs > 0) {
        if constexpr (sizeof(T) == 4) raw.halo = __float_as_uint(row[xs - 1]);
        else raw.halo = (uint32_t)row[xs - 1];
    }
    if (lane == 63 && xs + 64 * VEC < w) {
        if constexpr (sizeof(T) == 4) raw.halo = __float_as_uint(row[xs + 64 * VEC]);
        else raw.halo = (uint32_t)row[xs + 64 * VEC];
    }
}

// level indices of a fetched row: lam[1..VEC] own cells, lam[0] / lam[VEC+1]
// the cells left of the first and right of the last
template <typename T, int LM>
__device__ __forceinline__ void convert_row(const RawRow &raw, int64_t w, int64_t xs, int64_t x0, int lane,
                                            const LevelArgs &lv, const float *thr,
                                            uint32_t (&lam)[Elem<T>::VEC + 2]) {
    constexpr int VEC = Elem<T>::VEC;
    const uint32_t L = (uint32_t)lv.L;
#pragma unroll
    for (int i = 0; i < VEC; ++i)
        lam[i + 1] = (raw.valid && x0 + i < w) ? level_of<T, LM>(as_value<T>(Elem<T>::get(raw.w, i)), lv, thr) : L;
    uint32_t left = __shfl_up(lam[VEC], 1);
    uint32_t right = __shfl_down(lam[1], 1);
    if (lane == 0) left = (raw.valid && xs > 0) ? level_of<T, LM>(as_value<T>(raw.halo), lv, thr) : L;
    if (lane == 63) right = (raw.valid && xs + 64 * VEC < w) ? level_of<T, LM>(as_value<T>(raw.halo), lv, thr) : L;
    lam[0] = left;
    lam[VEC + 1] = right;
}

__device__ __forceinline__ void drain_2d(uint64_t *hist, int W, int lo, int L, int32_t *slot,
                                         bool first) {
    for (int b = threadIdx.x; b < W; b += blockDim.x) {
        const uint64_t v = hist[b];
        hist[b] = 0;
        const int64_t n = (int64_t)(v >> kShiftCnt2);
        const int64_t per = (int64_t)((v >> kShiftPer2) & ((1ull << (kShiftCnt2 - kShiftPer2)) - 1)) -
                            kPerBias2 * n;
        const int64_t ec = (int64_t)(v & ((1ull << kShiftPer2) - 1)) - kEcBias2 * n;
        int32_t *s0 = slot + lo + b, *s1 = slot + L + lo + b, *s2 = slot + 2 * L + lo + b;
        if (first) {
            *s0 = (int32_t)ec;
            *s1 = (int32_t)per;
            *s2 = (int32_t)n;
        } else {
            *s0 += (int32_t)ec;
            *s1 += (int32_t)per;
            *s2 += (int32_t)n;
        }
    }
}

template <typename T, int LM, bool ALIGNED, int PF>
__global__ void __launch_bounds__(256)
    ecc2d_stream(const T *__restrict__ data, int64_t h, int64_t w, LevelArgs lv, int32_t lo,
                 int32_t hi, const uint64_t *__restrict__ delta_lut, int32_t *__restrict__ partial,
                 int64_t row_lo, int64_t row_hi, int64_t n_segs, int64_t seg_rows, int64_t n_items,
                 int accumulate) {
    constexpr int VEC = Elem<T>::VEC;
    constexpr int CW = 64 * VEC;
    extern __shared__ uint64_t smem[];
    __shared__ uint64_t dl[256];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int W = hi - lo;
    const int L = lv.L;
    uint64_t *hist = smem;
    const float *thr = lv.thr;
    if constexpr (LM == LM_AFFINE || LM == LM_SEARCH) {
        if (L <= kThrLds) {
            float *t = reinterpret_cast<float *>(smem + W);
            for (int i = tid; i < L; i += 256) t[i] = lv.thr[i];
            thr = t;
        }
    }
    dl[tid] = delta_lut[tid];
    for (int b = tid; b < W; b += 256) hist[b] = 0;
    __syncthreads();

    const int G = gridDim.x;
    const int wg = xcd_order(blockIdx.x, G);
    const int64_t gw = (int64_t)wg * kWavesPerWG + wave, NW = (int64_t)G * kWavesPerWG;
    const int64_t i_beg = n_items * gw / NW, i_end = n_items * (gw + 1) / NW;

    for (int64_t item = i_beg; item < i_end; ++item) {
        const int64_t strip = item / n_segs, seg = item % n_segs;
        const int64_t ra = row_lo + seg * seg_rows;
        const int64_t rb = ra + seg_rows < row_hi ? ra + seg_rows : row_hi;
        const int64_t xs = strip * CW, x0 = xs + (int64_t)lane * VEC;

        uint32_t up[VEC + 2], mid[VEC + 2], dn[VEC + 2];
        {
            RawRow r0, r1;
            fetch_row<T, ALIGNED>(data, ra - 1, h, w, xs, x0, lane, r0);
            fetch_row<T, ALIGNED>(data, ra, h, w, xs, x0, lane, r1);
            convert_row<T, LM>(r0, w, xs, x0, lane, lv, thr, up);
            convert_row<T, LM>(r1, w, xs, x0, lane, lv, thr, mid);
        }
        RawRow ring[PF];
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            ring[k].valid = false;
            if (ra + 1 + k <= rb) fetch_row<T, ALIGNED>(data, ra + 1 + k, h, w, xs, x0, lane, ring[k]);
        }
        for (int64_t r0 = ra; r0 < rb; r0 += PF) {
#pragma unroll
            for (int k = 0; k < PF; ++k) {
                const int64_t r = r0 + k;  // current row; ring[k] holds row r + 1
                if (r < rb) {
                    convert_row<T, LM>(ring[k], w, xs, x0, lane, lv, thr, dn);
                    if (r + 1 + PF <= rb)
                        fetch_row<T, ALIGNED>(data, r + 1 + PF, h, w, xs, x0, lane, ring[k]);
#pragma unroll
                    for (int j = 1; j <= VEC; ++j) {
                        const uint32_t p = mid[j];
                        if (p - (uint32_t)lo < (uint32_t)W) {
                            // a neighbour earlier in memory order precedes p on
                            // a tie, a later one does not
                            const uint32_t pat = (uint32_t)(up[j - 1] <= p) | (uint32_t)(up[j] <= p) << 1 |
                                                 (uint32_t)(up[j + 1] <= p) << 2 | (uint32_t)(mid[j - 1] <= p) << 3 |
                                                 (uint32_t)(mid[j + 1] < p) << 4 | (uint32_t)(dn[j - 1] < p) << 5 |
                                                 (uint32_t)(dn[j] < p) << 6 | (uint32_t)(dn[j + 1] < p) << 7;
                            atomicAdd((unsigned long long *)&hist[p - lo], (unsigned long long)dl[pat]);
                        }
                    }
#pragma unroll
                    for (int j = 0; j < VEC + 2; ++j) {
                        up[j] = mid[j];
                        mid[j] = dn[j];
                    }
                }
            }
        }
    }
    __syncthreads();
    drain_2d(hist, W, lo, L, partial + (int64_t)wg * 3 * L, accumulate == 0);
}

// ---------------------------------------------------------------------------
// 3D (generic: every channel, table lookups over the 8 corner blocks)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void drain_3d(uint64_t *hist, uint32_t *hc, bool crease, int W, int lo,
                                         int L, int32_t *slot, bool first) {
    for (int b = threadIdx.x; b < W; b += blockDim.x) {
        const uint64_t v = hist[b];
        hist[b] = 0;
        const int64_t n = (int64_t)(v >> kShiftCnt3);
        const int64_t surf = (int64_t)((v >> kShiftSurf3) & ((1ull << (kShiftCnt3 - kShiftSurf3)) - 1)) -
                             kSurfBias3 * n;
        const int64_t ec = (int64_t)(v & ((1ull << kShiftSurf3) - 1)) - kEcBias3 * n;
        int64_t cr = 0;
        if (crease) {
            cr = (int64_t)hc[b] - kCreaseBias3 * n;
            hc[b] = 0;
        }
        int32_t *s = slot + lo + b;
        if (first) {
            s[0] = (int32_t)ec;
            s[L] = (int32_t)cr;
            s[2 * L] = (int32_t)surf;
            s[3 * L] = (int32_t)n;
        } else {
            s[0] += (int32_t)ec;
            s[L] += (int32_t)cr;
            s[2 * L] += (int32_t)surf;
            s[3 * L] += (int32_t)n;
        }
    }
}

template <typename T, int LM, bool CREASE>
__global__ void __launch_bounds__(256)
    ecc3d_tile(const T *__restrict__ data, int64_t d, int64_t h, int64_t w, LevelArgs lv,
               int32_t lo, int32_t hi, const int64_t *__restrict__ vtab,
               int32_t *__restrict__ partial, int64_t tiles_x, int64_t tiles_y, int64_t n_tiles,
               int flush_tiles) {
    constexpr int TX = kTile3DX, TY = kTile3DY, TZ = kTile3DZ;
    constexpr int SX = TX + 2, SY = TY + 2, SZ = TZ + 2;
    extern __shared__ uint64_t smem[];
    __shared__ int64_t vt[256];
    __shared__ uint16_t lam[SZ][SY][SX];

    const int t = threadIdx.x;
    const int W = hi - lo;
    const int L = lv.L;
    uint64_t *hist = smem;
    uint32_t *hc = reinterpret_cast<uint32_t *>(smem + W);
    const int G = gridDim.x;
    const int wg = xcd_order(blockIdx.x, G);
    const int64_t t_beg = n_tiles * wg / G, t_end = n_tiles * (wg + 1) / G;

    vt[t] = vtab[t];
    for (int b = t; b < W; b += 256) {
        hist[b] = 0;
        if (CREASE) hc[b] = 0;
    }
    int32_t *slot = partial + (int64_t)wg * 4 * L;
    bool first = true;
    int since = 0;
    const int lx = t % TX, ly = t / TX;
    __syncthreads();

    for (int64_t tile = t_beg; tile < t_end; ++tile) {
        const int64_t x0 = (tile % tiles_x) * TX;
        const int64_t y0 = ((tile / tiles_x) % tiles_y) * TY;
        const int64_t z0 = (tile / (tiles_x * tiles_y)) * TZ;
        for (int e = t; e < SZ * SY * SX; e += 256) {
            const int xx = e % SX, rest = e / SX;
            const int yy = rest % SY, zz = rest / SY;
            const int64_t x = x0 - 1 + xx, y = y0 - 1 + yy, z = z0 - 1 + zz;
            uint32_t l = (uint32_t)L;
            if (x >= 0 && x < w && y >= 0 && y < h && z >= 0 && z < d)
                l = level_of<T, LM>(data[(z * h + y) * w + x], lv, lv.thr);
            lam[zz][yy][xx] = (uint16_t)l;
        }
        __syncthreads();
        if (x0 + lx < w && y0 + ly < h) {
            // 3x3x3 window: win[k], k = (dz+1)*9 + (dy+1)*3 + (dx+1)
            uint32_t win[27];
#pragma unroll
            for (int pz = 0; pz < 2; ++pz)
#pragma unroll
                for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                    for (int dx = 0; dx < 3; ++dx) win[9 + pz * 9 + dy * 3 + dx] = lam[pz][ly + dy][lx + dx];
            const int planes = (int)(d - z0 < TZ ? d - z0 : TZ);
            for (int z = 0; z < planes; ++z) {
#pragma unroll
                for (int k = 0; k < 18; ++k) win[k] = win[k + 9];
#pragma unroll
                for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                    for (int dx = 0; dx < 3; ++dx) win[18 + dy * 3 + dx] = lam[z + 2][ly + dy][lx + dx];
                const uint32_t p = win[13];
                if (p - (uint32_t)lo >= (uint32_t)W) continue;
                // bit k set when neighbour k entered before p (earlier in memory
                // order wins ties); the centre bit stands for p itself
                uint32_t P = 1u << 13;
#pragma unroll
                for (int k = 0; k < 27; ++k) {
                    if (k == 13) continue;
                    const bool pr = k < 13 ? (win[k] <= p) : (win[k] < p);
                    P |= (uint32_t)pr << k;
                }
                // corner (cz,cy,cx) of p: its 2x2x2 block holds the neighbours
                // with offsets in {c-1, c} per axis; gather them into the
                // octant mask (bit bx + 2by + 4bz), with and without p
                int64_t acc = 0;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int cx = c & 1, cy = c >> 1 & 1, cz = c >> 2;
                    const uint32_t y = P >> (cz * 9 + cy * 3 + cx);
                    const uint32_t m1 = (y & 3u) | ((y >> 1) & 0xCu) | ((y >> 5) & 0x30u) | ((y >> 6) & 0xC0u);
                    const uint32_t m0 = m1 & ~(1u << (7 - c));
                    acc += vt[m1] - vt[m0];
                }
                // four signed 16-bit fields, each eight times the cell's delta
                const int64_t f0 = (int16_t)(acc & 0xFFFF);
                acc = (acc - f0) >> 16;
                const int64_t f1 = (int16_t)(acc & 0xFFFF);
                acc = (acc - f1) >> 16;
                const int64_t f2 = (int16_t)(acc & 0xFFFF);
                const int64_t f3 = (acc - f2) >> 16;
                const int64_t ec = f0 >> 3, cr = f1 >> 3, surf = f2 >> 3;
                (void)f3;  // volume delta is 1 for every cell; it is the count field
                const uint64_t word = (uint64_t)(ec + kEcBias3) |
                                      (uint64_t)(surf + kSurfBias3) << kShiftSurf3 |
                                      1ull << kShiftCnt3;
                atomicAdd((unsigned long long *)&hist[p - lo], (unsigned long long)word);
                if (CREASE) atomicAdd(&hc[p - lo], (uint32_t)(cr + kCreaseBias3));
            }
        }
        __syncthreads();
        if (++since >= flush_tiles) {
            drain_3d(hist, hc, CREASE, W, lo, L, slot, first);
            first = false;
            since = 0;
            __syncthreads();
        }
    }
    drain_3d(hist, hc, CREASE, W, lo, L, slot, first);
}

// ---------------------------------------------------------------------------
// merge of per-workgroup partials and prefix scan over levels
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
    ecc_reduce(const int32_t *__restrict__ partial, int G, int nch, int L, unsigned ch_mask,
               int64_t *__restrict__ sums) {
    const int ch = blockIdx.y;
    if (!(ch_mask >> ch & 1)) return;
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= L) return;
    const int groups = gridDim.z, z = blockIdx.z;
    const int g0 = (int)((int64_t)G * z / groups), g1 = (int)((int64_t)G * (z + 1) / groups);
    int64_t s = 0;
    const int64_t stride = (int64_t)nch * L;
    const int32_t *p = partial + (int64_t)ch * L + b;
#pragma unroll 4
    for (int g = g0; g < g1; ++g) s += p[g * stride];
    sums[((int64_t)z * nch + ch) * L + b] = s;
}

struct OutPtrs {
    int64_t *p[4];
};

__global__ void __launch_bounds__(1024)
    ecc_scan(const int64_t *__restrict__ sums, int groups, int nch, int L, OutPtrs out) {
    __shared__ int64_t part[1024];
    const int ch = blockIdx.x;
    int64_t *dst = out.p[ch];
    if (!dst) return;
    const int t = threadIdx.x;
    const int per = (L + 1023) / 1024;
    const int beg = t * per, end = beg + per < L ? beg + per : L;
    const int64_t gstride = (int64_t)nch * L;
    const int64_t *src = sums + (int64_t)ch * L;
    int64_t s = 0;
    for (int i = beg; i < end; ++i)
        for (int z = 0; z < groups; ++z) s += src[z * gstride + i];
    part[t] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the 1024 chunk sums
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - s;
    for (int i = beg; i < end; ++i) {
        for (int z = 0; z < groups; ++z) run += src[z * gstride + i];
        dst[i] = run;
    }
}

// level index of every integer value from the thresholds (integer fields with
// a threshold array)
__global__ void ecc_level_lut(const float *__restrict__ thr, int L, int n_values,
                              uint16_t *__restrict__ lut) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_values) return;
    const float x = (float)v;
    int lo = 0, hi = L;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (x <= thr[mid])
            hi = mid;
        else
            lo = mid + 1;
    }
    lut[v] = (uint16_t)lo;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
size_t lds_bytes_2d(int window, int L) {
    return (size_t)window * 8 + (L <= kThrLds ? (size_t)L * 4 : 0);
}
size_t lds_bytes_3d(int window, bool want_crease) { return (size_t)window * (want_crease ? 12 : 8); }

template <typename T, int LM, bool AL>
static int launch_2d_t(const Launch2D &a, hipStream_t s) {
    constexpr int VEC = Elem<T>::VEC, PF = 4;
    const int64_t n_strips = (a.w + 64 * VEC - 1) / (64 * VEC);
    const int64_t rows = a.row_hi - a.row_lo;
    const int64_t NW = (int64_t)a.grid * kWavesPerWG;
    // rows per item: about one item per wave, at least 8 rows
    int64_t seg = (rows * n_strips + NW - 1) / NW;
    if (seg < 8) seg = 8;
    if (seg > rows) seg = rows;
    const int64_t n_segs = (rows + seg - 1) / seg;
    const int64_t n_items = n_strips * n_segs;
    // the packed LDS bins of one workgroup must not see more than kFlush2D cells
    const int64_t items_per_wave = (n_items + NW - 1) / NW;
    if (kWavesPerWG * items_per_wave * seg * 64 * VEC > kFlush2D) return (int)hipErrorInvalidValue;
    const int W = a.hi - a.lo;
    hipLaunchKernelGGL((ecc2d_stream<T, LM, AL, PF>), dim3(a.grid), dim3(256),
                       lds_bytes_2d(W, a.lv.L), s, (const T *)a.data, a.h, a.w, a.lv, a.lo, a.hi,
                       a.delta_lut, a.partial, a.row_lo, a.row_hi, n_segs, seg, n_items,
                       a.accumulate ? 1 : 0);
    return (int)hipGetLastError();
}

template <typename T, int LM>
static int launch_2d_al(const Launch2D &a, hipStream_t s) {
    const bool al = ((uintptr_t)a.data % 16 == 0) && (a.w * (int64_t)sizeof(T)) % 16 == 0;
    return al ? launch_2d_t<T, LM, true>(a, s) : launch_2d_t<T, LM, false>(a, s);
}

template <typename T>
static int launch_2d_dt(const Launch2D &a, hipStream_t s) {
    switch (a.lv.mode) {
    case LM_IDENTITY: return launch_2d_al<T, LM_IDENTITY>(a, s);
    case LM_LUT: return launch_2d_al<T, LM_LUT>(a, s);
    case LM_AFFINE: return launch_2d_al<T, LM_AFFINE>(a, s);
    default: return launch_2d_al<T, LM_SEARCH>(a, s);
    }
}

int launch_2d(const Launch2D &a, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    switch (a.dtype) {
    case ECC_U8: return launch_2d_dt<uint8_t>(a, s);
    case ECC_U16: return launch_2d_dt<uint16_t>(a, s);
    default: return launch_2d_dt<float>(a, s);
    }
}

template <typename T, int LM, bool CR>
static int launch_3d_t(const Launch3D &a, hipStream_t s) {
    const int64_t tiles_x = (a.w + kTile3DX - 1) / kTile3DX;
    const int64_t tiles_y = (a.h + kTile3DY - 1) / kTile3DY;
    const int64_t tiles_z = (a.d + kTile3DZ - 1) / kTile3DZ;
    const int64_t n_tiles = tiles_x * tiles_y * tiles_z;
    const int flush = (int)(kFlush3D / (kTile3DX * kTile3DY * kTile3DZ));
    const int W = a.hi - a.lo;
    hipLaunchKernelGGL((ecc3d_tile<T, LM, CR>), dim3(a.grid), dim3(256), lds_bytes_3d(W, CR), s,
                       (const T *)a.data, a.d, a.h, a.w, a.lv, a.lo, a.hi, a.vtab, a.partial,
                       tiles_x, tiles_y, n_tiles, flush);
    return (int)hipGetLastError();
}

template <typename T, int LM>
static int launch_3d_cr(const Launch3D &a, hipStream_t s) {
    return a.want_crease ? launch_3d_t<T, LM, true>(a, s) : launch_3d_t<T, LM, false>(a, s);
}

template <typename T>
static int launch_3d_dt(const Launch3D &a, hipStream_t s) {
    switch (a.lv.mode) {
    case LM_IDENTITY: return launch_3d_cr<T, LM_IDENTITY>(a, s);
    case LM_LUT: return launch_3d_cr<T, LM_LUT>(a, s);
    case LM_AFFINE: return launch_3d_cr<T, LM_AFFINE>(a, s);
    default: return launch_3d_cr<T, LM_SEARCH>(a, s);
    }
}

int launch_3d(const Launch3D &a, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    switch (a.dtype) {
    case ECC_U8: return launch_3d_dt<uint8_t>(a, s);
    case ECC_U16: return launch_3d_dt<uint16_t>(a, s);
    default: return launch_3d_dt<float>(a, s);
    }
}

int launch_reduce(const int32_t *partial, int grid, int nch, int L, unsigned ch_mask, int groups,
                  int64_t *sums, void *stream) {
    hipLaunchKernelGGL(ecc_reduce, dim3((L + 255) / 256, nch, groups), dim3(256), 0,
                       (hipStream_t)stream, partial, grid, nch, L, ch_mask, sums);
    return (int)hipGetLastError();
}

int launch_scan(const int64_t *sums, int groups, int nch, int L, int64_t *const out[4], void *stream) {
    OutPtrs o;
    for (int c = 0; c < 4; ++c) o.p[c] = c < nch ? out[c] : nullptr;
    hipLaunchKernelGGL(ecc_scan, dim3(nch), dim3(1024), 0, (hipStream_t)stream, sums, groups, nch, L, o);
    return (int)hipGetLastError();
}

int launch_level_lut(const float *thr, int L, int n_values, uint16_t *lut, void *stream) {
    hipLaunchKernelGGL(ecc_level_lut, dim3((n_values + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, thr, L, n_values, lut);
    return (int)hipGetLastError();
}

}  // namespace ecc
