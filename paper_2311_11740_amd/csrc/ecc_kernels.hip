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
template <typename T, int LM>
__device__ __forceinline__ uint32_t level_of(T v, const LevelArgs &a) {
    if constexpr (LM == LM_IDENTITY) {
        const uint32_t u = (uint32_t)v;
        return u < (uint32_t)a.L ? u : (uint32_t)a.L;
    } else if constexpr (LM == LM_LUT) {
        return a.lut[(uint32_t)v];
    } else {
        const float x = (float)v;
        const int L = a.L;
        if (!(x == x)) return (uint32_t)L;  // NaN never enters
        int g;
        if constexpr (LM == LM_AFFINE) {
            float gf = floorf((x - a.t0) * a.inv_step) + 1.0f;
            gf = fminf(fmaxf(gf, 0.0f), (float)L);
            g = (int)gf;
            // exact correction against the caller's thresholds: afterwards
            // t[g-1] < x <= t[g] (with t[-1] = -inf, t[L] = +inf)
            while (g > 0 && x <= a.thr[g - 1]) --g;
            while (g < L && !(x <= a.thr[g])) ++g;
        } else {
            int lo = 0, hi = L;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (x <= a.thr[mid])
                    hi = mid;
                else
                    lo = mid + 1;
            }
            g = lo;
        }
        return (uint32_t)g;
    }
}

__device__ __forceinline__ int xcd_order(int bid, int G) {
    // workgroups are dispatched round-robin over the 8 XCDs; renumber them so
    // that each XCD holds a contiguous block of workgroup ids
    return (G & 7) == 0 ? (bid & 7) * (G >> 3) + (bid >> 3) : bid;
}

// ---------------------------------------------------------------------------
// 2D
// ---------------------------------------------------------------------------
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

template <typename T, int LM, int TH>
__global__ void __launch_bounds__(256)
    ecc2d_tile(const T *__restrict__ data, int64_t h, int64_t w, LevelArgs lv, int32_t lo,
               int32_t hi, const uint64_t *__restrict__ delta_lut, int32_t *__restrict__ partial,
               int64_t tiles_x, int64_t n_tiles, int flush_tiles) {
    constexpr int TW = kTile2DCols;
    extern __shared__ uint64_t hist[];
    __shared__ uint64_t dl[256];
    __shared__ uint16_t lam[TH + 2][TW + 2];

    const int t = threadIdx.x;
    const int W = hi - lo;
    const int L = lv.L;
    const int G = gridDim.x;
    const int wg = xcd_order(blockIdx.x, G);
    const int64_t t_beg = n_tiles * wg / G, t_end = n_tiles * (wg + 1) / G;

    dl[t] = delta_lut[t];
    for (int b = t; b < W; b += 256) hist[b] = 0;
    int32_t *slot = partial + (int64_t)wg * 3 * L;
    bool first = true;
    int since = 0;
    __syncthreads();

    for (int64_t tile = t_beg; tile < t_end; ++tile) {
        const int64_t r0 = (tile / tiles_x) * TH, c0 = (tile % tiles_x) * TW;
        // stage the levels of rows r0-1 .. r0+TH and columns c0-1 .. c0+TW
        for (int rr = 0; rr < TH + 2; ++rr) {
            const int64_t r = r0 - 1 + rr;
            const bool row_in = r >= 0 && r < h;
            for (int cc = t; cc < TW + 2; cc += 256) {
                const int64_t c = c0 - 1 + cc;
                uint32_t l = (uint32_t)L;
                if (row_in && c >= 0 && c < w) l = level_of<T, LM>(data[r * w + c], lv);
                lam[rr][cc] = (uint16_t)l;
            }
        }
        __syncthreads();
        if (c0 + t < w) {
            uint32_t a0 = lam[0][t], a1 = lam[0][t + 1], a2 = lam[0][t + 2];
            uint32_t b0 = lam[1][t], b1 = lam[1][t + 1], b2 = lam[1][t + 2];
            const int rows = (int)(h - r0 < TH ? h - r0 : TH);
            for (int r = 0; r < rows; ++r) {
                const uint32_t e0 = lam[r + 2][t], e1 = lam[r + 2][t + 1], e2 = lam[r + 2][t + 2];
                const uint32_t p = b1;
                if (p - (uint32_t)lo < (uint32_t)W) {
                    // neighbours that come earlier in memory order precede p on a
                    // tie, later ones do not
                    const uint32_t pat = (uint32_t)(a0 <= p) | (uint32_t)(a1 <= p) << 1 |
                                         (uint32_t)(a2 <= p) << 2 | (uint32_t)(b0 <= p) << 3 |
                                         (uint32_t)(b2 < p) << 4 | (uint32_t)(e0 < p) << 5 |
                                         (uint32_t)(e1 < p) << 6 | (uint32_t)(e2 < p) << 7;
                    atomicAdd((unsigned long long *)&hist[p - lo], (unsigned long long)dl[pat]);
                }
                a0 = b0; a1 = b1; a2 = b2;
                b0 = e0; b1 = e1; b2 = e2;
            }
        }
        __syncthreads();
        if (++since >= flush_tiles) {
            drain_2d(hist, W, lo, L, slot, first);
            first = false;
            since = 0;
            __syncthreads();
        }
    }
    drain_2d(hist, W, lo, L, slot, first);
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
                l = level_of<T, LM>(data[(z * h + y) * w + x], lv);
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
               int64_t *__restrict__ totals) {
    const int ch = blockIdx.y;
    if (!(ch_mask >> ch & 1)) return;
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= L) return;
    int64_t s = 0;
    const int32_t *p = partial + (int64_t)ch * L + b;
    const int64_t stride = (int64_t)nch * L;
#pragma unroll 8
    for (int g = 0; g < G; ++g) s += p[g * stride];
    totals[(int64_t)ch * L + b] = s;
}

struct OutPtrs {
    int64_t *p[4];
};

__global__ void __launch_bounds__(1024)
    ecc_scan(const int64_t *__restrict__ totals, int L, OutPtrs out) {
    __shared__ int64_t part[1024];
    const int ch = blockIdx.x;
    int64_t *dst = out.p[ch];
    if (!dst) return;
    const int t = threadIdx.x;
    const int per = (L + 1023) / 1024;
    const int beg = t * per, end = beg + per < L ? beg + per : L;
    const int64_t *src = totals + (int64_t)ch * L;
    int64_t s = 0;
    for (int i = beg; i < end; ++i) s += src[i];
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
        run += src[i];
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
size_t lds_bytes_2d(int window, int tile_rows) {
    (void)tile_rows;
    return (size_t)window * 8;
}
size_t lds_bytes_3d(int window, bool want_crease) { return (size_t)window * (want_crease ? 12 : 8); }

template <typename T, int LM>
static int launch_2d_t(const Launch2D &a, hipStream_t s) {
    constexpr int TH = 32;
    const int64_t tiles_x = (a.w + kTile2DCols - 1) / kTile2DCols;
    const int64_t tiles_y = (a.h + TH - 1) / TH;
    const int64_t n_tiles = tiles_x * tiles_y;
    const int flush = (int)(kFlush2D / (TH * kTile2DCols));
    const int W = a.hi - a.lo;
    hipLaunchKernelGGL((ecc2d_tile<T, LM, TH>), dim3(a.grid), dim3(256), lds_bytes_2d(W, TH), s,
                       (const T *)a.data, a.h, a.w, a.lv, a.lo, a.hi, a.delta_lut, a.partial,
                       tiles_x, n_tiles, flush);
    return (int)hipGetLastError();
}

template <typename T>
static int launch_2d_dt(const Launch2D &a, hipStream_t s) {
    switch (a.lv.mode) {
    case LM_IDENTITY: return launch_2d_t<T, LM_IDENTITY>(a, s);
    case LM_LUT: return launch_2d_t<T, LM_LUT>(a, s);
    case LM_AFFINE: return launch_2d_t<T, LM_AFFINE>(a, s);
    default: return launch_2d_t<T, LM_SEARCH>(a, s);
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

int launch_reduce(const int32_t *partial, int grid, int nch, int L, unsigned ch_mask,
                  int64_t *totals, void *stream) {
    hipLaunchKernelGGL(ecc_reduce, dim3((L + 255) / 256, nch), dim3(256), 0, (hipStream_t)stream,
                       partial, grid, nch, L, ch_mask, totals);
    return (int)hipGetLastError();
}

int launch_scan(const int64_t *totals, int nch, int L, int64_t *const out[4], void *stream) {
    OutPtrs o;
    for (int c = 0; c < 4; ++c) o.p[c] = c < nch ? out[c] : nullptr;
    hipLaunchKernelGGL(ecc_scan, dim3(nch), dim3(1024), 0, (hipStream_t)stream, totals, L, o);
    return (int)hipGetLastError();
}

int launch_level_lut(const float *thr, int L, int n_values, uint16_t *lut, void *stream) {
    hipLaunchKernelGGL(ecc_level_lut, dim3((n_values + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, thr, L, n_values, lut);
    return (int)hipGetLastError();
}

}  // namespace ecc
