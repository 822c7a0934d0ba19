// 3D vertex class counts (the contribution map of Table 2): per level, the
// number of lattice vertices whose 2x2x2 block of active voxels is of each of
// the 21 octant classes.
//
// When voxel p enters (voxels ordered by level, ties by position), each of the
// 8 lattice vertices at its corners moves from the class of its block without
// p to the class of its block with p: +1 to the new class, -1 to the old one
// (none when the block was empty), in p's level bin.  So a voxel's events
// depend on which of its 26 neighbours entered before it.
//
// The class bins of every level do not fit in LDS (21 int32 per level), so the
// levels are split into windows of W levels, one pass per window.  A pass
// stages a tile's levels (plus a one-voxel halo) into LDS; each wave then
// collects the voxels of its share of the tile whose level lies in the window
// into a queue and processes them 64 at a time, one voxel per lane, so that the
// per-voxel work (27 neighbour reads, 8 corner transitions, 16 LDS atomics) is
// done once per voxel over all passes, not once per pass.  At the end of a
// pass the workgroup adds its bins into per-XCD int64 accumulators.
#include "ecc_device.h"

namespace ecc {

constexpr int kCls3TX = 64, kCls3TY = 8, kCls3TZ = 16;           // tile of 8192 voxels
constexpr int kCls3SX = kCls3TX + 2, kCls3SY = kCls3TY + 2, kCls3SZ = kCls3TZ + 2;  // with halo
constexpr int kCls3Threads = 1024;
constexpr int kCls3Waves = kCls3Threads / 64;
constexpr int kCls3Queue = 128;  // per wave: at most 63 waiting plus 64 appended

// LDS of the class-count kernel besides its bins
size_t lds_fixed_classes_3d() {
    return sizeof(uint16_t) * (kCls3SZ * kCls3SY * kCls3SX + kCls3Waves * kCls3Queue + 8 * 256) + 1024;
}

template <typename T, int LM>
__global__ void __launch_bounds__(kCls3Threads)
    ecc3d_classes(const T *__restrict__ data, int64_t d, int64_t h, int64_t w, LevelArgs lv, int32_t lo,
                  int32_t hi, const uint16_t *__restrict__ trans, int64_t *__restrict__ acc, int64_t tiles_x,
                  int64_t tiles_y, int64_t n_tiles) {
    extern __shared__ int32_t bins[];  // [W][kNumClasses3D], then one spare bin per lane
    __shared__ uint16_t lam[kCls3SZ][kCls3SY][kCls3SX];
    __shared__ uint16_t queue[kCls3Waves][kCls3Queue];
    __shared__ uint16_t tr[8][256];  // corner c, block mask -> new class | old class << 8 (0xFF: empty)

    const int t = threadIdx.x, lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int W = hi - lo, L = lv.L;
    const int nb = W * kNumClasses3D;
    for (int i = t; i < nb + 64; i += kCls3Threads) bins[i] = 0;
    for (int i = t; i < 8 * 256; i += kCls3Threads) (&tr[0][0])[i] = trans[i];
    const int G = gridDim.x;
    const int wg = xcd_order(blockIdx.x, G);
    const int64_t t_beg = n_tiles * wg / G, t_end = n_tiles * (wg + 1) / G;
    const uint32_t spare = (uint32_t)(nb + lane);  // a lane's bin for the events of an empty old block
    uint16_t *q = queue[wave];
    __syncthreads();

    // Staging: the staged tile is kCls3SZ x kCls3SY rows of kCls3SX levels;
    // wave w loads the 64 interior columns of rows w, w + 16, ... (one element
    // per lane, coalesced) and threads 0..359 the two halo columns.  Every load
    // is unconditional, at coordinates clamped into the field (cells outside
    // it are set to "never" when stored), and a tile's loads are issued while
    // the previous tile is processed.
    // Tile coordinates step through the workgroup's range (x fastest) without
    // divisions; rows of the staged tile are addressed by (z h + y) w from
    // clamped coordinates.
    constexpr int kRows = kCls3SZ * kCls3SY, kRowIt = (kRows + kCls3Waves - 1) / kCls3Waves;
    struct TileXYZ {
        int64_t x0, y0, z0;
    };
    auto step = [&](TileXYZ c) {
        c.x0 += kCls3TX;
        if (c.x0 >= tiles_x * kCls3TX) {
            c.x0 = 0;
            c.y0 += kCls3TY;
            if (c.y0 >= tiles_y * kCls3TY) {
                c.y0 = 0;
                c.z0 += kCls3TZ;
            }
        }
        return c;
    };
    uint32_t raw[kRowIt + 1];
    auto clampi = [](int64_t v, int64_t n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); };
    // offsets of this wave's staged rows from the staged corner (tiles away
    // from the y and z faces of the field need no clamping)
    int64_t roff[kRowIt];
#pragma unroll
    for (int i = 0; i < kRowIt; ++i) {
        const int r = min(wave + kCls3Waves * i, kRows - 1);
        roff[i] = ((int64_t)(r / kCls3SY) * h + r % kCls3SY) * w;
    }
    auto load_tile = [&](const TileXYZ &c) {
        const int64_t x = clampi(c.x0 + lane, w);
        if (c.y0 >= 1 && c.y0 - 1 + kCls3SY <= h && c.z0 >= 1 && c.z0 - 1 + kCls3SZ <= d) {  // uniform
            const T *base = data + ((c.z0 - 1) * h + (c.y0 - 1)) * w + x;
#pragma unroll
            for (int i = 0; i < kRowIt; ++i) raw[i] = elem_bits(base + roff[i]);
        } else {
#pragma unroll
            for (int i = 0; i < kRowIt; ++i) {
                const int r = min(wave + kCls3Waves * i, kRows - 1);  // uniform
                const int64_t y = clampi(c.y0 - 1 + r % kCls3SY, h), z = clampi(c.z0 - 1 + r / kCls3SY, d);
                raw[i] = elem_bits(data + (z * h + y) * w + x);
            }
        }
        const int r = min(t >> 1, kRows - 1);
        const int64_t y = clampi(c.y0 - 1 + r % kCls3SY, h), z = clampi(c.z0 - 1 + r / kCls3SY, d);
        raw[kRowIt] = elem_bits(data + (z * h + y) * w + clampi((t & 1) ? c.x0 + kCls3TX : c.x0 - 1, w));
    };
    auto store_tile = [&](const TileXYZ &c) {
        auto level = [&](uint32_t bits, bool in) {
            return in ? (uint32_t)level_of<T, LM>(as_value<T>(bits), lv, ThrGlobal{lv.thr}) : (uint32_t)L;
        };
        const bool x_in = c.x0 + lane < w;
#pragma unroll
        for (int i = 0; i < kRowIt; ++i) {
            const int r = wave + kCls3Waves * i;
            if (r < kRows) {  // uniform
                const int yy = r % kCls3SY, zz = r / kCls3SY;
                const int64_t y = c.y0 - 1 + yy, z = c.z0 - 1 + zz;
                const bool yz_in = y >= 0 && y < h && z >= 0 && z < d;  // uniform
                lam[zz][yy][lane + 1] = (uint16_t)level(raw[i], x_in && yz_in);
            }
        }
        if (t < 2 * kRows) {
            const int r = t >> 1, yy = r % kCls3SY, zz = r / kCls3SY;
            const int xx = (t & 1) ? kCls3SX - 1 : 0;
            const int64_t x = c.x0 - 1 + xx, y = c.y0 - 1 + yy, z = c.z0 - 1 + zz;
            lam[zz][yy][xx] = (uint16_t)level(raw[kRowIt], x >= 0 && x < w && y >= 0 && y < h && z >= 0 && z < d);
        }
    };
    TileXYZ cur{(t_beg % tiles_x) * kCls3TX, ((t_beg / tiles_x) % tiles_y) * kCls3TY,
                (t_beg / (tiles_x * tiles_y)) * kCls3TZ};
    if (t_beg < t_end) load_tile(cur);

    for (int64_t tile = t_beg; tile < t_end; ++tile) {
        const int64_t x0 = cur.x0, y0 = cur.y0, z0 = cur.z0;
        store_tile(cur);
        cur = step(cur);
        if (tile + 1 < t_end) load_tile(cur);  // in flight while this tile is processed
        __syncthreads();
        int qn = 0;  // voxels waiting in this wave's queue (wave-uniform)
        // voxel v of the tile: x = v % 64 (the lane), y = v / 64 % 8, z = v / 512
        for (int k = 0; k < kCls3TX * kCls3TY * kCls3TZ / kCls3Threads + 1; ++k) {
            const bool tail = k == kCls3TX * kCls3TY * kCls3TZ / kCls3Threads;  // uniform: drain the queue
            if (!tail) {
                const int v = k * kCls3Threads + t;
                const int x = v & 63, y = (v >> 6) & 7, z = v >> 9;
                const uint32_t l = lam[z + 1][y + 1][x + 1];
                const bool in = l - (uint32_t)lo < (uint32_t)W && x0 + x < w && y0 + y < h && z0 + z < d;
                const uint64_t m = __ballot(in);
                if (in) q[qn + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0))] =
                    (uint16_t)v;
                qn += __popcll(m);
            }
            while (qn >= 64 || (tail && qn > 0)) {  // uniform
                const bool act = lane < qn;
                if (act) {
                    const int v = q[lane];
                    const int x = v & 63, y = (v >> 6) & 7, z = v >> 9;
                    // the 3x3x3 window, one pair of dwords per row of three
                    // (rows are an even number of levels apart, so the first
                    // level of every row has the parity of the corner's)
                    static_assert(kCls3SX % 2 == 0, "rows must start on whole dwords");
                    const int e = (z * kCls3SY + y) * kCls3SX + x;  // corner (-1, -1, -1) of the window
                    const uint32_t *lw = reinterpret_cast<const uint32_t *>(&lam[0][0][0]) + (e >> 1);
                    const uint32_t sh = (uint32_t)(e & 1) * 16u;
                    uint32_t win[27];
#pragma unroll
                    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
                        for (int dy = 0; dy < 3; ++dy) {
                            const int o = (dz * kCls3SY * kCls3SX + dy * kCls3SX) / 2;
                            const uint32_t a = lw[o], c = lw[o + 1];
                            const uint32_t ab = __builtin_amdgcn_alignbit(c, a, sh);  // levels x-1 and x
                            win[dz * 9 + dy * 3 + 0] = ab & 0xFFFFu;
                            win[dz * 9 + dy * 3 + 1] = ab >> 16;
                            win[dz * 9 + dy * 3 + 2] = (c >> sh) & 0xFFFFu;
                        }
                    const uint32_t p = win[13];
                    // bit k: neighbour k entered before p (earlier in memory
                    // order wins ties); bit 13 is p itself
                    uint32_t P = 1u << 13;
#pragma unroll
                    for (int k2 = 0; k2 < 27; ++k2) {
                        if (k2 == 13) continue;
                        const bool pr = k2 < 13 ? (win[k2] <= p) : (win[k2] < p);
                        P |= (uint32_t)pr << k2;
                    }
                    const uint32_t row = (p - (uint32_t)lo) * kNumClasses3D;
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        // corner (cx, cy, cz): the block of neighbours with
                        // offsets in {c - 1, c} per axis, as an octant mask
                        // (bit bx + 2 by + 4 bz)
                        const int cx = c & 1, cy = c >> 1 & 1, cz = c >> 2;
                        const uint32_t yb = P >> (cz * 9 + cy * 3 + cx);
                        const uint32_t m1 =
                            (yb & 3u) | ((yb >> 1) & 0xCu) | ((yb >> 5) & 0x30u) | ((yb >> 6) & 0xC0u);
                        const uint32_t e = tr[c][m1];
                        const uint32_t oc = e >> 8;
                        lds_add32(lds_addr(bins) + 4u * (row + (e & 0xFFu)), 1u);
                        lds_add32(lds_addr(bins) + 4u * (oc == 0xFFu ? spare : row + oc), 0xFFFFFFFFu);
                    }
                }
                // the entries beyond the 64 processed move to the front
                if (qn > 64 && lane < qn - 64) {
                    const uint16_t mv = q[64 + lane];
                    q[lane] = mv;
                }
                qn = qn > 64 ? qn - 64 : 0;
            }
        }
        __syncthreads();  // lam is restaged by the next tile
    }
    __syncthreads();
    // bins -> this XCD's accumulator copy [kNumClasses3D][L]
    int64_t *a = acc + (int64_t)xcc_copy() * kNumClasses3D * L;
    for (int i = t; i < nb; i += kCls3Threads) {
        const int32_t v = bins[i];
        if (v == 0) continue;
        const int b = i / kNumClasses3D, c = i - b * kNumClasses3D;
        acc_add(a + (int64_t)c * L + lo + b, (int64_t)v);
    }
}

template <typename T, int LM>
static int launch_cls_t(const Launch3DClasses &a, hipStream_t s) {
    const int64_t tiles_x = (a.w + kCls3TX - 1) / kCls3TX;
    const int64_t tiles_y = (a.h + kCls3TY - 1) / kCls3TY;
    const int64_t tiles_z = (a.d + kCls3TZ - 1) / kCls3TZ;
    const size_t lds = (size_t)((a.hi - a.lo) * kNumClasses3D + 64) * sizeof(int32_t);
    hipExtLaunchKernelGGL((ecc3d_classes<T, LM>), dim3(a.grid), dim3(kCls3Threads), lds, s,
                          (hipEvent_t)a.ev_start, (hipEvent_t)a.ev_stop, 0, (const T *)a.data, a.d, a.h, a.w,
                          a.lv, a.lo, a.hi, a.trans, a.acc, tiles_x, tiles_y, tiles_x * tiles_y * tiles_z);
    return (int)hipGetLastError();
}

int launch_classes_3d(const Launch3DClasses &a, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    switch (a.dtype) {
    case ECC_U8:
        return a.lv.mode == LM_LUT ? launch_cls_t<uint8_t, LM_LUT>(a, s) : launch_cls_t<uint8_t, LM_IDENTITY>(a, s);
    case ECC_U16:
        return a.lv.mode == LM_LUT ? launch_cls_t<uint16_t, LM_LUT>(a, s)
                                   : launch_cls_t<uint16_t, LM_IDENTITY>(a, s);
    default:
        return a.lv.mode == LM_AFFINE ? launch_cls_t<float, LM_AFFINE>(a, s) : launch_cls_t<float, LM_SEARCH>(a, s);
    }
}

}  // namespace ecc
