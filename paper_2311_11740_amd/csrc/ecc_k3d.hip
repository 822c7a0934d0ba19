// 3D kernels: the z-marching kernel (slab decomposition) and the generic tile
// kernel (curves with the crease measure, vertex class counts), with their
// launchers.
#include "ecc_device.h"
#include "ecc_levels.h"
#include "ecc_schedule.h"

namespace ecc {

// ---------------------------------------------------------------------------
// 3D bins -> partials
// ---------------------------------------------------------------------------
__device__ __forceinline__ void drain_3d(uint64_t *hist, uint32_t *hc, bool crease, int W, int lo,
                                         int L, int G, int wg, int32_t *__restrict__ partial, bool first) {
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
        const int64_t i0 = ((int64_t)(lo + b)) * G + wg, cs = (int64_t)L * G;
        // (the crease slot is left alone when the crease is not computed: the
        // merge skips that channel)
        if (first) {
            partial[i0] = (int32_t)ec;
            if (crease) partial[i0 + cs] = (int32_t)cr;
            partial[i0 + 2 * cs] = (int32_t)surf;
            partial[i0 + 3 * cs] = (int32_t)n;
        } else {
            partial[i0] += (int32_t)ec;
            if (crease) partial[i0 + cs] += (int32_t)cr;
            partial[i0 + 2 * cs] += (int32_t)surf;
            partial[i0 + 3 * cs] += (int32_t)n;
        }
    }
}

// the same bins added into the XCD's accumulator copy [4][L] (atomic drain)
__device__ __forceinline__ void drain_3d_acc(const uint64_t *hist, const uint32_t *hc, bool crease, int W, int lo,
                                             int L, int64_t *__restrict__ acc, bool pack) {
    int64_t *a = acc + (int64_t)xcc_copy() * 4 * L;
    for (int b = threadIdx.x; b < W; b += blockDim.x) {
        const uint64_t v = hist[b];
        const int64_t n = (int64_t)(v >> kShiftCnt3);
        if (n == 0) continue;
        const int64_t surf = (int64_t)((v >> kShiftSurf3) & ((1ull << (kShiftCnt3 - kShiftSurf3)) - 1)) -
                             kSurfBias3 * n;
        const int64_t ec = (int64_t)(v & ((1ull << kShiftSurf3) - 1)) - kEcBias3 * n;
        acc_add(a + lo + b, ec);
        if (crease) acc_add(a + L + lo + b, (int64_t)hc[b] - kCreaseBias3 * n);
        if (pack) {  // uniform
            acc_add(a + 2 * L + lo + b, surf + kPackBias * n + (n << kPackShift));
        } else {
            acc_add(a + 2 * L + lo + b, surf);
            acc_add(a + 3 * L + lo + b, n);
        }
    }
}

// ---------------------------------------------------------------------------
// 3D: slab decomposition, z-marching waves
// ---------------------------------------------------------------------------
// The closure of the active voxels splits into lattice cells that lie in a
// z-plane Z (vertices, x/y edges, xy faces) and cells that span a voxel layer
// z (z edges, xz/yz faces, voxels).  A cell in plane Z is present exactly when
// the 2D cell under it is present in the image min(lam[Z-1], lam[Z]) (the
// "min image"); a cell spanning layer z when its 2D counterpart is present in
// layer z, with dimension one higher.  Hence for the 26-connected EC
//   chi26 = sum_Z chi8(min image Z) - sum_z chi8(layer z),
// and dually, for the 6-connected complex (cells = voxels),
//   chi6 = sum_z chi4(layer z) - sum_Z chi4(max(lam[Z-1], lam[Z])).
// So every voxel needs two 2D 8-neighbour patterns: its own layer's, and the
// one of the min (max) image between its layer and the next.  The 2D event of
// a min-image pixel happens at the level of the voxel that enters first of
// the two (last, for the max image), so it is added to that voxel's event:
// one LDS atomic per voxel.  The surface adds the two vertical faces, the
// volume is the count.  The crease measure, when wanted, comes from the same
// planes (see March3D).
//
// A wave owns TY rows of a strip of 64*VEC columns and marches z, holding the
// level indices of planes z-1, z, z+1 (TY+2 rows each, packed as in 2D) in
// three buffers that rotate with z.  The cells left and right of the strip
// come from one extra unconditional element load per lane and row.
template <typename T>
struct Elem3 {
    static constexpr int VEC = 4;                    // cells per lane
    static constexpr int WORDS = 4 * sizeof(T) / 4;  // raw dwords per lane and row
};

struct RawRow3 {
    uint32_t w[4];
    uint32_t halo;   // lane 0: element left of the strip; lane 63: right of it
    uint32_t shift;  // elements the block must move down (kLoadVector at the buffer end)
};

template <typename T>
__device__ __forceinline__ uint32_t elem3(const RawRow3 &r, int i) {
    if constexpr (sizeof(T) == 1) return (r.w[0] >> (8 * i)) & 0xFFu;
    else if constexpr (sizeof(T) == 2) return (r.w[i >> 1] >> (16 * (i & 1))) & 0xFFFFu;
    else return r.w[i];
}

// one block of VEC elements (4 * sizeof(T) bytes) at element index e
template <typename T, bool UNALIGNED>
__device__ __forceinline__ void load_block3(const T *p, RawRow3 &raw) {
    if constexpr (sizeof(T) == 1) {
        typedef uint32_t u32_u __attribute__((aligned(1)));
        typedef uint32_t u32_a __attribute__((aligned(4)));
        if constexpr (UNALIGNED)
            raw.w[0] = __builtin_nontemporal_load(reinterpret_cast<const u32_u *>(p));
        else
            raw.w[0] = __builtin_nontemporal_load(reinterpret_cast<const u32_a *>(p));
    } else if constexpr (sizeof(T) == 2) {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        typedef u32x2 u32x2_u __attribute__((aligned(1)));
        u32x2 q;
        if constexpr (UNALIGNED)
            q = __builtin_nontemporal_load(reinterpret_cast<const u32x2_u *>(p));
        else
            q = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(p));
        raw.w[0] = q.x; raw.w[1] = q.y;
    } else {
        u32x4 q;
        if constexpr (UNALIGNED)
            q = __builtin_nontemporal_load(reinterpret_cast<const u32x4_u *>(p));
        else
            q = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
        raw.w[0] = q.x; raw.w[1] = q.y; raw.w[2] = q.z; raw.w[3] = q.w;
    }
}

// row y of plane z (both clamped into the field by the caller); unconditional
// loads, in the two modes of the 2D kernels (a block is 4 elements here)
template <typename T, int AL>
__device__ __forceinline__ void fetch_row3(const T *__restrict__ data, int64_t h, int64_t w, int z, int y,
                                           int64_t xs, int64_t x0, int lane, int64_t last_block, RawRow3 &raw) {
    constexpr int VEC = Elem3<T>::VEC;
    const int64_t rbase = ((int64_t)z * h + y) * w;
    const T *row = data + rbase;
    raw.w[0] = raw.w[1] = raw.w[2] = raw.w[3] = 0;
    raw.shift = 0;
    if constexpr (AL == kLoadAligned) {  // whole blocks: inside or outside the row
        load_block3<T, false>(row + (x0 < w ? x0 : 0), raw);
    } else {
        const int64_t li = rbase + (x0 < w ? x0 : 0);
        const int64_t lc = li < last_block ? li : last_block;  // last_block = d * h * w - VEC
        load_block3<T, true>(data + lc, raw);
        raw.shift = (uint32_t)(li - lc);
    }
    int64_t hx = lane == 0 ? xs - 1 : (lane == 63 ? xs + 64 * VEC : x0);
    hx = hx < 0 ? 0 : (hx >= w ? w - 1 : hx);
    raw.halo = elem_bits(row + hx);
}

template <typename T>
__device__ __forceinline__ void unshift_row3(RawRow3 &raw) {
    const uint32_t sb = raw.shift * (uint32_t)sizeof(T);  // bytes, < 4 * sizeof(T)
    uint64_t lo = (uint64_t)raw.w[0] | (uint64_t)raw.w[1] << 32;
    uint64_t hi = (uint64_t)raw.w[2] | (uint64_t)raw.w[3] << 32;
    if (sb >= 8) {
        lo = hi >> (8 * (sb - 8));
        hi = 0;
    } else if (sb > 0) {
        lo = (lo >> (8 * sb)) | (hi << (64 - 8 * sb));
        hi >>= 8 * sb;
    }
    raw.w[0] = (uint32_t)lo; raw.w[1] = (uint32_t)(lo >> 32);
    raw.w[2] = (uint32_t)hi; raw.w[3] = (uint32_t)(hi >> 32);
}

// bin index (kBinOff convention) of one value
template <typename T, int LM, typename TH>
__device__ __forceinline__ uint32_t bin3(uint32_t bits, const LevelArgs &lv, const TH &thr, int lo, int W,
                                         float cpass, const LaneBins &lb) {
    if constexpr (LM == LM_AFFINE) {
        const float x = __uint_as_float(bits);
        const float y = __builtin_fmaf(x, lv.inv_step, cpass);
        const float m = y + kMagic;
        const float r = y - (m - kMagic);
        // clamped bin estimate (in the first pass at least the bin of level
        // 0: values at or below t0 have level 0)
        const float mlo = kMagic + (float)(lo == 0 ? (uint32_t)kBinOff : lb.below);
        uint32_t l = __float_as_uint(__builtin_amdgcn_fmed3f(m, mlo, kMagic + (float)lb.never)) - kMagicBits;
        if (!(__builtin_fabsf(r) <= 0.5f - lv.eps)) {  // near a threshold (or NaN / inf)
            const int k = (int)l;
            if (k >= kBinOff - 1 && k <= W + kBinOff) {
                const int g0 = k + lo - kBinOff < 0 ? 0 : k + lo - kBinOff;
                const int g = (int)level_settle(cmp_value(x, lv.neg), (uint32_t)g0, lv.L, thr);
                l = g < lo ? lb.below : (g >= lo + W ? lb.never : (uint32_t)(g - lo + kBinOff));
            }
        }
        return l;
    } else if constexpr (LM == LM_SEARCH) {
        return bin_search(__uint_as_float(bits ^ lv.neg), lo, lo + W, thr, lb);
    } else {
        const int l = (int)level_of<T, LM>(as_value<T>(bits), lv, thr);
        return (uint32_t)min(max(l - lo + kBinOff, (int)lb.below), (int)lb.never);
    }
}

// packed bin pairs of one row (P[i] = (bin[i-1], bin[i]) with the strip
// neighbours at both ends); rows outside the field never enter
template <typename T, int LM, typename TH>
__device__ __forceinline__ void convert_row3(const RawRow3 &raw_in, bool row_ok, int64_t w, int64_t xs, int64_t x0,
                                             int lane, const LevelArgs &lv, const TH &thr, int lo, int W,
                                             float cpass, const LaneBins &lb, uint32_t (&P)[Elem3<T>::VEC + 1]) {
    constexpr int VEC = Elem3<T>::VEC;
    const uint32_t never = lb.never;
    RawRow3 raw = raw_in;
    if (__any(raw.shift != 0)) unshift_row3<T>(raw);  // rare: blocks at the end of the buffer
    if constexpr (LM == LM_IDENTITY) {  // integer values, two per packed operation
        const uint32_t nv2 = never * 0x10001u;
        uint32_t Q[2];
        if (lo == 0) {  // uniform
            const u16x2 off = {(unsigned short)kBinOff, (unsigned short)kBinOff};
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                u16x2 v = __builtin_bit_cast(u16x2, raw_pair<T>(raw.w, 2 * k));
                v = __builtin_elementwise_min(__builtin_elementwise_add_sat(v, off), __builtin_bit_cast(u16x2, nv2));
                Q[k] = __builtin_bit_cast(uint32_t, v);
            }
        } else {
            const unsigned short sub = (unsigned short)(lo - kBinOff);
            const u16x2 off = {sub, sub};
            const uint32_t bl2 = lb.below * 0x10001u;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                u16x2 v = __builtin_bit_cast(u16x2, raw_pair<T>(raw.w, 2 * k));
                v = __builtin_elementwise_max(__builtin_elementwise_sub_sat(v, off), __builtin_bit_cast(u16x2, bl2));
                v = __builtin_elementwise_min(v, __builtin_bit_cast(u16x2, nv2));
                Q[k] = __builtin_bit_cast(uint32_t, v);
            }
        }
        if (!(xs + 64 * VEC <= w)) {  // uniform: cells outside the field never enter
            const uint32_t m0 = (x0 < w ? 0u : 0xFFFFu) | (x0 + 1 < w ? 0u : 0xFFFF0000u);
            const uint32_t m1 = (x0 + 2 < w ? 0u : 0xFFFFu) | (x0 + 3 < w ? 0u : 0xFFFF0000u);
            Q[0] = bit_select(m0, nv2, Q[0]);
            Q[1] = bit_select(m1, nv2, Q[1]);
        }
        const uint32_t hl = bin3<T, LM>(raw.halo, lv, thr, lo, W, cpass, lb);
        uint32_t lq = from_lane_below(Q[1]);
        uint32_t rq = from_lane_above(Q[0]);
        if (lane == 0) lq = (xs > 0 ? hl : never) << 16;
        if (lane == 63) rq = xs + 64 * VEC < w ? hl : never;
        P[0] = straddle(lq, Q[0]);
        P[1] = Q[0];
        P[2] = straddle(Q[0], Q[1]);
        P[3] = Q[1];
        P[4] = straddle(Q[1], rq);
    } else {
        uint32_t lam[VEC];
#pragma unroll
        for (int i = 0; i < VEC; ++i)
            lam[i] = x0 + i < w ? bin3<T, LM>(elem3<T>(raw, i), lv, thr, lo, W, cpass, lb) : never;
        const uint32_t hl = bin3<T, LM>(raw.halo, lv, thr, lo, W, cpass, lb);
        uint32_t left = from_lane_below(lam[VEC - 1]);
        uint32_t right = from_lane_above(lam[0]);
        if (lane == 0) left = xs > 0 ? hl : never;
        if (lane == 63) right = xs + 64 * VEC < w ? hl : never;
        P[0] = pack_lo16(left, lam[0]);
#pragma unroll
        for (int i = 1; i < VEC; ++i) P[i] = pack_lo16(lam[i - 1], lam[i]);
        P[VEC] = pack_lo16(lam[VEC - 1], right);
    }
    // rows outside the field (uniform; rare: the first and last planes and
    // rows of the volume) never enter; filled after the conversion, which
    // read a clamped row
    if (!row_ok) {
#pragma unroll
        for (int i = 0; i <= VEC; ++i) P[i] = never | never << 16;
    }
}

// 8-neighbour "entered before" pattern of the two cells of pair j (low / high
// half), rows u (above), m (current), d (below), as offsets into tables of
// 4-byte entries (lut_lo / lut_hi).  The north relation comes in as
// sn = self - up per 16-bit half: that is the south difference of the row
// above, complemented (up - (self + 1) = ~(self - up)), so the rows of a
// column hand it down instead of subtracting again; the tables are indexed
// with the north bit complemented (kNorthFlip2D).  `south` returns this row's
// south difference.
template <int VEC>
__device__ __forceinline__ uint32_t pattern_pair_sn(const uint32_t (&u)[VEC + 1], const uint32_t (&m)[VEC + 1],
                                                    const uint32_t (&d)[VEC + 1], int j, uint32_t sn,
                                                    uint32_t &south) {
    const uint32_t self = m[j], self1 = self + 0x00010001u;
    south = pk_diff(d[j], self);
    return gather_offsets<2>(pk_diff(u[j - 1], self1), sn, pk_diff(u[j + 1], self1), pk_diff(m[j - 1], self1),
                             pk_diff(m[j + 1], self), pk_diff(d[j - 1], self), south, pk_diff(d[j + 1], self));
}

// pattern of the two cells of `self` from their 8 neighbours in one plane:
// u = the row that precedes in memory order (wins ties), w/e = the neighbours
// before/after along the in-row axis, d = the row that follows
__device__ __forceinline__ uint32_t plane_pattern(uint32_t u0, uint32_t u1, uint32_t u2, uint32_t wv, uint32_t ev,
                                                  uint32_t d0, uint32_t d1, uint32_t d2, uint32_t self) {
    const uint32_t self1 = self + 0x00010001u;
    return gather_offsets<2>(pk_diff(u0, self1), pk_diff(u1, self1), pk_diff(u2, self1), pk_diff(wv, self1),
                             pk_diff(ev, self), pk_diff(d0, self), pk_diff(d1, self), pk_diff(d2, self));
}

// per-pixel image of two planes: min (26-C) or max (6-C), packed
template <bool MAXIMG>
__device__ __forceinline__ uint32_t pk_merge(uint32_t a, uint32_t b) {
    const u16x2 x = __builtin_bit_cast(u16x2, a), y = __builtin_bit_cast(u16x2, b);
    if constexpr (MAXIMG)
        return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(x, y));
    else
        return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(x, y));
}

// LDS tables (set up by the host, 256 entries each):
//   tl[p]: layer term of a voxel with layer pattern p, packed as the low
//          word of a 3D bin: (+-EC of the 2D cell) + 7 + (perimeter + 8) << 22,
//          minus 2 << 22 for the min image (see below)
//   tm[p]: 2D EC delta of an image pixel with pattern p, sign included,
//          minus 2 << 22 for the max image
// A voxel's low word is tl[p_layer] + (its share of the two images' deltas)
// - 2 * (vertical neighbours that entered before it) << 22.  Both terms
// come from one relation per voxel, whether the voxel above entered first:
// with ab_z that relation for voxel z, the image between z and z+1 belongs
// to voxel z + 1 when ab_z (min image; to voxel z when ab_z, max image), and
// the vertical neighbours already in number (1 - ab_(z-1)) + ab_z.  So each
// voxel computes u = (its part of its own image term, minus 2 ab_z << 22),
// adds the carry of the voxel below and hands carry = tm - u to the voxel
// above (the biases of the constant parts are in the tables).
// With CR the crease channel comes along: the crease of a voxel is the change
// of kappa over the 12 lattice edges around it; the four edges parallel to one
// axis are the voxel's corners in the plane normal to that axis, so its delta
// is the sum of three 2D deltas looked up by the 8-neighbour patterns of its
// xy (the layer pattern), yz and xz planes (tc: delta + 4 per plane), added to
// a second, 32-bit bin word as crease + 12.
template <typename T, int LM, int AL, bool MAXIMG, bool CR, int TY, typename TH>
struct March3D {
    static constexpr int VEC = Elem3<T>::VEC;
    static constexpr int NR = TY + 2;
    const T *__restrict__ data;
    int d;
    int64_t h, w;
    const LevelArgs &lv;
    const TH &thr;
    int lo, W;
    float cpass;
    const uint32_t *tl;
    const uint32_t *tm;
    uint32_t hist_base;  // LDS address of bin 0 (8 bytes per bin)
    int64_t xs, x0;
    int y0, zb, lane;
    int64_t last_block;
    LaneBins lb;
    const uint32_t *tc;  // CR: per-plane crease deltas + 4
    uint32_t hc_base;    // CR: LDS address of the crease word of bin 0 (4 bytes per bin)

    // Buffers rotate with period NB: three level planes with the crease
    // channel (it needs plane z - 1), two without (one fewer plane and one
    // fewer plane of loads in flight keep the registers under 168, three
    // waves per SIMD)
    static constexpr int NB = CR ? 3 : 2;
    uint32_t R[NB][NR][VEC + 1];  // level planes; R[(z - za + 1) % NB] holds plane z
    uint32_t C[TY][VEC];          // carry from the voxel below each voxel of the current plane
    RawRow3 ring[NB][NR];         // raw rows of upcoming planes; ring[(z - za) % NB] holds plane z + 1

    __device__ __forceinline__ int clampz(int z) const { return z < 0 ? 0 : (z >= d ? d - 1 : z); }
    __device__ __forceinline__ int clampy(int y) const { return y < 0 ? 0 : (y >= (int)h ? (int)h - 1 : y); }
    __device__ __forceinline__ bool row_ok(int z, int y) const { return z >= 0 && z < d && y >= 0 && y < (int)h; }

    __device__ __forceinline__ void fetch_plane(int z, RawRow3 (&dst)[NR]) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
            fetch_row3<T, AL>(data, h, w, clampz(z), clampy(y0 - 1 + r), xs, x0, lane, last_block, dst[r]);
    }
    __device__ __forceinline__ void convert_plane(int z, const RawRow3 (&src)[NR], uint32_t (&dst)[NR][VEC + 1]) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
            convert_row3<T, LM>(src[r], row_ok(z, y0 - 1 + r), w, xs, x0, lane, lv, thr, lo, W, cpass, lb, dst[r]);
    }
    __device__ __forceinline__ void image(const uint32_t (&a)[NR][VEC + 1], const uint32_t (&b)[NR][VEC + 1],
                                          uint32_t (&m)[NR][VEC + 1]) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int i = 0; i <= VEC; ++i) m[r][i] = pk_merge<MAXIMG>(a[r][i], b[r][i]);
    }

    // the share u of a voxel's own image term (see above) from its image
    // delta and the mask of "the voxel above entered first"
    __device__ __forceinline__ static uint32_t own_share(uint32_t tmv, uint32_t ab) {
        if constexpr (MAXIMG)
            return ab & tmv;
        else
            return bit_select(ab, 0xFF800000u, tmv);  // -(2 << 22) when ab
    }
    // per voxel of the pair, all ones when the upper neighbour (sign of the
    // packed difference upper - self) entered first
    __device__ __forceinline__ static uint32_t mask_lo(uint32_t dz) { return (uint32_t)((int32_t)(dz << 16) >> 31); }
    __device__ __forceinline__ static uint32_t mask_hi(uint32_t dz) { return (uint32_t)((int32_t)dz >> 31); }

    // planes za-1 and za converted, the carries of the image between them,
    // planes za+1 .. za+3 in flight
    __device__ __forceinline__ void prologue(int za) {
        {
            RawRow3 a[NR], b[NR];
            fetch_plane(za - 1, a);
            fetch_plane(za, b);
#pragma unroll
            for (int k = 0; k < NB; ++k) fetch_plane(za + 1 + k < zb ? za + 1 + k : zb, ring[k]);
            convert_plane(za - 1, a, R[0]);
            convert_plane(za, b, R[1]);
        }
        uint32_t M[NR][VEC + 1];
        image(R[0], R[1], M);
        uint32_t snm[VEC / 2];  // north relations of the image rows (see pattern_pair_sn)
#pragma unroll
        for (int q = 0; q < VEC / 2; ++q) snm[q] = pk_diff(M[1][2 * q + 1], M[0][2 * q + 1]);
#pragma unroll
        for (int t = 0; t < TY; ++t)
#pragma unroll
            for (int j = 1; j < VEC + 1; j += 2) {
                const uint32_t pm = pattern_pair_sn<VEC>(M[t], M[t + 1], M[t + 2], j, snm[j / 2], snm[j / 2]);
                // voxel za (upper) against voxel za - 1: the upper one is
                // later in memory, so it precedes only when strictly lower
                const uint32_t dz = pk_diff(R[1][t + 1][j], R[0][t + 1][j]);
                const uint32_t t0 = lut_lo<uint32_t, 2>(tm, pm), t1 = lut_hi<uint32_t, 2>(tm, pm);
                C[t][j - 1] = t0 - own_share(t0, mask_lo(dz));
                C[t][j] = t1 - own_share(t1, mask_hi(dz));
            }
    }

    // voxels of plane z, with K = (z - za) % 3
    template <int K>
    __device__ __forceinline__ void step(int z) {
        // (with NB = 2, plane z + 1 replaces plane z - 1, which only the
        // crease channel reads)
        uint32_t(&Pp)[NR][VEC + 1] = R[K % NB];
        uint32_t(&Pc)[NR][VEC + 1] = R[(K + 1) % NB];
        uint32_t(&Pn)[NR][VEC + 1] = R[(K + 2) % NB];
        convert_plane(z + 1, ring[K], Pn);
        fetch_plane(z + 1 + NB < zb ? z + 1 + NB : zb, ring[K]);
        uint32_t M[NR][VEC + 1];
        image(Pc, Pn, M);
        (void)Pp;
        // north relations of the layer and image rows, handed down the column
        uint32_t snl[VEC / 2], snm[VEC / 2];
#pragma unroll
        for (int q = 0; q < VEC / 2; ++q) {
            snl[q] = pk_diff(Pc[1][2 * q + 1], Pc[0][2 * q + 1]);
            snm[q] = pk_diff(M[1][2 * q + 1], M[0][2 * q + 1]);
        }
#pragma unroll
        for (int t = 0; t < TY; ++t) {
            // table reads of the row's VEC voxels first, then their atomics
            uint32_t tlv[VEC], tmv[VEC], dz[VEC / 2], addr[VEC];
            uint32_t crv[CR ? VEC : 1];
#pragma unroll
            for (int q = 0; q < VEC / 2; ++q) {
                const int j = 2 * q + 1;
                const uint32_t self = Pc[t + 1][j];
                const uint32_t pl = pattern_pair_sn<VEC>(Pc[t], Pc[t + 1], Pc[t + 2], j, snl[q], snl[q]);
                const uint32_t pm = pattern_pair_sn<VEC>(M[t], M[t + 1], M[t + 2], j, snm[q], snm[q]);
                // the voxel above (z+1) is later in memory: it entered first
                // only when strictly lower
                dz[q] = pk_diff(Pn[t + 1][j], self);
                addr[2 * q] = mad_lo16(self, 8u, hist_base);
                addr[2 * q + 1] = mad_hi16(self, 8u, hist_base);
                tlv[2 * q] = lut_lo<uint32_t, 2>(tl, pl);
                tlv[2 * q + 1] = lut_hi<uint32_t, 2>(tl, pl);
                tmv[2 * q] = lut_lo<uint32_t, 2>(tm, pm);
                tmv[2 * q + 1] = lut_hi<uint32_t, 2>(tm, pm);
                if constexpr (CR) {
                    // yz plane through the voxel's column, xz plane through its row
                    const uint32_t pyz = plane_pattern(Pp[t][j], Pp[t + 1][j], Pp[t + 2][j], Pc[t][j], Pc[t + 2][j],
                                                       Pn[t][j], Pn[t + 1][j], Pn[t + 2][j], self);
                    const uint32_t pxz = plane_pattern(Pp[t + 1][j - 1], Pp[t + 1][j], Pp[t + 1][j + 1],
                                                       Pc[t + 1][j - 1], Pc[t + 1][j + 1], Pn[t + 1][j - 1],
                                                       Pn[t + 1][j], Pn[t + 1][j + 1], self);
                    // (the layer pattern indexes the north-flipped half of tc)
                    crv[2 * q] = lut_lo<uint32_t, 2>(tc + 256, pl) + lut_lo<uint32_t, 2>(tc, pyz) +
                                 lut_lo<uint32_t, 2>(tc, pxz);
                    crv[2 * q + 1] = lut_hi<uint32_t, 2>(tc + 256, pl) + lut_hi<uint32_t, 2>(tc, pyz) +
                                     lut_hi<uint32_t, 2>(tc, pxz);
                }
            }
#pragma unroll
            for (int q = 0; q < VEC / 2; ++q) {
#pragma unroll
                for (int hv = 0; hv < 2; ++hv) {
                    const int i = 2 * q + hv;
                    const uint32_t u = own_share(tmv[i], hv ? mask_hi(dz[q]) : mask_lo(dz[q]));
                    const uint32_t low = tlv[i] + C[t][i] + u;
                    C[t][i] = tmv[i] - u;
                    constexpr uint64_t cnt = 1ull << kShiftCnt3;
                    lds_add64(addr[i], cnt | low);
                    if constexpr (CR) {
                        const uint32_t self = Pc[t + 1][2 * q + 1];
                        lds_add32(hv ? mad_hi16(self, 4u, hc_base) : mad_lo16(self, 4u, hc_base), crv[i]);
                    }
                }
            }
        }
    }

    __device__ __forceinline__ void run(int za, ProgressPrio &pp, int64_t done0) {
        prologue(za);
        int z = za;
        for (; z + NB <= zb; z += NB) {
            pp.update(done0 + (z - za));
            step<0>(z);
            step<1>(z + 1);
            if constexpr (NB == 3) step<2>(z + 2);
        }
        if (z < zb) step<0>(z);
        if constexpr (NB == 3)
            if (z + 1 < zb) step<1>(z + 1);
    }
};

// Work split: units (column, z) with column = (strip, block of TY rows), z
// fastest, in equal contiguous ranges per wave.  Integer fields at aligned
// addresses without the crease channel hold their registers to three waves
// per SIMD (the other variants would spill).
template <typename T, int LM, int AL, bool MAXIMG, bool CR, int TY>
__global__ void __launch_bounds__(256, (!CR && sizeof(T) < 4 && AL == kLoadAligned) ? 3 : 2)
    ecc3d_stream(const T *__restrict__ data, int64_t d, int64_t h, int64_t w, LevelArgs lv, int32_t lo,
                 int32_t hi, float cpass, const uint32_t *__restrict__ tables,
                 const uint32_t *__restrict__ crease_table, int32_t *__restrict__ partial, int64_t z_lo,
                 int64_t z_hi, int accumulate, int prio, int64_t *acc, int pack_surf) {
    constexpr int VEC = Elem3<T>::VEC;
    extern __shared__ uint64_t smem[];
    __shared__ uint32_t tl[256];
    __shared__ uint32_t tm[256];
    __shared__ uint32_t tc[CR ? 512 : 1];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int W = hi - lo;
    const int L = lv.L;
    // bins [0, W + 2 kBinOff) (kBinOff .. kBinOff + W - 1 are the window's
    // levels), the crease words of the same bins, then thresholds
    const int n_bins = W + 2 * kBinOff;
    uint64_t *hist = smem;
    uint32_t *hc = reinterpret_cast<uint32_t *>(smem + n_bins);  // CR: crease words
    float *thr_s = reinterpret_cast<float *>(hc + (CR ? n_bins : 0));
    constexpr bool kThr = LM == LM_AFFINE || LM == LM_SEARCH;
    if (kThr)
        for (int i = tid; i < W + 3; i += 256) {
            int k = lo - 2 + i;
            k = k < 0 ? 0 : (k >= L ? L - 1 : k);
            thr_s[i] = lv.thr[k];
        }
    tl[tid] = tables[tid];
    tm[tid] = tables[256 + tid];
    if constexpr (CR) {
        tc[tid] = crease_table[tid];
        tc[256 + tid] = crease_table[256 + tid];
    }
    for (int b = tid; b < n_bins; b += 256) {
        hist[b] = 0;
        if constexpr (CR) hc[b] = 0;
    }
    __syncthreads();

    const int G = gridDim.x;
    const int wg = xcd_order(blockIdx.x, G);
    const int64_t gw = (int64_t)wg * kWavesPerWG + wave, NW = (int64_t)G * kWavesPerWG;
    const int64_t D = z_hi - z_lo;
    const int64_t n_strips = (w + 64 * VEC - 1) / (64 * VEC);
    const int64_t n_yb = (h + TY - 1) / TY;
    const int64_t units = n_strips * n_yb * D;
    const int64_t u_end = units * (gw + 1) / NW;
    const ThrLds thr{thr_s, lo - 2};
    const LaneBins lb{(uint32_t)lane, (uint32_t)(W + kBinOff + lane)};
    const int64_t u_beg = units * gw / NW;
    ProgressPrio pp;
    pp.init(prio != 0, u_end - u_beg);
    for (int64_t u = u_beg; u < u_end;) {
        const int64_t col = u / D, za = u % D;
        const int64_t zb = za + (u_end - u) < D ? za + (u_end - u) : D;
        const int64_t strip = col % n_strips, yb = col / n_strips;
        const int64_t xs = strip * 64 * VEC;
        March3D<T, LM, AL, MAXIMG, CR, TY, ThrLds> m{data, (int)d, h, w, lv, thr, lo, W, cpass, tl, tm,
                                                      lds_addr(hist), xs, xs + (int64_t)lane * VEC, (int)(yb * TY),
                                                      (int)(z_lo + zb), lane, d * h * w > VEC ? d * h * w - VEC : 0,
                                                      lb, tc, lds_addr(hc)};
        m.run((int)(z_lo + za), pp, u - u_beg);
        u += zb - za;
    }
    __syncthreads();
    if (acc)
        drain_3d_acc(hist + kBinOff, CR ? hc + kBinOff : nullptr, CR, W, lo, L, acc, pack_surf != 0);
    else
        drain_3d(hist + kBinOff, CR ? hc + kBinOff : nullptr, CR, W, lo, L, G, wg, partial, accumulate == 0);
}


// ---------------------------------------------------------------------------
// 3D (generic: every channel, table lookups over the 8 corner blocks)
// ---------------------------------------------------------------------------
// One tile of TX x TY x TZ voxels: its levels and a one-voxel halo are staged
// into LDS, then each of the 256 threads walks its (x, y) column up the
// tile's planes with a 3x3x3 window.  MODE 0: EC, surface, volume; 1: also
// the crease.  Cells whose level is outside the window [lo, lo + W) add
// nothing.  Starts and ends with the workgroup in step.
typedef uint16_t TileLevels[kTile3DZ + 2][kTile3DY + 2][kTile3DX + 2];

template <typename T, int LM, int MODE>
__device__ __forceinline__ void tile_3d(const T *__restrict__ data, int64_t d, int64_t h, int64_t w,
                                        const LevelArgs &lv, int lo, int W, const int64_t *vt, TileLevels &lam,
                                        uint64_t *hist, uint32_t *hc, int64_t x0, int64_t y0,
                                        int64_t z0) {
    constexpr bool CREASE = MODE == 1;
    constexpr int TX = kTile3DX, TY = kTile3DY, TZ = kTile3DZ;
    constexpr int SX = TX + 2, SY = TY + 2, SZ = TZ + 2;
    const int t = threadIdx.x;
    const int L = lv.L;
    const int lx = t % TX, ly = t / TX;
    for (int e = t; e < SZ * SY * SX; e += 256) {
        const int xx = e % SX, rest = e / SX;
        const int yy = rest % SY, zz = rest / SY;
        const int64_t x = x0 - 1 + xx, y = y0 - 1 + yy, z = z0 - 1 + zz;
        uint32_t l = (uint32_t)L;
        if (x >= 0 && x < w && y >= 0 && y < h && z >= 0 && z < d)
            l = level_of<T, LM>(data[(z * h + y) * w + x], lv, ThrGlobal{lv.thr});
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
            {
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
                const int64_t ec = f0 >> 3, cr = f1 >> 3, surf = f2 >> 3;
                // (the volume field is 1 for every cell: it is the count field)
                const uint64_t word = (uint64_t)(ec + kEcBias3) |
                                      (uint64_t)(surf + kSurfBias3) << kShiftSurf3 |
                                      1ull << kShiftCnt3;
                atomicAdd((unsigned long long *)&hist[p - lo], (unsigned long long)word);
                if (CREASE) atomicAdd(&hc[p - lo], (uint32_t)(cr + kCreaseBias3));
            }
        }
    }
    __syncthreads();
}

template <typename T, int LM, int MODE>
__global__ void __launch_bounds__(256)
    ecc3d_tile(const T *__restrict__ data, int64_t d, int64_t h, int64_t w, LevelArgs lv,
               int32_t lo, int32_t hi, const int64_t *__restrict__ vtab,
               int32_t *__restrict__ partial, int64_t tiles_x, int64_t tiles_y, int64_t n_tiles,
               int flush_tiles) {
    constexpr bool CREASE = MODE == 1;
    extern __shared__ uint64_t smem[];
    __shared__ int64_t vt[256];
    __shared__ TileLevels lam;

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
    bool first = true;
    int since = 0;
    __syncthreads();

    for (int64_t tile = t_beg; tile < t_end; ++tile) {
        const int64_t x0 = (tile % tiles_x) * kTile3DX;
        const int64_t y0 = ((tile / tiles_x) % tiles_y) * kTile3DY;
        const int64_t z0 = (tile / (tiles_x * tiles_y)) * kTile3DZ;
        tile_3d<T, LM, MODE>(data, d, h, w, lv, lo, W, vt, lam, hist, hc, x0, y0, z0);
        if (++since >= flush_tiles) {
            drain_3d(hist, hc, CREASE, W, lo, L, G, wg, partial, first);
            first = false;
            since = 0;
            __syncthreads();
        }
    }
    drain_3d(hist, hc, CREASE, W, lo, L, G, wg, partial, first);
}

// ---------------------------------------------------------------------------
// 3D batched: many volumes in one persistent launch
// ---------------------------------------------------------------------------
// q = floor(e / n) for 0 <= e < 2^15 and 1 <= n <= 2^15, from r = 1/n in
// float32: (e + 0.5) r lies at least 0.5/n from an integer and its rounding
// error is below 2^-8 of that
__device__ __forceinline__ int small_div(int e, float r) { return (int)(((float)e + 0.5f) * r); }

// Levels of a volume in memory (d x h x w, C order).
template <typename T, int LM>
struct VolumeLevels {
    const T *__restrict__ data;
    int64_t h, w;
    const LevelArgs &lv;
    __device__ __forceinline__ uint32_t operator()(int64_t z, int64_t y, int64_t x) const {
        return level_of<T, LM>(data[(z * h + y) * w + x], lv, ThrGlobal{lv.thr});
    }
};

// One tile of tx x ty x tz voxels (shape chosen per volume) of the volume
// whose levels `src(z, y, x)` gives (called for in-volume voxels only): its
// levels and a one-voxel halo are staged into `lam` ((tx+2) x (ty+2) x
// (planes+2) slots), then the threads take the tile's (x, y) columns in rounds
// of 256 and walk each up the planes with a 3x3x3 window, as in the generic
// tile pass.  Starts and ends with the workgroup in step.
template <bool CREASE, typename Src>
__device__ __forceinline__ void tile_3d_flex(const Src &src, int64_t d, int64_t h, int64_t w, int L,
                                             const int64_t *vt, uint16_t *lam, uint64_t *hist, uint32_t *hc,
                                             int64_t x0, int64_t y0, int64_t z0, int tx, int ty, int tz) {
    const int t = threadIdx.x;
    const int sx = tx + 2, sy = ty + 2;
    const int planes = (int)(d - z0 < tz ? d - z0 : tz);
    const int n_st = sx * sy * (planes + 2);
    const float rsx = 1.0f / (float)sx, rsy = 1.0f / (float)sy, rtx = 1.0f / (float)tx;
    for (int e = t; e < n_st; e += 256) {
        const int row = small_div(e, rsx), xx = e - row * sx;
        const int zz = small_div(row, rsy), yy = row - zz * sy;
        const int64_t x = x0 - 1 + xx, y = y0 - 1 + yy, z = z0 - 1 + zz;
        uint32_t l = (uint32_t)L;
        if (x >= 0 && x < w && y >= 0 && y < h && z >= 0 && z < d) l = src(z, y, x);
        lam[e] = (uint16_t)l;
    }
    __syncthreads();
    const int ps = sx * sy;  // plane stride
    for (int c = t; c < tx * ty; c += 256) {
        const int ly = small_div(c, rtx), lx = c - ly * tx;
        if (x0 + lx >= w || y0 + ly >= h) continue;
        const uint16_t *col = lam + ly * sx + lx;  // (dx, dy) = (-1, -1) corner of the column in plane 0
        uint32_t win[27];
#pragma unroll
        for (int pz = 0; pz < 2; ++pz)
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) win[9 + pz * 9 + dy * 3 + dx] = col[pz * ps + dy * sx + dx];
        for (int z = 0; z < planes; ++z) {
#pragma unroll
            for (int k = 0; k < 18; ++k) win[k] = win[k + 9];
            const uint16_t *pl = col + (z + 2) * ps;
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) win[18 + dy * 3 + dx] = pl[dy * sx + dx];
            const uint32_t p = win[13];
            if (p >= (uint32_t)L) continue;
            uint32_t P = 1u << 13;
#pragma unroll
            for (int k = 0; k < 27; ++k) {
                if (k == 13) continue;
                const bool pr = k < 13 ? (win[k] <= p) : (win[k] < p);
                P |= (uint32_t)pr << k;
            }
            int64_t acc = 0;
#pragma unroll
            for (int cc = 0; cc < 8; ++cc) {
                const int cx = cc & 1, cy = cc >> 1 & 1, cz = cc >> 2;
                const uint32_t y = P >> (cz * 9 + cy * 3 + cx);
                const uint32_t m1 = (y & 3u) | ((y >> 1) & 0xCu) | ((y >> 5) & 0x30u) | ((y >> 6) & 0xC0u);
                const uint32_t m0 = m1 & ~(1u << (7 - cc));
                acc += vt[m1] - vt[m0];
            }
            const int64_t f0 = (int16_t)(acc & 0xFFFF);
            acc = (acc - f0) >> 16;
            const int64_t f1 = (int16_t)(acc & 0xFFFF);
            acc = (acc - f1) >> 16;
            const int64_t f2 = (int16_t)(acc & 0xFFFF);
            const int64_t ec = f0 >> 3, cr = f1 >> 3, surf = f2 >> 3;
            const uint64_t word = (uint64_t)(ec + kEcBias3) | (uint64_t)(surf + kSurfBias3) << kShiftSurf3 |
                                  1ull << kShiftCnt3;
            atomicAdd((unsigned long long *)&hist[p], (unsigned long long)word);
            if (CREASE) atomicAdd(&hc[p], (uint32_t)(cr + kCreaseBias3));
        }
    }
    __syncthreads();
}

// Running sums over the L levels of a workgroup's LDS bins straight into the
// field's curves (a field done by one item needs no global histogram).
__device__ __forceinline__ void scan_bins_3d(const uint64_t *hist, const uint32_t *hc, bool crease, int L,
                                             int64_t *const out[4], int64_t (*part)[256]) {
    const int tid = threadIdx.x;
    const int per = (L + 255) / 256;
    const int beg = tid * per, end = beg + per < L ? beg + per : L;
    int64_t s[4] = {0, 0, 0, 0};
    for (int i = beg; i < end; ++i) {
        const uint64_t v = hist[i];
        const int64_t n = (int64_t)(v >> kShiftCnt3);
        s[0] += (int64_t)(v & ((1ull << kShiftSurf3) - 1)) - kEcBias3 * n;
        if (crease) s[1] += (int64_t)hc[i] - kCreaseBias3 * n;
        s[2] += (int64_t)((v >> kShiftSurf3) & ((1ull << (kShiftCnt3 - kShiftSurf3)) - 1)) - kSurfBias3 * n;
        s[3] += n;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) part[c][tid] = s[c];
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {  // inclusive scans of the chunk sums
        int64_t v[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = tid >= off ? part[c][tid - off] : 0;
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 4; ++c) part[c][tid] += v[c];
        __syncthreads();
    }
    int64_t run[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) run[c] = part[c][tid] - s[c];
    for (int i = beg; i < end; ++i) {
        const uint64_t v = hist[i];
        const int64_t n = (int64_t)(v >> kShiftCnt3);
        run[0] += (int64_t)(v & ((1ull << kShiftSurf3) - 1)) - kEcBias3 * n;
        if (crease) run[1] += (int64_t)hc[i] - kCreaseBias3 * n;
        run[2] += (int64_t)((v >> kShiftSurf3) & ((1ull << (kShiftCnt3 - kShiftSurf3)) - 1)) - kSurfBias3 * n;
        run[3] += n;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (out[c]) out[c][i] = run[c];
    }
    __syncthreads();
}

// The host cuts every volume into items of whole tiles (of the volume's tile
// shape) and deals them to workgroups (as for 2D fields).  A workgroup runs an
// item's tiles into LDS bins over all of the field's levels (at most
// kBatchMaxLevels, one pass).  A field of one item is scanned from those bins
// straight into its curves; otherwise the workgroup adds its bins into the
// field's int32 histogram [ec, crease, surface, count][L] with device atomics
// and takes the field's ticket, and the workgroup that finishes the last item
// scans the histogram into the curves and clears it and the ticket for the
// next launch.
template <typename T, int LM>
__global__ void __launch_bounds__(256)
    ecc3d_batch(const BatchField3D *__restrict__ fields, const BatchItem *__restrict__ items,
                const int32_t *__restrict__ wg_first, const int64_t *__restrict__ vt3) {
    extern __shared__ uint64_t smem[];
    __shared__ int64_t vt[2][256];
    __shared__ uint16_t lam[kBatch3DTileElems];
    __shared__ int64_t part[4][256];
    const int tid = threadIdx.x;
    vt[0][tid] = vt3[tid];
    vt[1][tid] = vt3[256 + tid];
    const int i_beg = wg_first[blockIdx.x], i_end = wg_first[blockIdx.x + 1];
    for (int it = i_beg; it < i_end; ++it) {
        const BatchItem item = items[it];
        const BatchField3D &f = fields[item.field];
        const int L = f.L;
        const bool crease = f.out[1] != nullptr;
        uint64_t *hist = smem;
        uint32_t *hc = reinterpret_cast<uint32_t *>(smem + L);
        for (int b = tid; b < L; b += 256) {
            hist[b] = 0;
            hc[b] = 0u;
        }
        __syncthreads();
        LevelArgs lv;
        lv.L = L;
        lv.mode = LM;
        lv.thr = f.thr;
        lv.lut = f.lut;
        lv.u0 = f.u0;
        lv.inv_step = f.inv_step;
        lv.u0d = 0.0;
        lv.eps = f.eps;
        lv.eps_far = f.eps;
        lv.neg = f.neg;
        const int64_t *vtab = vt[f.conn_idx];
        const VolumeLevels<T, LM> src{(const T *)f.data, f.h, f.w, lv};
        for (int tile = item.u0; tile < item.u1; ++tile) {
            const int64_t x0 = (int64_t)(tile % f.tiles_x) * f.tx;
            const int64_t y0 = (int64_t)((tile / f.tiles_x) % f.tiles_y) * f.ty;
            const int64_t z0 = (int64_t)(tile / (f.tiles_x * f.tiles_y)) * f.tz;
            if (crease)  // uniform
                tile_3d_flex<true>(src, f.d, f.h, f.w, L, vtab, lam, hist, hc, x0, y0, z0, f.tx, f.ty, f.tz);
            else
                tile_3d_flex<false>(src, f.d, f.h, f.w, L, vtab, lam, hist, hc, x0, y0, z0, f.tx, f.ty, f.tz);
        }
        if (f.n_items == 1) {  // uniform: the whole field is in this workgroup's bins
            int64_t *const out[4] = {f.out[0], f.out[1], f.out[2], f.out[3]};
            scan_bins_3d(hist, hc, crease, L, out, part);
            continue;
        }
        // bins -> the field's histogram (channels in curve order: ec, crease, surface, count)
        for (int b = tid; b < L; b += 256) {
            const uint64_t v = hist[b];
            const int64_t n = (int64_t)(v >> kShiftCnt3);
            if (n == 0) continue;
            const int64_t surf = (int64_t)((v >> kShiftSurf3) & ((1ull << (kShiftCnt3 - kShiftSurf3)) - 1)) -
                                 kSurfBias3 * n;
            const int64_t ec = (int64_t)(v & ((1ull << kShiftSurf3) - 1)) - kEcBias3 * n;
            int32_t *dst = f.hist + b;
            if (ec) atomicAdd(dst, (int32_t)ec);
            if (crease) {
                const int64_t cr = (int64_t)hc[b] - kCreaseBias3 * n;
                if (cr) atomicAdd(dst + L, (int32_t)cr);
            }
            if (surf) atomicAdd(dst + 2 * L, (int32_t)surf);
            atomicAdd(dst + 3 * L, (int32_t)n);
        }
        // the workgroup that adds last scans the field's histogram into its
        // curves (and clears it)
        if (take_field_ticket(f.done, f.n_items))  // uniform
            scan_field_hist(f.hist, 4, L, f.out, reinterpret_cast<int64_t *>(smem), part[0], f.done);
    }
}

// ---------------------------------------------------------------------------
// 4D fields: slabs along the first axis
// ---------------------------------------------------------------------------
// The closure of the active hypercubes of a field of a slices (each a d x h x
// w volume) splits, like the 3D one, into cells lying in the hyperplanes
// between slices and cells spanning a slice: a cell in hyperplane t (between
// slices t-1 and t, t = 0..a) is present exactly when its 3D counterpart is in
// the closure of the union of those two slices (the "min image" M_t of their
// levels; outside slices never enter), and a cell spanning slice t when its 3D
// counterpart is in the closure of slice t, with one dimension more.  Hence
//   chi80 = sum_t chi26(M_t) - sum_t chi26(slice t),
// and for the face-adjacency complex (blocks of active cells)
//   chi8 = sum_t chi6(slice t) - sum_t chi6(max image of slices t-1, t).
// Boundary 3-faces: those spanning a slice are its 3D surface faces, those in
// hyperplane t separate one active cell from an inactive one, counted from
// the images as 2 |M_t| - |slice t-1| - |slice t| (closure) or
// |slice t-1| + |slice t| - 2 |max image| (faces).  So one pass over the
// "virtual volumes" (the slices, then the images) with the 3D tile pass gives
// every curve: each item adds its bins (EC, surface, count) into per-pass
// accumulators, and a finishing kernel combines and scans them.
template <typename T, int LM>
struct SlabLevels {
    const T *__restrict__ data;
    int64_t a, d, h, w;
    const LevelArgs &lv;
    int64_t t;  // slice or image index
    int mode;   // 0: slice t; 1: min image of slices t-1, t; 2: max image
    __device__ __forceinline__ uint32_t at(int64_t s, int64_t z, int64_t y, int64_t x) const {
        if (s < 0 || s >= a) return (uint32_t)lv.L;
        return level_of<T, LM>(data[((s * d + z) * h + y) * w + x], lv, ThrGlobal{lv.thr});
    }
    __device__ __forceinline__ uint32_t operator()(int64_t z, int64_t y, int64_t x) const {
        if (mode == 0) return at(t, z, y, x);
        const uint32_t l0 = at(t - 1, z, y, x), l1 = at(t, z, y, x);
        return mode == 1 ? (l0 < l1 ? l0 : l1) : (l0 > l1 ? l0 : l1);
    }
};

// items: (virtual volume, tile range); virtual volume v < a is slice v, else
// image t = v - a (closure, t = 0..a) or t = v - a + 1 (faces, t = 1..a-1).
// acc: [kAccCopies][pass][EC, surface, count][L] int64, pass 0 = slices.
template <typename T, int LM>
__global__ void __launch_bounds__(256)
    ecc4d_slabs(const T *__restrict__ data, int64_t a, int64_t d, int64_t h, int64_t w, LevelArgs lv, int faces,
                const BatchItem *__restrict__ items, const int32_t *__restrict__ wg_first,
                const int64_t *__restrict__ vtab, int64_t *__restrict__ acc, int tx, int ty, int tz, int tiles_x,
                int tiles_y) {
    extern __shared__ uint64_t smem[];
    __shared__ int64_t vt[256];
    __shared__ uint16_t lam[kBatch3DTileElems];
    const int tid = threadIdx.x;
    const int L = lv.L;
    vt[tid] = vtab[tid];
    uint64_t *hist = smem;
    int64_t *mine = acc + (int64_t)xcc_copy() * 6 * L;
    const int i_beg = wg_first[blockIdx.x], i_end = wg_first[blockIdx.x + 1];
    for (int it = i_beg; it < i_end; ++it) {
        const BatchItem item = items[it];
        for (int b = tid; b < L; b += 256) hist[b] = 0;
        __syncthreads();
        const int64_t v = item.field;
        const bool slice = v < a;
        const SlabLevels<T, LM> src{data, a, d, h, w, lv, slice ? v : (faces ? v - a + 1 : v - a),
                                    slice ? 0 : (faces ? 2 : 1)};
        for (int tile = item.u0; tile < item.u1; ++tile) {
            const int64_t x0 = (int64_t)(tile % tiles_x) * tx;
            const int64_t y0 = (int64_t)((tile / tiles_x) % tiles_y) * ty;
            const int64_t z0 = (int64_t)(tile / (tiles_x * tiles_y)) * tz;
            tile_3d_flex<false>(src, d, h, w, L, vt, lam, hist, nullptr, x0, y0, z0, tx, ty, tz);
        }
        int64_t *dst = mine + (slice ? 0 : 3 * L);
        for (int b = tid; b < L; b += 256) {
            const uint64_t bin = hist[b];
            const int64_t n = (int64_t)(bin >> kShiftCnt3);
            if (n == 0) continue;
            const int64_t surf = (int64_t)((bin >> kShiftSurf3) & ((1ull << (kShiftCnt3 - kShiftSurf3)) - 1)) -
                                 kSurfBias3 * n;
            const int64_t ec = (int64_t)(bin & ((1ull << kShiftSurf3) - 1)) - kEcBias3 * n;
            acc_add(dst + b, ec);
            acc_add(dst + L + b, surf);
            acc_add(dst + 2 * L + b, n);
        }
        __syncthreads();
    }
}

// Combine the passes per level (see above), scan over levels into the curves
// (NULL outputs skipped) and clear the accumulators; one block.
__global__ void __launch_bounds__(1024)
    ecc4d_finish(int64_t *__restrict__ acc, int L, int faces, OutPtrs out, int64_t *__restrict__ totals) {
    for (int l = threadIdx.x; l < L; l += blockDim.x) {
        int64_t v[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            int64_t x[kAccCopies];  // every copy's load in flight at once
#pragma unroll
            for (int c = 0; c < kAccCopies; ++c) x[c] = acc[((int64_t)c * 6 + k) * L + l];
#pragma unroll
            for (int c = 0; c < kAccCopies; ++c) {
                v[k] += x[c];
                acc[((int64_t)c * 6 + k) * L + l] = 0;
            }
        }
        // v: slices (EC, surface, count), images (EC, surface, count)
        totals[l] = faces ? v[0] - v[3] : v[3] - v[0];
        totals[L + l] = faces ? v[1] + 2 * v[2] - 2 * v[5] : v[1] + 2 * v[5] - 2 * v[2];
        totals[2 * L + l] = v[2];
    }
    __syncthreads();
    scan_totals_block(totals, 3, L, out);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
size_t lds_bytes_3d(int window, bool want_crease) { return (size_t)window * (want_crease ? 12 : 8); }


template <typename T>
static int launch_batch3_t(int lm, const BatchField3D *fields, const BatchItem *items, const int32_t *wg_first,
                           int grid, const int64_t *vt3, size_t lds, hipStream_t s) {
    switch (lm) {
    case LM_IDENTITY:
        if constexpr (sizeof(T) < 4)
            hipLaunchKernelGGL((ecc3d_batch<T, LM_IDENTITY>), dim3(grid), dim3(256), lds, s, fields, items, wg_first,
                               vt3);
        break;
    case LM_LUT:
        if constexpr (sizeof(T) < 4)
            hipLaunchKernelGGL((ecc3d_batch<T, LM_LUT>), dim3(grid), dim3(256), lds, s, fields, items, wg_first, vt3);
        break;
    case LM_AFFINE:
        if constexpr (sizeof(T) == 4)
            hipLaunchKernelGGL((ecc3d_batch<T, LM_AFFINE>), dim3(grid), dim3(256), lds, s, fields, items, wg_first,
                               vt3);
        break;
    default:
        if constexpr (sizeof(T) == 4)
            hipLaunchKernelGGL((ecc3d_batch<T, LM_SEARCH>), dim3(grid), dim3(256), lds, s, fields, items, wg_first,
                               vt3);
        break;
    }
    return (int)hipGetLastError();
}


template <typename T, int LM>
static int launch_4d_t(const Launch4D &g, hipStream_t s) {
    hipLaunchKernelGGL((ecc4d_slabs<T, LM>), dim3(g.grid), dim3(256), lds_bytes_4d(g.lv.L), s, (const T *)g.data,
                       g.a, g.d, g.h, g.w, g.lv, g.faces ? 1 : 0, g.items, g.wg_first, g.vtab, g.acc, g.tx, g.ty,
                       g.tz, g.tiles_x, g.tiles_y);
    return (int)hipGetLastError();
}

int launch_4d(const Launch4D &g, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    int e;
    switch (g.dtype) {
    case ECC_U8: e = g.lv.mode == LM_LUT ? launch_4d_t<uint8_t, LM_LUT>(g, s) : launch_4d_t<uint8_t, LM_IDENTITY>(g, s); break;
    case ECC_U16:
        e = g.lv.mode == LM_LUT ? launch_4d_t<uint16_t, LM_LUT>(g, s) : launch_4d_t<uint16_t, LM_IDENTITY>(g, s);
        break;
    default:
        e = g.lv.mode == LM_AFFINE ? launch_4d_t<float, LM_AFFINE>(g, s) : launch_4d_t<float, LM_SEARCH>(g, s);
        break;
    }
    if (e) return e;
    OutPtrs o;
    for (int c = 0; c < 4; ++c) o.p[c] = c < 3 ? g.out[c] : nullptr;
    hipLaunchKernelGGL(ecc4d_finish, dim3(1), dim3(1024), 0, s, g.acc, g.lv.L, g.faces ? 1 : 0, o, g.totals);
    return (int)hipGetLastError();
}

int launch_batch_3d(int dtype, int lm, const BatchField3D *fields, const BatchItem *items,
                    const int32_t *wg_first, int grid, const int64_t *vt3, int max_L, void *stream) {
    const size_t lds = lds_bytes_batch_3d(max_L);
    hipStream_t s = (hipStream_t)stream;
    if ((dtype == ECC_F32) != (lm == LM_AFFINE || lm == LM_SEARCH)) return (int)hipErrorInvalidValue;
    switch (dtype) {
    case ECC_U8: return launch_batch3_t<uint8_t>(lm, fields, items, wg_first, grid, vt3, lds, s);
    case ECC_U16: return launch_batch3_t<uint16_t>(lm, fields, items, wg_first, grid, vt3, lds, s);
    default: return launch_batch3_t<float>(lm, fields, items, wg_first, grid, vt3, lds, s);
    }
}

template <typename T, int LM, int MODE>
static int launch_3d_t(const Launch3D &a, hipStream_t s) {
    const int64_t tiles_x = (a.w + kTile3DX - 1) / kTile3DX;
    const int64_t tiles_y = (a.h + kTile3DY - 1) / kTile3DY;
    const int64_t tiles_z = (a.d + kTile3DZ - 1) / kTile3DZ;
    const int64_t n_tiles = tiles_x * tiles_y * tiles_z;
    const int flush = (int)(kFlush3D / (kTile3DX * kTile3DY * kTile3DZ));
    const int W = a.hi - a.lo;
    const size_t lds = lds_bytes_3d(W, MODE == 1);
    hipExtLaunchKernelGGL((ecc3d_tile<T, LM, MODE>), dim3(a.grid), dim3(256), lds, s, (hipEvent_t)a.ev_start,
                          (hipEvent_t)a.ev_stop, 0, (const T *)a.data, a.d, a.h, a.w, a.lv, a.lo, a.hi, a.vtab,
                          a.partial, tiles_x, tiles_y, n_tiles, flush);
    return (int)hipGetLastError();
}

// cells one workgroup of the z-marching kernel may add to its bins
static int64_t max_wg_cells_3d(int64_t cols, int64_t depth, int grid) {
    const int64_t NW = (int64_t)grid * kWavesPerWG;
    return kWavesPerWG * ((cols * depth + NW - 1) / NW) * kZmCellsPerUnit;
}

int zmarch_3d_columns(int64_t h, int64_t w) {
    const int64_t n = ((w + kZmStripX - 1) / kZmStripX) * ((h + kZmTY - 1) / kZmTY);
    return n > INT32_MAX ? INT32_MAX : (int)n;
}

bool zmarch_3d_fits(int64_t h, int64_t w, int grid) {
    return max_wg_cells_3d(zmarch_3d_columns(h, w), 1, grid) <= kFlush3D;
}

template <typename T, int LM, int AL, bool MAXIMG, bool CR>
static int launch_zm_t(const Launch3D &a, hipStream_t s) {
    constexpr bool kThr = LM == LM_AFFINE || LM == LM_SEARCH;
    const int W = a.hi - a.lo;
    const int64_t cols = zmarch_3d_columns(a.h, a.w);
    // bound the cells per workgroup between drains by splitting z
    int64_t chunk = a.z_hi - a.z_lo;
    while (chunk > 1 && max_wg_cells_3d(cols, chunk, a.grid) > kFlush3D) chunk = (chunk + 1) / 2;
    if (max_wg_cells_3d(cols, chunk, a.grid) > kFlush3D) return (int)hipErrorInvalidValue;
    const float cpass = pass_constant(a.lv.u0d, a.lo);  // and the margin that holds for it
    LevelArgs lv = a.lv;
    if (a.lo != 0) lv.eps = lv.eps_far;
    const size_t lds = (size_t)(W + 2 * kBinOff) * (CR ? 12 : 8) + (kThr ? (size_t)(W + 3) * 4 : 0);
    for (int64_t z0 = a.z_lo; z0 < a.z_hi; z0 += chunk) {
        const int64_t z1 = z0 + chunk < a.z_hi ? z0 + chunk : a.z_hi;
        const bool acc = a.accumulate || z0 > a.z_lo;
        hipExtLaunchKernelGGL((ecc3d_stream<T, LM, AL, MAXIMG, CR, kZmTY>), dim3(a.grid), dim3(256), lds, s,
                              z0 == a.z_lo ? (hipEvent_t)a.ev_start : nullptr,
                              z1 == a.z_hi ? (hipEvent_t)a.ev_stop : nullptr, 0, (const T *)a.data, a.d, a.h, a.w,
                              lv, a.lo, a.hi, cpass, a.zm_tables, a.crease_table, a.partial, z0, z1, acc ? 1 : 0,
                              progress_prio() ? 1 : 0, a.acc, a.acc && a.pack_surf ? 1 : 0);
        const int e = (int)hipGetLastError();
        if (e) return e;
    }
    return 0;
}

template <typename T, int LM, bool MAXIMG>
static int launch_zm_al(const Launch3D &a, hipStream_t s) {
    constexpr int VB = Elem3<T>::VEC * (int)sizeof(T);
    const bool al = (uintptr_t)a.data % VB == 0 && (a.w * (int64_t)sizeof(T)) % VB == 0;
    if (a.crease_table)
        return al ? launch_zm_t<T, LM, kLoadAligned, MAXIMG, true>(a, s)
                  : launch_zm_t<T, LM, kLoadVector, MAXIMG, true>(a, s);
    return al ? launch_zm_t<T, LM, kLoadAligned, MAXIMG, false>(a, s)
              : launch_zm_t<T, LM, kLoadVector, MAXIMG, false>(a, s);
}


template <typename T, int LM>
static int launch_3d_cr(const Launch3D &a, hipStream_t s) {
    if (a.zm_tables) return a.conn6 ? launch_zm_al<T, LM, true>(a, s) : launch_zm_al<T, LM, false>(a, s);
    return a.want_crease ? launch_3d_t<T, LM, 1>(a, s) : launch_3d_t<T, LM, 0>(a, s);
}

template <typename T>
static int launch_3d_dt(const Launch3D &a, hipStream_t s) {
    if constexpr (sizeof(T) < 4)
        return a.lv.mode == LM_LUT ? launch_3d_cr<T, LM_LUT>(a, s) : launch_3d_cr<T, LM_IDENTITY>(a, s);
    else
        return a.lv.mode == LM_AFFINE ? launch_3d_cr<T, LM_AFFINE>(a, s) : launch_3d_cr<T, LM_SEARCH>(a, s);
}

int launch_3d(const Launch3D &a, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    switch (a.dtype) {
    case ECC_U8: return launch_3d_dt<uint8_t>(a, s);
    case ECC_U16: return launch_3d_dt<uint16_t>(a, s);
    default: return launch_3d_dt<float>(a, s);
    }
}

}  // namespace ecc
