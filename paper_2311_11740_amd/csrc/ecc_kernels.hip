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
// Kernel layout (details at each kernel):
//   * 2D (`ecc2d_stream`): a wave streams the rows of a strip of columns from
//     HBM (one vector load per lane and row, several rows in flight), maps
//     values to level indices once, forms each cell's "entered before"
//     neighbour pattern from packed 16-bit differences and adds the cell's
//     packed delta to the workgroup's LDS histogram with one 64-bit atomic
//     (fields biased to stay non-negative, see ecc_internal.h);
//   * 3D (`ecc3d_stream`): a wave marches the z-planes of a column of 4 rows
//     x 256 columns with a slab decomposition that needs two 2D patterns per
//     voxel, and two more (its yz and xz planes) when the crease channel is
//     wanted; `ecc3d_tile` (LDS-staged
//     3x3x3 windows) computes every channel for planes too large to march, and
//     the vertex class counts;
//   * the 2D kernel also counts vertex classes (two words per level bin);
//   * each workgroup drains its histogram into its slice of level-major
//     partials; `ecc_merge` sums them per level and its last block scans;
//   * `ecc2d_batch` runs many fields in one persistent launch.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include <algorithm>

#include "ecc_internal.h"

namespace ecc {

// ---------------------------------------------------------------------------
// level index: first l with value <= t_l (Eq. (2)); L = never active
// ---------------------------------------------------------------------------
// Thresholds are read through one of two accessors so that the compiler
// emits LDS reads (ds_read) or global reads, never generic flat accesses.
// ThrLds holds the window of thresholds [base, base + n) of one level pass.
struct ThrLds {
    const float *p;
    int base;
    __device__ float operator[](int i) const { return p[i - base]; }
};
struct ThrGlobal {
    const float *__restrict__ p;
    __device__ float operator[](int i) const { return p[i]; }
};

template <int LM, typename TH>
__device__ __forceinline__ uint32_t level_of_float(float x, const LevelArgs &a, const TH &thr) {
    const int L = a.L;
    if (!(x == x)) return (uint32_t)L;  // NaN never enters
    if constexpr (LM == LM_AFFINE) {
        const float u = __builtin_fmaf(x, a.inv_step, a.u0);
        const float fr = __builtin_amdgcn_fractf(u);
        const float uc = __builtin_amdgcn_fmed3f(u, -2.0f, (float)L + 2.0f);
        int g = (int)__builtin_floorf(uc) + 1;
        g = g < 0 ? 0 : (g > L ? L : g);
        if (!(__builtin_fabsf(fr - 0.5f) <= 0.5f - a.eps)) {
            // within eps of a grid point: the level is g-1, g or g+1 (the
            // host bounds the grid deviation plus rounding below one step);
            // settle it against the caller's thresholds
            const float ta = thr[g > 0 ? g - 1 : 0], tb = thr[g < L ? g : L - 1];
            if (g > 0 && x <= ta)
                --g;
            else if (g < L && !(x <= tb))
                ++g;
        }
        return (uint32_t)g;
    } else {
        int lo = 0, hi = L;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (x <= thr[mid])
                hi = mid;
            else
                lo = mid + 1;
        }
        return (uint32_t)lo;
    }
}

template <typename T, int LM, typename TH>
__device__ __forceinline__ uint32_t level_of(T v, const LevelArgs &a, const TH &thr) {
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
// One wave walks down a run of rows of a strip of columns, keeping the level
// indices of three rows (above, current, below) in registers.  Each lane
// holds VEC consecutive cells of a row (16 bytes of input).  Strips overlap by
// one lane on each side: lanes 1..62 own the strip's 62*VEC cells, lanes 0
// and 63 hold the cells just left and right of them and only serve as halo,
// so a full strip reads each row with one unconditional 16-byte load per lane
// and gets every horizontal neighbour by a lane shuffle.  Raw rows are fetched
// PF rows ahead into a register ring so that several row loads per wave are
// in flight.
//
// Level indices of a row are kept as VEC+1 packed 16-bit pairs
// P[i] = (lam[i], lam[i+1]) where lam[0] and lam[VEC+1] are the neighbours
// from the adjacent lanes.  For the two cells (j, j+1) of P[j] every
// neighbour pair is one of these words (W = P[j-1], E = P[j+1], and P[j-1..j+1]
// of the rows above and below), so each "entered before" relation of both
// cells is one packed subtraction: q precedes p  <=>  q < p (later
// neighbours) or q < p + 1 (earlier neighbours, which win ties).
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
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));

// per 16-bit half: 1 when q < ref (both in [0, 2^15)), else 0
__device__ __forceinline__ uint32_t pk_lt(uint32_t q, uint32_t ref) {
    const i16x2 d = __builtin_bit_cast(i16x2, q) - __builtin_bit_cast(i16x2, ref);
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, d) >> (unsigned short)15);
}

// Pattern of the 8 neighbours of two cells.  d[k] = q_k - ref_k per 16-bit
// half (k = NW N NE W E SW S SE, ref = cell level, +1 for neighbours that win
// ties), so the sign bit of each half says whether neighbour k entered
// before that cell.  The index of a cell has bit i (i < 4) for neighbour 2i
// and bit 4 + i for neighbour 2i + 1 (the host tables are built in this
// order).  Returned as byte offsets into a table of 2^S-byte entries: the low
// cell's is y & (0xFF << S), the high cell's (y >> 8) & (0xFF << S); the
// other bits of y are garbage.
__device__ __forceinline__ uint32_t pk_diff(uint32_t q, uint32_t ref) {
    return __builtin_bit_cast(uint32_t, __builtin_bit_cast(i16x2, q) - __builtin_bit_cast(i16x2, ref));
}

// (m & a) | (~m & b) in one three-input bitwise operation (truth table 0xCA:
// the first operand selects between the other two)
__device__ __forceinline__ uint32_t bit_select(uint32_t m, uint32_t a, uint32_t b) {
    return __builtin_amdgcn_bitop3_b32(m, a, b, (unsigned char)0xCA);
}

template <int S>
__device__ __forceinline__ uint32_t gather_offsets(uint32_t d0, uint32_t d1, uint32_t d2, uint32_t d3, uint32_t d4,
                                                   uint32_t d5, uint32_t d6, uint32_t d7) {
    // a byte permute with selectors 8-11 turns the sign bits of two words into
    // 0x00/0xFF bytes: [low cell, even k | high cell, even k | low cell, odd k
    // | high cell, odd k]
    constexpr uint32_t kSel = 0x0B0A0908u;
    const uint32_t p0 = __builtin_amdgcn_perm(d1, d0, kSel);
    const uint32_t p1 = __builtin_amdgcn_perm(d3, d2, kSel);
    const uint32_t p2 = __builtin_amdgcn_perm(d5, d4, kSel);
    const uint32_t p3 = __builtin_amdgcn_perm(d7, d6, kSel);
    // bit S + i of every byte from p_i (bit selects; the other bits are don't-care)
    constexpr uint32_t B = 0x01010101u << S, B2 = 0x01010101u << (S + 2), B01 = 0x03030303u << S;
    const uint32_t t01 = bit_select(B, p0, p1);
    const uint32_t t23 = bit_select(B2, p2, p3);
    const uint32_t r = bit_select(B01, t01, t23);
    // even-k nibbles stay, odd-k nibbles (bytes 2, 3) move down next to them
    constexpr uint32_t M = (0x0Fu << S) | (0x0Fu << (S + 8));
    return bit_select(M, r, r >> 12);
}

template <typename E, int S>
__device__ __forceinline__ E lut_lo(const E *t, uint32_t y) {
    return *reinterpret_cast<const E *>(reinterpret_cast<const char *>(t) + (y & (0xFFu << S)));
}
template <typename E, int S>
__device__ __forceinline__ E lut_hi(const E *t, uint32_t y) {
    return *reinterpret_cast<const E *>(reinterpret_cast<const char *>(t) + ((y >> 8) & (0xFFu << S)));
}

struct RawRow {
    uint32_t w[4];   // 16 bytes: VEC raw elements of this lane
    uint32_t valid;  // bit i: element i lies inside the field
    uint32_t shift;  // elements the block must move down (loads clamped at the buffer end)
};

typedef u32x4 u32x4_u __attribute__((aligned(1)));

// How a lane loads its VEC elements of a row:
//  kLoadAligned: base and row pitch are multiples of 16 bytes, so each lane's
//    block lies wholly inside the row or wholly outside it; one 16-byte load
//    (clamped to column 0 when outside).
//  kLoadVector: any alignment; one 16-byte load at the block's address (the
//    hardware serves unaligned vector loads).  Elements past the row end come
//    from the next row and are masked.  A block that would run past the end
//    of the buffer is loaded from the last 16 bytes of the buffer instead and
//    shifted back into place when converted.  Fields of fewer than VEC
//    elements are handed over padded to VEC elements by the host.
// The row index is clamped into the field by the caller: loads are never
// skipped, so the compiler can keep several of them in flight (a skipped load
// would make it wait for all outstanding ones).
enum LoadMode : int { kLoadVector = 1, kLoadAligned = 2 };

template <typename T, int AL>
__device__ __forceinline__ void fetch_row(const T *__restrict__ data, int r, int64_t w, int64_t x0,
                                          int64_t last_block, RawRow &raw) {
    constexpr int VEC = Elem<T>::VEC;
    const T *row = data + (int64_t)r * w;
    const bool in = x0 >= 0 && x0 < w;
    if constexpr (AL == kLoadAligned) {
        const u32x4 q = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(row + (in ? x0 : 0)));
        raw.w[0] = q.x; raw.w[1] = q.y; raw.w[2] = q.z; raw.w[3] = q.w;
        raw.valid = in ? (1u << VEC) - 1u : 0u;
        raw.shift = 0;
    } else {
        const int64_t li = (int64_t)r * w + (in ? x0 : 0);      // element index of the block
        const int64_t lc = li < last_block ? li : last_block;  // last_block = h * w - VEC
        const u32x4 q = __builtin_nontemporal_load(reinterpret_cast<const u32x4_u *>(data + lc));
        raw.w[0] = q.x; raw.w[1] = q.y; raw.w[2] = q.z; raw.w[3] = q.w;
        const int64_t n_in = in ? w - x0 : 0;
        raw.valid = n_in >= VEC ? (1u << VEC) - 1u : (1u << n_in) - 1u;
        raw.shift = (uint32_t)(li - lc);
    }
}

// moves a block loaded from a clamped address down by raw.shift elements
template <typename T>
__device__ __forceinline__ void unshift_row(RawRow &raw) {
    const uint32_t sb = raw.shift * (uint32_t)sizeof(T);  // bytes, < 16
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

// exact level of x given an estimate g that is off by at most one; only
// called for g in [lo - 1, hi], whose neighbouring thresholds are staged
template <typename TH>
__device__ __forceinline__ uint32_t level_settle(float x, uint32_t g, int L, const TH &thr) {
    if (!(x == x)) return (uint32_t)L;
    const int gi = (int)g;
    const float a = thr[gi > 0 ? gi - 1 : 0], b = thr[gi < L ? gi : L - 1];
    const int dec = (gi > 0 && x <= a) ? 1 : 0;
    const int inc = (gi < L && !(x <= b)) ? 1 : 0;
    return (uint32_t)(gi - dec + inc);
}

// level of x mapped into the pass window (see convert_row) by a binary search
// over the staged thresholds [lo - 1, hi)
template <typename TH>
__device__ __forceinline__ uint32_t level_search_window(float x, int lo, int hi, const TH &thr) {
    const int W = hi - lo;
    if (lo > 0 && x <= thr[lo - 1]) return 0u;
    if (!(x <= thr[hi - 1])) return (uint32_t)(W + 1);  // also NaN
    int a = lo, b = hi - 1;                              // x <= thr[b]
    while (a < b) {
        const int m = (a + b) >> 1;
        if (x <= thr[m])
            b = m;
        else
            a = m + 1;
    }
    return (uint32_t)(a - lo + 1);
}

// Level indices of one row mapped into the pass window [lo, lo + W) as
// lam' = clamp(lam - lo + 1, 0, W + 1): 0 below the window, 1..W inside, W+1
// above it and for cells that never enter.  For a cell inside the window every
// "entered before" relation is unchanged, and lam' <= 4097 fits the packed
// 16-bit compares.  Packed as pairs P[i] = (lam'[i-1], lam'[i]) of the lane's
// cells, with the neighbouring lanes' cells at both ends.
//
// Float fields with (nearly) evenly spaced thresholds: y = fma(x, 1/step, c)
// with c = -t0/step + 1.5 - lo estimates lam' - 0.5; adding 1.5*2^23 rounds y
// to an integer k in the low mantissa bits of m (exact for |y| < 2^22), and
// r = y - k is the rounding residual.  k = lam' unless |r| is within eps of
// 1/2, i.e. x sits within the host's error bound of a threshold; those cells
// are settled against the thresholds.
constexpr float kMagic = 12582912.0f;  // 1.5 * 2^23
constexpr uint32_t kMagicBits = 0x4B400000u;

__device__ __forceinline__ uint32_t pack_lo16(uint32_t a, uint32_t b) {  // (a.lo, b.lo)
    return __builtin_amdgcn_perm(b, a, 0x05040100u);
}

// Integer values with identity levels, two per word: the pair of values in
// the 16-bit halves of q mapped to lam' = min(max(v + 1 - lo, 0), W + 1) with
// saturating packed arithmetic (a value at or above L lands on W + 1 too).
__device__ __forceinline__ uint32_t identity_pair(uint32_t q, uint32_t lo2, uint32_t never2) {
    u16x2 v = __builtin_bit_cast(u16x2, q);
    v = __builtin_elementwise_add_sat(v, (u16x2){1, 1});
    v = __builtin_elementwise_sub_sat(v, __builtin_bit_cast(u16x2, lo2));
    v = __builtin_elementwise_min(v, __builtin_bit_cast(u16x2, never2));
    return __builtin_bit_cast(uint32_t, v);
}

// values k and k+1 (k even) of a lane's raw block as the halves of a word
template <typename T>
__device__ __forceinline__ uint32_t raw_pair(const uint32_t *w, int k) {
    if constexpr (sizeof(T) == 2)
        return w[k >> 1];
    else  // bytes k, k+1 of the block into the low bytes of the two halves
        return __builtin_amdgcn_perm(0u, w[k >> 2], (k & 2) ? 0x0C030C02u : 0x0C010C00u);
}

// (a.hi, b.lo): the 16-bit value just below b's low half
__device__ __forceinline__ uint32_t straddle(uint32_t a, uint32_t b) {
    return __builtin_amdgcn_alignbit(b, a, 16);
}

template <typename T, int LM, typename TH>
__device__ __forceinline__ void convert_row(const RawRow &raw_in, bool row_ok, bool full, const LevelArgs &lv,
                                            const TH &thr, int lo, int W, float cpass,
                                            uint32_t (&P)[Elem<T>::VEC + 1]) {
    constexpr int VEC = Elem<T>::VEC;
    const uint32_t never = (uint32_t)(W + 1);
    if (!row_ok) {  // uniform
#pragma unroll
        for (int i = 0; i <= VEC; ++i) P[i] = never | never << 16;
        return;
    }
    RawRow raw = raw_in;
    if (__any(raw.shift != 0)) unshift_row<T>(raw);  // rare: blocks at the end of the buffer
    if constexpr (LM == LM_IDENTITY) {  // integer values, two per packed operation
        const uint32_t lo2 = (uint32_t)lo * 0x10001u, nv2 = never * 0x10001u;
        uint32_t Q[VEC / 2];  // Q[k] = (lam'[2k], lam'[2k+1])
#pragma unroll
        for (int k = 0; k < VEC / 2; ++k) Q[k] = identity_pair(raw_pair<T>(raw.w, 2 * k), lo2, nv2);
        if (!full) {  // uniform: cells outside the field never enter
#pragma unroll
            for (int k = 0; k < VEC / 2; ++k) {
                const uint32_t m = ((raw.valid >> (2 * k)) & 1u ? 0u : 0xFFFFu) |
                                   ((raw.valid >> (2 * k + 1)) & 1u ? 0u : 0xFFFF0000u);
                Q[k] = (Q[k] & ~m) | (nv2 & m);
            }
        }
        const uint32_t lq = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)Q[VEC / 2 - 1], 0x138, 0xf, 0xf, false);
        const uint32_t rq = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)Q[0], 0x130, 0xf, 0xf, false);
        P[0] = straddle(lq, Q[0]);
#pragma unroll
        for (int k = 0; k < VEC / 2; ++k) {
            P[2 * k + 1] = Q[k];
            P[2 * k + 2] = straddle(Q[k], k + 1 < VEC / 2 ? Q[k + 1] : rq);
        }
        return;
    }
    uint32_t lam[VEC];  // low 16 bits: lam'
    const int base = lo - 1;
    if constexpr (LM == LM_AFFINE) {
        const float hme = 0.5f - lv.eps;
        // estimates clamp to [0, W + 1]; in the first pass to [1, W + 1],
        // since every value at or below t0 (however far) has level 0
        const float mlo = lo == 0 ? kMagic + 1.0f : kMagic;
        const float mhi = kMagic + (float)never;
        bool nr[VEC];
        bool any = false;
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
            const float y = __builtin_fmaf(__uint_as_float(raw.w[i]), lv.inv_step, cpass);
            const float m = y + kMagic;
            const float r = y - (m - kMagic);
            nr[i] = !(__builtin_fabsf(r) <= hme);  // also NaN and +-inf
            lam[i] = __float_as_uint(__builtin_amdgcn_fmed3f(m, mlo, mhi));
            any |= nr[i];
        }
        if (__any(any)) {  // rare: a value within eps of a threshold
#pragma unroll
            for (int i = 0; i < VEC; ++i) {
                const int k = (int)(lam[i] - kMagicBits);  // clamped estimate of lam'
                if (nr[i] && k >= 0 && k <= W + 1) {
                    // only estimates inside or next to the window can matter;
                    // the estimate is a level, so at least 0 (k = 0 with lo = 0
                    // would otherwise stand for level -1)
                    const int g0 = k + base < 0 ? 0 : k + base;
                    const int g = level_settle(__uint_as_float(raw.w[i]), (uint32_t)g0, lv.L, thr);
                    lam[i] = (uint32_t)min(max(g - base, 0), (int)never);
                }
            }
        }
    } else if constexpr (LM == LM_SEARCH) {
#pragma unroll
        for (int i = 0; i < VEC; ++i) lam[i] = level_search_window(as_value<float>(raw.w[i]), lo, lo + W, thr);
    } else {
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
            const int l = (int)level_of<T, LM>(as_value<T>(Elem<T>::get(raw.w, i)), lv, thr);
            lam[i] = (uint32_t)min(max(l - base, 0), (int)never);
        }
    }
    if (!full) {  // uniform: some lanes hold cells outside the field
#pragma unroll
        for (int i = 0; i < VEC; ++i)
            if (!(raw.valid >> i & 1u)) lam[i] = never;
    }
    // neighbours from the adjacent lanes by DPP wave shifts (lane 0's left and
    // lane 63's right are never used: those lanes only serve as halo)
    const uint32_t left = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)lam[VEC - 1], 0x138, 0xf, 0xf, false);
    const uint32_t right = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)lam[0], 0x130, 0xf, 0xf, false);
    P[0] = pack_lo16(left, lam[0]);
#pragma unroll
    for (int i = 1; i < VEC; ++i) P[i] = pack_lo16(lam[i - 1], lam[i]);
    P[VEC] = pack_lo16(lam[VEC - 1], right);
}

// Partials are stored level-major, [channel][level][workgroup] (int32), so that
// the merge reads the values of one bin contiguously.
__device__ __forceinline__ void drain_2d(const uint64_t *hist, int W, int lo, int L, int G, int wg,
                                         int32_t *__restrict__ partial, bool first) {
    for (int b = threadIdx.x; b < W; b += blockDim.x) {
        const uint64_t v = hist[b];
        const int64_t n = (int64_t)(v >> kShiftCnt2);
        const int64_t per = (int64_t)((v >> kShiftPer2) & ((1ull << (kShiftCnt2 - kShiftPer2)) - 1)) -
                            kPerBias2 * n;
        const int64_t ec = (int64_t)(v & ((1ull << kShiftPer2) - 1)) - kEcBias2 * n;
        const int64_t i0 = ((int64_t)(lo + b)) * G + wg, cs = (int64_t)L * G;
        if (first) {
            partial[i0] = (int32_t)ec;
            partial[i0 + cs] = (int32_t)per;
            partial[i0 + 2 * cs] = (int32_t)n;
        } else {
            partial[i0] += (int32_t)ec;
            partial[i0 + cs] += (int32_t)per;
            partial[i0 + 2 * cs] += (int32_t)n;
        }
    }
}

// class-count bins (two words per level) -> partials [class][level][workgroup]
__device__ __forceinline__ void drain_cls(const uint64_t *hist, int W, int lo, int L, int G, int wg,
                                          int32_t *__restrict__ partial, bool first) {
    constexpr uint64_t m21 = (1ull << kClsShift1) - 1;
    for (int b = threadIdx.x; b < W; b += blockDim.x) {
        const uint64_t v0 = hist[2 * b], v1 = hist[2 * b + 1];
        const int64_t n = (int64_t)(v0 >> kClsShift2);
        int32_t c[5];
        c[0] = (int32_t)((int64_t)(v0 & m21) - kClsBias * n);
        c[1] = (int32_t)((int64_t)((v0 >> kClsShift1) & m21) - kClsBias * n);
        c[2] = (int32_t)((int64_t)(v1 & m21) - kClsBias * n);
        c[3] = (int32_t)((int64_t)((v1 >> kClsShift1) & m21) - kClsBias * n);
        c[4] = (int32_t)(v1 >> kClsShift2);
        const int64_t i0 = ((int64_t)(lo + b)) * G + wg, cs = (int64_t)L * G;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            if (first)
                partial[i0 + k * cs] = c[k];
            else
                partial[i0 + k * cs] += c[k];
        }
    }
}

// The deltas of the VEC cells of `mid` into the LDS bins: the bin of a cell
// is lam' itself (hist[1..W] are the levels of the pass window).  Cells
// outside the window (lam' = 0 or W + 1, among them every cell outside the
// field) and every cell of a halo lane (whose window wl is 0) go to the
// lane's own scratch bin, which is never drained: masses of such cells would
// otherwise all hit one address, and the atomics stay unconditional, so all
// table reads of a group can be issued before its atomics.
// With CLS the bins hold class counts: two words per bin (hist[2 * bin] and
// hist[2 * bin + 1]) and two tables (dl[0..255], dl[256..511]).
template <int VEC, bool CLS>
__device__ __forceinline__ void emit_row(const uint32_t (&up)[VEC + 1], const uint32_t (&mid)[VEC + 1],
                                         const uint32_t (&dn)[VEC + 1], uint32_t wl, uint32_t scratch,
                                         const uint64_t *dl, uint64_t *hist) {
    // groups of up to 4 cell pairs: all table reads of a group are issued
    // before its atomics, so the atomics wait for one LDS round trip, not one each
    constexpr int NP = VEC / 2, GP = CLS ? (NP < 2 ? NP : 2) : (NP < 4 ? NP : 4);
#pragma unroll
    for (int g0 = 0; g0 < NP; g0 += GP) {
        uint64_t dv[2 * GP], dv2[CLS ? 2 * GP : 1];
        uint32_t bin[2 * GP];
#pragma unroll
        for (int q = 0; q < GP; ++q) {
            const int j = 2 * (g0 + q) + 1;
            const uint32_t self = mid[j], self1 = self + 0x00010001u;
            const uint32_t acc = gather_offsets<3>(pk_diff(up[j - 1], self1), pk_diff(up[j], self1),
                                                   pk_diff(up[j + 1], self1), pk_diff(mid[j - 1], self1),
                                                   pk_diff(mid[j + 1], self), pk_diff(dn[j - 1], self),
                                                   pk_diff(dn[j], self), pk_diff(dn[j + 1], self));
            const uint32_t b0 = self & 0xFFFFu, b1 = self >> 16;
            bin[2 * q] = b0 - 1u < wl ? b0 : scratch;
            bin[2 * q + 1] = b1 - 1u < wl ? b1 : scratch;
            dv[2 * q] = lut_lo<uint64_t, 3>(dl, acc);
            dv[2 * q + 1] = lut_hi<uint64_t, 3>(dl, acc);
            if constexpr (CLS) {
                dv2[2 * q] = lut_lo<uint64_t, 3>(dl + 256, acc);
                dv2[2 * q + 1] = lut_hi<uint64_t, 3>(dl + 256, acc);
            }
        }
#pragma unroll
        for (int q = 0; q < 2 * GP; ++q) {
            if constexpr (CLS) {
                atomicAdd((unsigned long long *)&hist[2 * bin[q]], (unsigned long long)dv[q]);
                atomicAdd((unsigned long long *)&hist[2 * bin[q] + 1], (unsigned long long)dv2[q]);
            } else {
                atomicAdd((unsigned long long *)&hist[bin[q]], (unsigned long long)dv[q]);
            }
        }
    }
}

// rows [ra, rb) of one strip; three row buffers whose roles rotate with the
// row index (PF is a multiple of 3, so the unrolled loop needs no copies)
template <typename T, int LM, int AL, int PF, bool CLS, typename TH>
__device__ __forceinline__ void stream_run_2d(const T *__restrict__ data, int h, int64_t w,
                                              const LevelArgs &lv, const TH &thr, int32_t lo, int W,
                                              float cpass, const uint64_t *dl, uint64_t *hist, int64_t strip,
                                              int ra, int rb, int lane, uint32_t wl, uint32_t scratch) {
    static_assert(PF % 3 == 0, "PF must be a multiple of 3");
    constexpr int VEC = Elem<T>::VEC;
    constexpr int CE = 62 * VEC;  // cells owned per strip
    const int64_t xs = strip * CE - VEC;  // first column of lane 0
    const int64_t x0 = xs + (int64_t)lane * VEC;
    const bool full = xs >= 0 && xs + 64 * VEC <= w;
    auto clamp_row = [h](int r) { return r < 0 ? 0 : (r >= h ? h - 1 : r); };
    // tiny fields arrive padded to one whole block, so the clamp stays at or above 0
    const int64_t last_block = (int64_t)h * w > VEC ? (int64_t)h * w - VEC : 0;

    uint32_t R[3][VEC + 1];  // R[r % 3] holds row r (relative to ra)
    RawRow ring[PF];
    {
        RawRow r0, r1;
        fetch_row<T, AL>(data, clamp_row(ra - 1), w, x0, last_block, r0);
        fetch_row<T, AL>(data, ra, w, x0, last_block, r1);
        // ring[k] holds row ra + 1 + k (rows past rb are clamped reloads)
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int rr = ra + 1 + k < rb ? ra + 1 + k : rb;
            fetch_row<T, AL>(data, clamp_row(rr), w, x0, last_block, ring[k]);
        }
        convert_row<T, LM>(r0, ra - 1 >= 0, full, lv, thr, lo, W, cpass, R[2]);
        convert_row<T, LM>(r1, true, full, lv, thr, lo, W, cpass, R[0]);
    }
    int r0 = ra;
    // full blocks of PF rows: no conditional loads, so PF loads stay in flight
    for (; r0 + PF <= rb; r0 += PF) {
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int r = r0 + k;  // current row (buffer k%3); ring[k] holds row r + 1
            convert_row<T, LM>(ring[k], r + 1 < h, full, lv, thr, lo, W, cpass, R[(k + 1) % 3]);
            const int nx = r + 1 + PF < rb ? r + 1 + PF : rb;
            fetch_row<T, AL>(data, clamp_row(nx), w, x0, last_block, ring[k]);
            emit_row<VEC, CLS>(R[(k + 2) % 3], R[k % 3], R[(k + 1) % 3], wl, scratch, dl, hist);
        }
    }
    // remaining rows (fewer than PF); here r - ra = r0 - ra + k with r0 - ra
    // a multiple of PF, so the buffer roles are those of k again
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        const int r = r0 + k;
        if (r < rb) {
            convert_row<T, LM>(ring[k], r + 1 < h, full, lv, thr, lo, W, cpass, R[(k + 1) % 3]);
            emit_row<VEC, CLS>(R[(k + 2) % 3], R[k % 3], R[(k + 1) % 3], wl, scratch, dl, hist);
        }
    }
}

// Work split: the (strip, row) units of rows [row_lo, row_hi), strip-major,
// are divided into equal contiguous ranges, one per wave (a range may run from
// the end of one strip into the next).
template <typename T, int LM, int AL, int PF, bool CLS>
__global__ void __launch_bounds__(256)
    ecc2d_stream(const T *__restrict__ data, int64_t h, int64_t w, LevelArgs lv, int32_t lo,
                 int32_t hi, float cpass, const uint64_t *__restrict__ delta_lut, int32_t *__restrict__ partial,
                 int64_t row_lo, int64_t row_hi, int accumulate) {
    constexpr int VEC = Elem<T>::VEC;
    constexpr int CE = 62 * VEC;
    constexpr int BW = CLS ? 2 : 1;  // words per bin
    extern __shared__ uint64_t smem[];
    __shared__ uint64_t dl[256 * BW];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: keeps loop control scalar
    const int W = hi - lo;
    const int L = lv.L;
    // LDS: bins 0..W+1 (1..W are the window's levels), a scratch bin per
    // lane, then thresholds [lo-2, hi+1)
    const int n_bins = W + 2 + 64;
    uint64_t *hist = smem;
    float *thr_s = reinterpret_cast<float *>(smem + BW * n_bins);
    constexpr bool kThr = LM == LM_AFFINE || LM == LM_SEARCH;
    if (kThr)
        for (int i = tid; i < W + 3; i += 256) {
            int k = lo - 2 + i;
            k = k < 0 ? 0 : (k >= L ? L - 1 : k);
            thr_s[i] = lv.thr[k];
        }
#pragma unroll
    for (int k = 0; k < BW; ++k) dl[256 * k + tid] = delta_lut[256 * k + tid];
    for (int b = tid; b < BW * n_bins; b += 256) hist[b] = 0;
    __syncthreads();

    const int G = gridDim.x;
    const int wg = xcd_order(blockIdx.x, G);
    const int64_t gw = (int64_t)wg * kWavesPerWG + wave, NW = (int64_t)G * kWavesPerWG;
    const int64_t H = row_hi - row_lo;
    const int64_t n_strips = (w + CE - 1) / CE;
    const int64_t units = n_strips * H;
    const int64_t u_end = units * (gw + 1) / NW;
    // lanes 0 and 63 only serve as halo: their window is empty
    const uint32_t wl = lane == 0 || lane == 63 ? 0u : (uint32_t)W;
    const ThrLds thr{thr_s, lo - 2};
    for (int64_t u = units * gw / NW; u < u_end;) {
        const int64_t strip = u / H, ra = u % H;
        const int64_t rb = ra + (u_end - u) < H ? ra + (u_end - u) : H;
        stream_run_2d<T, LM, AL, PF, CLS>(data, (int)h, w, lv, thr, lo, W, cpass, dl, hist, strip,
                                          (int)(row_lo + ra), (int)(row_lo + rb), lane, wl, (uint32_t)(W + 2 + lane));
        u += rb - ra;
    }
    __syncthreads();
    if constexpr (CLS)
        drain_cls(hist + 2, W, lo, L, G, wg, partial, accumulate == 0);
    else
        drain_2d(hist + 1, W, lo, L, G, wg, partial, accumulate == 0);
}

// ---------------------------------------------------------------------------
// 2D batched: many fields in one persistent launch
// ---------------------------------------------------------------------------
// The host cuts every field into items of (strip, row) units and assigns
// items to workgroups.  A workgroup runs its items one after another with the
// single-field machinery (its four waves split an item's units), draining its
// LDS bins into the field's global per-level histogram after each item.  The
// workgroup that finishes a field's last item (a ticket counter per field)
// scans that histogram into the field's curves and clears it, so one launch
// covers every field with no second pass.
template <typename T, int LM>
__global__ void __launch_bounds__(256)
    ecc2d_batch(const BatchField2D *__restrict__ fields, const BatchItem *__restrict__ items,
                const int32_t *__restrict__ wg_first, const uint64_t *__restrict__ luts) {
    constexpr int PF = sizeof(T) == 1 ? 3 : 6;
    constexpr bool kThr = LM == LM_AFFINE || LM == LM_SEARCH;
    extern __shared__ uint64_t smem[];
    __shared__ uint64_t dl[2][256];
    __shared__ int64_t part[256];
    __shared__ int last;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    dl[0][tid] = luts[tid];
    dl[1][tid] = luts[256 + tid];
    const int i_beg = wg_first[blockIdx.x], i_end = wg_first[blockIdx.x + 1];
    const bool halo_lane = lane == 0 || lane == 63;
    for (int it = i_beg; it < i_end; ++it) {
        const BatchItem item = items[it];
        const BatchField2D &f = fields[item.field];
        const int L = f.L;
        const int h = (int)f.h;
        const int64_t w = f.w;
        uint64_t *hist = smem;  // bins 0..L+1, then a scratch bin per lane
        float *thr_s = reinterpret_cast<float *>(smem + L + 2 + 64);
        for (int b = tid; b < L + 2; b += 256) hist[b] = 0;
        if (kThr)
            for (int i = tid; i < L + 3; i += 256) {
                int k = i - 2;
                k = k < 0 ? 0 : (k >= L ? L - 1 : k);
                thr_s[i] = f.thr[k];
            }
        __syncthreads();
        LevelArgs lv;
        lv.L = L;
        lv.mode = LM;
        lv.thr = f.thr;
        lv.lut = f.lut;
        lv.u0 = 0.f;
        lv.inv_step = f.inv_step;
        lv.u0d = 0.0;
        lv.eps = f.eps;
        const ThrLds thr{thr_s, -2};
        const int n = item.u1 - item.u0;
        const int u_end = item.u0 + (int)((int64_t)n * (wave + 1) / kWavesPerWG);
        for (int u = item.u0 + (int)((int64_t)n * wave / kWavesPerWG); u < u_end;) {
            const int strip = u / h, ra = u % h;
            const int rb = ra + (u_end - u) < h ? ra + (u_end - u) : h;
            stream_run_2d<T, LM, kLoadVector, PF, false>((const T *)f.data, h, w, lv, thr, 0, L, f.cpass, dl[f.conn_idx],
                                                  hist, strip, ra, rb, lane, halo_lane ? 0u : (uint32_t)L,
                                                  (uint32_t)(L + 2 + lane));
            u += rb - ra;
        }
        __syncthreads();
        // bins -> the field's global histogram (levels hist[1..L])
        for (int b = tid + 1; b <= L; b += 256) {
            const uint64_t v = hist[b];
            if (v == 0) continue;
            const int64_t cnt = (int64_t)(v >> kShiftCnt2);
            const int64_t per = (int64_t)((v >> kShiftPer2) & ((1ull << (kShiftCnt2 - kShiftPer2)) - 1)) -
                                kPerBias2 * cnt;
            const int64_t ec = (int64_t)(v & ((1ull << kShiftPer2) - 1)) - kEcBias2 * cnt;
            int32_t *dst = f.hist + (b - 1);
            if (ec) atomicAdd(dst, (int32_t)ec);
            if (per) atomicAdd(dst + L, (int32_t)per);
            atomicAdd(dst + 2 * L, (int32_t)cnt);
        }
        // publish (every thread's atomics), take the field's ticket
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid == 0)
            last = __hip_atomic_fetch_add(f.done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) ==
                   (uint32_t)(f.n_items - 1);
        __syncthreads();
        if (last) {  // uniform: scan the field's histogram into its curves and clear it
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const int per = (L + 255) / 256;
            const int beg = tid * per, end = beg + per < L ? beg + per : L;
            for (int ch = 0; ch < 3; ++ch) {
                int32_t *src = f.hist + (int64_t)ch * L;
                int64_t *dst = f.out[ch];
                int64_t s = 0;
                for (int i = beg; i < end; ++i) s += src[i];
                part[tid] = s;
                __syncthreads();
                for (int off = 1; off < 256; off <<= 1) {  // inclusive scan of the chunk sums
                    const int64_t v = tid >= off ? part[tid - off] : 0;
                    __syncthreads();
                    part[tid] += v;
                    __syncthreads();
                }
                int64_t run = part[tid] - s;
                for (int i = beg; i < end; ++i) {
                    run += src[i];
                    src[i] = 0;
                    if (dst) dst[i] = run;
                }
                __syncthreads();
            }
            if (tid == 0) *f.done = 0u;
        }
    }
}

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
__device__ __forceinline__ uint32_t elem_bits(const T *p) {
    if constexpr (sizeof(T) == 4)
        return __float_as_uint(*p);
    else
        return (uint32_t)*p;
}

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

template <typename T, int LM, typename TH>
__device__ __forceinline__ uint32_t level3(uint32_t bits, const LevelArgs &lv, const TH &thr, int lo, int W,
                                           float cpass) {
    const int base = lo - 1;
    const uint32_t never = (uint32_t)(W + 1);
    if constexpr (LM == LM_AFFINE) {
        const float x = __uint_as_float(bits);
        const float y = __builtin_fmaf(x, lv.inv_step, cpass);
        const float m = y + kMagic;
        const float r = y - (m - kMagic);
        // clamped estimate of lam' (at least 1 in the first pass: values at
        // or below t0 have level 0)
        const float mlo = lo == 0 ? kMagic + 1.0f : kMagic;
        uint32_t l = __float_as_uint(__builtin_amdgcn_fmed3f(m, mlo, kMagic + (float)never)) - kMagicBits;
        if (!(__builtin_fabsf(r) <= 0.5f - lv.eps)) {  // near a threshold (or NaN / inf)
            const int k = (int)l;
            if (k >= 0 && k <= W + 1) {
                const int g0 = k + base < 0 ? 0 : k + base;
                const int g = (int)level_settle(x, (uint32_t)g0, lv.L, thr);
                l = (uint32_t)min(max(g - base, 0), (int)never);
            }
        }
        return l;
    } else if constexpr (LM == LM_SEARCH) {
        return level_search_window(__uint_as_float(bits), lo, lo + W, thr);
    } else {
        const int l = (int)level_of<T, LM>(as_value<T>(bits), lv, thr);
        return (uint32_t)min(max(l - base, 0), (int)never);
    }
}

// packed level pairs of one row (P[i] = (lam'[i-1], lam'[i]) with the strip
// neighbours at both ends); rows outside the field are "never"
template <typename T, int LM, typename TH>
__device__ __forceinline__ void convert_row3(const RawRow3 &raw_in, bool row_ok, int64_t w, int64_t xs, int64_t x0,
                                             int lane, const LevelArgs &lv, const TH &thr, int lo, int W,
                                             float cpass, uint32_t (&P)[Elem3<T>::VEC + 1]) {
    constexpr int VEC = Elem3<T>::VEC;
    const uint32_t never = (uint32_t)(W + 1);
    if (!row_ok) {  // uniform
#pragma unroll
        for (int i = 0; i <= VEC; ++i) P[i] = never | never << 16;
        return;
    }
    RawRow3 raw = raw_in;
    if (__any(raw.shift != 0)) unshift_row3<T>(raw);  // rare: blocks at the end of the buffer
    if constexpr (LM == LM_IDENTITY) {  // integer values, two per packed operation
        const uint32_t lo2 = (uint32_t)lo * 0x10001u, nv2 = never * 0x10001u;
        uint32_t Q0 = identity_pair(raw_pair<T>(raw.w, 0), lo2, nv2);
        uint32_t Q1 = identity_pair(raw_pair<T>(raw.w, 2), lo2, nv2);
        if (!(xs + 64 * VEC <= w)) {  // uniform: cells outside the field never enter
            const uint32_t m0 = (x0 < w ? 0u : 0xFFFFu) | (x0 + 1 < w ? 0u : 0xFFFF0000u);
            const uint32_t m1 = (x0 + 2 < w ? 0u : 0xFFFFu) | (x0 + 3 < w ? 0u : 0xFFFF0000u);
            Q0 = (Q0 & ~m0) | (nv2 & m0);
            Q1 = (Q1 & ~m1) | (nv2 & m1);
        }
        const uint32_t hl = level3<T, LM>(raw.halo, lv, thr, lo, W, cpass);
        uint32_t lq = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)Q1, 0x138, 0xf, 0xf, false);
        uint32_t rq = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)Q0, 0x130, 0xf, 0xf, false);
        if (lane == 0) lq = (xs > 0 ? hl : never) << 16;
        if (lane == 63) rq = xs + 64 * VEC < w ? hl : never;
        P[0] = straddle(lq, Q0);
        P[1] = Q0;
        P[2] = straddle(Q0, Q1);
        P[3] = Q1;
        P[4] = straddle(Q1, rq);
        return;
    }
    uint32_t lam[VEC];
#pragma unroll
    for (int i = 0; i < VEC; ++i)
        lam[i] = x0 + i < w ? level3<T, LM>(elem3<T>(raw, i), lv, thr, lo, W, cpass) : never;
    const uint32_t hl = level3<T, LM>(raw.halo, lv, thr, lo, W, cpass);
    uint32_t left = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)lam[VEC - 1], 0x138, 0xf, 0xf, false);
    uint32_t right = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)lam[0], 0x130, 0xf, 0xf, false);
    if (lane == 0) left = xs > 0 ? hl : never;
    if (lane == 63) right = xs + 64 * VEC < w ? hl : never;
    P[0] = pack_lo16(left, lam[0]);
#pragma unroll
    for (int i = 1; i < VEC; ++i) P[i] = pack_lo16(lam[i - 1], lam[i]);
    P[VEC] = pack_lo16(lam[VEC - 1], right);
}

// 8-neighbour "entered before" pattern of the two cells of pair j (low / high
// half), rows u (above), m (current), d (below), as offsets into tables of
// 4-byte entries (lut_lo / lut_hi)
template <int VEC>
__device__ __forceinline__ uint32_t pattern_pair(const uint32_t (&u)[VEC + 1], const uint32_t (&m)[VEC + 1],
                                                 const uint32_t (&d)[VEC + 1], int j) {
    const uint32_t self = m[j], self1 = self + 0x00010001u;
    return gather_offsets<2>(pk_diff(u[j - 1], self1), pk_diff(u[j], self1), pk_diff(u[j + 1], self1),
                             pk_diff(m[j - 1], self1), pk_diff(m[j + 1], self), pk_diff(d[j - 1], self),
                             pk_diff(d[j], self), pk_diff(d[j + 1], self));
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
//          word of a 3D bin: (+-EC of the 2D cell) + 7 + (perimeter + 8) << 22
//   tm[p]: 2D EC delta of an image pixel with pattern p, sign included
// A voxel's low word is tl[p_layer] + (its share of the two images' deltas)
// - 2 * (vertical neighbours that entered before it) << 22.
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
    const int32_t *tm;
    uint64_t *hist;
    int64_t xs, x0;
    int y0, zb, lane;
    int64_t last_block;
    uint32_t scratch;  // this lane's scratch bin, W + 2 + lane
    const uint32_t *tc;  // CR: per-plane crease deltas + 4
    uint32_t *hc;        // CR: crease words of the bins

    uint32_t R[3][NR][VEC + 1];  // level planes; R[(z - za + 1) % 3] holds plane z
    int32_t E[TY][VEC];          // image delta of the pixel below each voxel of the current plane
    RawRow3 ring[3][NR];         // raw rows of upcoming planes; ring[(z - za) % 3] holds plane z + 1

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
            convert_row3<T, LM>(src[r], row_ok(z, y0 - 1 + r), w, xs, x0, lane, lv, thr, lo, W, cpass, dst[r]);
    }
    __device__ __forceinline__ void image(const uint32_t (&a)[NR][VEC + 1], const uint32_t (&b)[NR][VEC + 1],
                                          uint32_t (&m)[NR][VEC + 1]) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int i = 0; i <= VEC; ++i) m[r][i] = pk_merge<MAXIMG>(a[r][i], b[r][i]);
    }

    // planes za-1 and za converted, E of the image between them, planes
    // za+1 .. za+3 in flight
    __device__ __forceinline__ void prologue(int za) {
        {
            RawRow3 a[NR], b[NR];
            fetch_plane(za - 1, a);
            fetch_plane(za, b);
#pragma unroll
            for (int k = 0; k < 3; ++k) fetch_plane(za + 1 + k < zb ? za + 1 + k : zb, ring[k]);
            convert_plane(za - 1, a, R[0]);
            convert_plane(za, b, R[1]);
        }
        uint32_t M[NR][VEC + 1];
        image(R[0], R[1], M);
#pragma unroll
        for (int t = 0; t < TY; ++t)
#pragma unroll
            for (int j = 1; j < VEC + 1; j += 2) {
                const uint32_t pm = pattern_pair<VEC>(M[t], M[t + 1], M[t + 2], j);
                E[t][j - 1] = lut_lo<int32_t, 2>(tm, pm);
                E[t][j] = lut_hi<int32_t, 2>(tm, pm);
            }
    }

    // voxels of plane z, with K = (z - za) % 3
    template <int K>
    __device__ __forceinline__ void step(int z) {
        uint32_t(&Pp)[NR][VEC + 1] = R[K];
        uint32_t(&Pc)[NR][VEC + 1] = R[(K + 1) % 3];
        uint32_t(&Pn)[NR][VEC + 1] = R[(K + 2) % 3];
        convert_plane(z + 1, ring[K], Pn);
        fetch_plane(z + 4 < zb ? z + 4 : zb, ring[K]);
        uint32_t M[NR][VEC + 1];
        image(Pc, Pn, M);
#pragma unroll
        for (int t = 0; t < TY; ++t) {
            // table reads of the row's VEC voxels first, then their atomics
            uint32_t tlv[VEC], pm[VEC / 2], selfv[VEC / 2], below[VEC / 2], above[VEC / 2];
            uint32_t crv[CR ? VEC : 1];
            int32_t en[VEC];
#pragma unroll
            for (int q = 0; q < VEC / 2; ++q) {
                const int j = 2 * q + 1;
                const uint32_t self = Pc[t + 1][j], self1 = self + 0x00010001u;
                const uint32_t pl = pattern_pair<VEC>(Pc[t], Pc[t + 1], Pc[t + 2], j);
                pm[q] = pattern_pair<VEC>(M[t], M[t + 1], M[t + 2], j);
                // vertical neighbours: the one below (z-1) precedes on ties,
                // the one above (z+1) does not
                below[q] = pk_lt(Pp[t + 1][j], self1);
                above[q] = pk_lt(Pn[t + 1][j], self);
                selfv[q] = self;
                tlv[2 * q] = lut_lo<uint32_t, 2>(tl, pl);
                tlv[2 * q + 1] = lut_hi<uint32_t, 2>(tl, pl);
                en[2 * q] = lut_lo<int32_t, 2>(tm, pm[q]);
                en[2 * q + 1] = lut_hi<int32_t, 2>(tm, pm[q]);
                if constexpr (CR) {
                    // yz plane through the voxel's column, xz plane through its row
                    const uint32_t pyz = plane_pattern(Pp[t][j], Pp[t + 1][j], Pp[t + 2][j], Pc[t][j], Pc[t + 2][j],
                                                       Pn[t][j], Pn[t + 1][j], Pn[t + 2][j], self);
                    const uint32_t pxz = plane_pattern(Pp[t + 1][j - 1], Pp[t + 1][j], Pp[t + 1][j + 1],
                                                       Pc[t + 1][j - 1], Pc[t + 1][j + 1], Pn[t + 1][j - 1],
                                                       Pn[t + 1][j], Pn[t + 1][j + 1], self);
                    crv[2 * q] = lut_lo<uint32_t, 2>(tc, pl) + lut_lo<uint32_t, 2>(tc, pyz) +
                                 lut_lo<uint32_t, 2>(tc, pxz);
                    crv[2 * q + 1] = lut_hi<uint32_t, 2>(tc, pl) + lut_hi<uint32_t, 2>(tc, pyz) +
                                     lut_hi<uint32_t, 2>(tc, pxz);
                }
            }
#pragma unroll
            for (int q = 0; q < VEC / 2; ++q) {
                const int j = 2 * q + 1;
                // an image pixel's event goes to the voxel of its pair that
                // enters first (min image) or last (max image)
                const uint32_t tb = MAXIMG ? below[q] : below[q] ^ 0x00010001u;
                const uint32_t ta = MAXIMG ? above[q] : above[q] ^ 0x00010001u;
                const uint32_t nb = below[q] + above[q];  // per half: vertical neighbours already in
                const uint32_t lo0 = tlv[2 * q] + (uint32_t)((tb & 1u) ? E[t][j - 1] : 0) +
                                     (uint32_t)((ta & 1u) ? en[2 * q] : 0) - ((nb & 0xFFFFu) << 23);
                const uint32_t lo1 = tlv[2 * q + 1] + (uint32_t)((tb >> 16) ? E[t][j] : 0) +
                                     (uint32_t)((ta >> 16) ? en[2 * q + 1] : 0) - ((nb >> 16) << 23);
                E[t][j - 1] = en[2 * q];
                E[t][j] = en[2 * q + 1];
                const uint32_t self = selfv[q];
                // bins lam' (1..W); a voxel outside the window or the field goes
                // to its lane's own scratch bin (never drained) rather than
                // branching: one address per lane keeps such voxels apart
                uint32_t b0 = self & 0xFFFFu, b1 = self >> 16;
                b0 = b0 - 1u < (uint32_t)W ? b0 : scratch;
                b1 = b1 - 1u < (uint32_t)W ? b1 : scratch;
                constexpr uint64_t cnt = 1ull << kShiftCnt3;
                atomicAdd((unsigned long long *)&hist[b0], (unsigned long long)(cnt | lo0));
                atomicAdd((unsigned long long *)&hist[b1], (unsigned long long)(cnt | lo1));
                if constexpr (CR) {
                    atomicAdd(&hc[b0], crv[2 * q]);
                    atomicAdd(&hc[b1], crv[2 * q + 1]);
                }
            }
        }
    }

    __device__ __forceinline__ void run(int za) {
        prologue(za);
        int z = za;
        for (; z + 3 <= zb; z += 3) {
            step<0>(z);
            step<1>(z + 1);
            step<2>(z + 2);
        }
        if (z < zb) step<0>(z);
        if (z + 1 < zb) step<1>(z + 1);
    }
};

// Work split: units (column, z) with column = (strip, block of TY rows), z
// fastest, in equal contiguous ranges per wave.
template <typename T, int LM, int AL, bool MAXIMG, bool CR, int TY>
__global__ void __launch_bounds__(256)
    ecc3d_stream(const T *__restrict__ data, int64_t d, int64_t h, int64_t w, LevelArgs lv, int32_t lo,
                 int32_t hi, float cpass, const uint32_t *__restrict__ tables,
                 const uint32_t *__restrict__ crease_table, int32_t *__restrict__ partial, int64_t z_lo,
                 int64_t z_hi, int accumulate) {
    constexpr int VEC = Elem3<T>::VEC;
    extern __shared__ uint64_t smem[];
    __shared__ uint32_t tl[256];
    __shared__ int32_t tm[256];
    __shared__ uint32_t tc[CR ? 256 : 1];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int W = hi - lo;
    const int L = lv.L;
    const int n_bins = W + 2 + 64;  // 1..W are the window's levels, then a scratch bin per lane
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
    tm[tid] = (int32_t)tables[256 + tid];
    if constexpr (CR) tc[tid] = crease_table[tid];
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
    for (int64_t u = units * gw / NW; u < u_end;) {
        const int64_t col = u / D, za = u % D;
        const int64_t zb = za + (u_end - u) < D ? za + (u_end - u) : D;
        const int64_t strip = col % n_strips, yb = col / n_strips;
        const int64_t xs = strip * 64 * VEC;
        March3D<T, LM, AL, MAXIMG, CR, TY, ThrLds> m{data, (int)d, h, w, lv, thr, lo, W, cpass, tl, tm,
                                                      hist, xs, xs + (int64_t)lane * VEC, (int)(yb * TY),
                                                      (int)(z_lo + zb), lane, d * h * w > VEC ? d * h * w - VEC : 0,
                                                      (uint32_t)(W + 2 + lane), tc, hc};
        m.run((int)(z_lo + za));
        u += zb - za;
    }
    __syncthreads();
    drain_3d(hist + 1, CR ? hc + 1 : nullptr, CR, W, lo, L, G, wg, partial, accumulate == 0);
}


// 3D class-count bins [level][class] (int32) -> partials [class][level][workgroup]
__device__ __forceinline__ void drain_cls3(int32_t *hcls, int W, int lo, int L, int G, int wg,
                                           int32_t *__restrict__ partial, bool first) {
    for (int i = threadIdx.x; i < W * kNumClasses3D; i += blockDim.x) {
        const int b = i / kNumClasses3D, c = i - b * kNumClasses3D;
        const int32_t v = hcls[i];
        hcls[i] = 0;
        const int64_t idx = ((int64_t)c * L + lo + b) * G + wg;
        if (first)
            partial[idx] = v;
        else
            partial[idx] += v;
    }
}

// ---------------------------------------------------------------------------
// 3D (generic: every channel, table lookups over the 8 corner blocks)
// ---------------------------------------------------------------------------
// MODE 0: EC, surface, volume; 1: also the crease; 2: vertex class counts
// (vtab then holds the class of each octant mask, -1 for empty, and each
// corner adds +1 to its new class and -1 to its old one in the cell's bin).
template <typename T, int LM, int MODE>
__global__ void __launch_bounds__(256)
    ecc3d_tile(const T *__restrict__ data, int64_t d, int64_t h, int64_t w, LevelArgs lv,
               int32_t lo, int32_t hi, const int64_t *__restrict__ vtab,
               int32_t *__restrict__ partial, int64_t tiles_x, int64_t tiles_y, int64_t n_tiles,
               int flush_tiles) {
    constexpr bool CREASE = MODE == 1;
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
    int32_t *hcls = reinterpret_cast<int32_t *>(smem);  // MODE 2: [W][kNumClasses3D]
    const int G = gridDim.x;
    const int wg = xcd_order(blockIdx.x, G);
    const int64_t t_beg = n_tiles * wg / G, t_end = n_tiles * (wg + 1) / G;

    vt[t] = vtab[t];
    if constexpr (MODE == 2) {
        for (int b = t; b < W * kNumClasses3D; b += 256) hcls[b] = 0;
    } else {
        for (int b = t; b < W; b += 256) {
            hist[b] = 0;
            if (CREASE) hc[b] = 0;
        }
    }
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
                if constexpr (MODE == 2) {
                    int32_t *row = hcls + (p - lo) * kNumClasses3D;
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const int cx = c & 1, cy = c >> 1 & 1, cz = c >> 2;
                        const uint32_t y = P >> (cz * 9 + cy * 3 + cx);
                        const uint32_t m1 = (y & 3u) | ((y >> 1) & 0xCu) | ((y >> 5) & 0x30u) | ((y >> 6) & 0xC0u);
                        const uint32_t m0 = m1 & ~(1u << (7 - c));
                        const int cn = (int)vt[m1], co = (int)vt[m0];
                        atomicAdd(&row[cn], 1);
                        if (co >= 0) atomicAdd(&row[co], -1);
                    }
                    continue;
                }
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
            if constexpr (MODE == 2)
                drain_cls3(hcls, W, lo, L, G, wg, partial, first);
            else
                drain_3d(hist, hc, CREASE, W, lo, L, G, wg, partial, first);
            first = false;
            since = 0;
            __syncthreads();
        }
    }
    if constexpr (MODE == 2)
        drain_cls3(hcls, W, lo, L, G, wg, partial, first);
    else
        drain_3d(hist, hc, CREASE, W, lo, L, G, wg, partial, first);
}

// ---------------------------------------------------------------------------
// merge of per-workgroup partials and prefix scan over levels
// ---------------------------------------------------------------------------
struct OutPtrs {
    int64_t *p[4];
};

// One wave per (channel, level) sums the G workgroup partials of that bin
// (coalesced reads, shuffle reduction).  The block that finishes last (ticket
// on a counter that it then resets) takes the running sum over levels of
// every requested channel and writes the caller's int64 curves.
__global__ void __launch_bounds__(1024)
    ecc_merge(const int32_t *__restrict__ partial, int G, int nch, int L, OutPtrs out,
              int64_t *__restrict__ totals, unsigned *__restrict__ counter) {
    __shared__ bool last;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int waves = blockDim.x >> 6;
    const int64_t n_bins = (int64_t)nch * L;
    for (int64_t bin = (int64_t)blockIdx.x * waves + wave; bin < n_bins; bin += (int64_t)gridDim.x * waves) {
        const int ch = (int)(bin / L);
        if (!out.p[ch]) continue;
        const int32_t *src = partial + bin * G;
        int64_t s = 0;
        if ((G & 3) == 0) {  // 16-byte loads, several in flight per lane
            const u32x4 *s4 = reinterpret_cast<const u32x4 *>(src);
            const int G4 = G >> 2;
#pragma unroll 4
            for (int g = lane; g < G4; g += 64) {
                const u32x4 v = __builtin_nontemporal_load(s4 + g);
                s += (int64_t)(int32_t)v.x + (int32_t)v.y + (int32_t)v.z + (int32_t)v.w;
            }
        } else {
            for (int g = lane; g < G; g += 64) s += src[g];
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) totals[bin] = s;
    }
    // publish this block's totals (release), take a ticket; the last block
    // acquires everything the others published
    __syncthreads();
    if (threadIdx.x == 0)
        last = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
    __syncthreads();
    if (!last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    // running sums over levels, all channels at once (independent loads and
    // shuffle chains overlap): each thread sums a chunk of levels, the chunk
    // sums are scanned within waves by shuffles, then over the wave totals
    const int t = threadIdx.x, nt = blockDim.x;
    const int per = (L + nt - 1) / nt;
    const int beg = t * per, end = beg + per < L ? beg + per : L;
    int64_t sum[4] = {0, 0, 0, 0}, x[4];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch)
        if (ch < nch && out.p[ch])
            for (int i = beg; i < end; ++i) sum[ch] += totals[(int64_t)ch * L + i];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) x[ch] = sum[ch];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            const int64_t y = __shfl_up(x[ch], off);
            if (lane >= off) x[ch] += y;
        }
    }
    __shared__ int64_t wtot[4][16];
    if (lane == 63)
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) wtot[ch][wave] = x[ch];
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) {
            int64_t v = lane < waves ? wtot[ch][lane] : 0;
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) {
                const int64_t y = __shfl_up(v, off);
                if (lane >= off) v += y;
            }
            if (lane < waves) wtot[ch][lane] = v;
        }
    }
    __syncthreads();
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
        int64_t *dst = ch < nch ? out.p[ch] : nullptr;
        if (!dst) continue;  // uniform
        int64_t run = (wave > 0 ? wtot[ch][wave - 1] : 0) + x[ch] - sum[ch];
        for (int i = beg; i < end; ++i) {
            run += totals[(int64_t)ch * L + i];
            dst[i] = run;
        }
    }
    if (threadIdx.x == 0) *counter = 0u;  // ready for the next merge
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
size_t lds_bytes_3d(int window, bool want_crease) { return (size_t)window * (want_crease ? 12 : 8); }

int load_mode_2d(const void *data, int64_t h, int64_t w, int elem_bytes) {
    (void)h;
    return ((uintptr_t)data % 16 == 0 && (w * elem_bytes) % 16 == 0) ? kLoadAligned : kLoadVector;
}

// cells one workgroup may add to its LDS bins in a launch of `rows` rows
static int64_t max_wg_cells_2d(int64_t rows, int64_t w, int vec, int grid) {
    const int64_t ce = 62 * vec;
    const int64_t units = ((w + ce - 1) / ce) * rows;
    const int64_t NW = (int64_t)grid * kWavesPerWG;
    return kWavesPerWG * ((units + NW - 1) / NW + 1) * ce;
}

template <typename T, int LM, int AL, bool CLS>
static int launch_2d_t(const Launch2D &a, hipStream_t s) {
    constexpr int VEC = Elem<T>::VEC, PF = sizeof(T) == 1 ? 3 : 6;
    const int W = a.hi - a.lo;
    // the packed LDS bins of one workgroup may see at most kFlush2D (class
    // counts: kFlushCls) cells: split tall fields into row chunks that respect
    // it (later chunks add to the partials of the first)
    const int64_t flush = CLS ? kFlushCls : kFlush2D;
    int64_t chunk = a.row_hi - a.row_lo;
    while (chunk > 1 && max_wg_cells_2d(chunk, a.w, VEC, a.grid) > flush) chunk = (chunk + 1) / 2;
    if (max_wg_cells_2d(chunk, a.w, VEC, a.grid) > flush) return (int)hipErrorInvalidValue;
    // affine levels: the pass constant -t0/step + 1.5 - lo, rounded once
    const float cpass = (float)(a.lv.u0d + 1.5 - a.lo);
    const size_t lds = (size_t)(CLS ? 2 : 1) * (W + 2 + 64) * 8 + (size_t)(W + 3) * 4;
    for (int64_t r0 = a.row_lo; r0 < a.row_hi; r0 += chunk) {
        const int64_t r1 = r0 + chunk < a.row_hi ? r0 + chunk : a.row_hi;
        const bool acc = a.accumulate || r0 > a.row_lo;
        hipLaunchKernelGGL((ecc2d_stream<T, LM, AL, PF, CLS>), dim3(a.grid), dim3(256), lds, s,
                           (const T *)a.data, a.h, a.w, a.lv, a.lo, a.hi, cpass, a.delta_lut, a.partial, r0, r1,
                           acc ? 1 : 0);
        const int e = (int)hipGetLastError();
        if (e) return e;
    }
    return 0;
}

template <typename T, int LM>
static int launch_2d_al(const Launch2D &a, hipStream_t s) {
    // class counts load at any alignment (one variant per dtype and level mode)
    if (a.classes) return launch_2d_t<T, LM, kLoadVector, true>(a, s);
    return load_mode_2d(a.data, a.h, a.w, (int)sizeof(T)) == kLoadAligned
               ? launch_2d_t<T, LM, kLoadAligned, false>(a, s)
               : launch_2d_t<T, LM, kLoadVector, false>(a, s);
}

template <typename T>
static int launch_2d_dt(const Launch2D &a, hipStream_t s) {
    // integer fields have identity levels or a value -> level table; float
    // fields always have thresholds (affine or searched)
    if constexpr (sizeof(T) < 4)
        return a.lv.mode == LM_LUT ? launch_2d_al<T, LM_LUT>(a, s) : launch_2d_al<T, LM_IDENTITY>(a, s);
    else
        return a.lv.mode == LM_AFFINE ? launch_2d_al<T, LM_AFFINE>(a, s) : launch_2d_al<T, LM_SEARCH>(a, s);
}

int launch_2d(const Launch2D &a, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    switch (a.dtype) {
    case ECC_U8: return launch_2d_dt<uint8_t>(a, s);
    case ECC_U16: return launch_2d_dt<uint16_t>(a, s);
    default: return launch_2d_dt<float>(a, s);
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
    const size_t lds = MODE == 2 ? (size_t)W * kNumClasses3D * 4 : lds_bytes_3d(W, MODE == 1);
    hipLaunchKernelGGL((ecc3d_tile<T, LM, MODE>), dim3(a.grid), dim3(256), lds, s,
                       (const T *)a.data, a.d, a.h, a.w, a.lv, a.lo, a.hi, a.vtab, a.partial,
                       tiles_x, tiles_y, n_tiles, flush);
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
    const float cpass = (float)(a.lv.u0d + 1.5 - a.lo);
    const size_t lds = (size_t)(W + 2 + 64) * (CR ? 12 : 8) + (kThr ? (size_t)(W + 3) * 4 : 0);
    for (int64_t z0 = a.z_lo; z0 < a.z_hi; z0 += chunk) {
        const int64_t z1 = z0 + chunk < a.z_hi ? z0 + chunk : a.z_hi;
        const bool acc = a.accumulate || z0 > a.z_lo;
        hipLaunchKernelGGL((ecc3d_stream<T, LM, AL, MAXIMG, CR, kZmTY>), dim3(a.grid), dim3(256), lds, s,
                           (const T *)a.data, a.d, a.h, a.w, a.lv, a.lo, a.hi, cpass, a.zm_tables, a.crease_table,
                           a.partial, z0, z1, acc ? 1 : 0);
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
    if (a.classes) return launch_3d_t<T, LM, 2>(a, s);
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

size_t lds_bytes_batch_2d(int lm, int max_L) {
    const bool thr = lm == LM_AFFINE || lm == LM_SEARCH;
    return (size_t)(max_L + 2 + 64) * 8 + (thr ? (size_t)(max_L + 3) * 4 : 0);
}

template <typename T>
static int launch_batch_t(int lm, const BatchField2D *fields, const BatchItem *items, const int32_t *wg_first,
                          int grid, const uint64_t *luts, size_t lds, hipStream_t s) {
    if constexpr (sizeof(T) < 4) {
        if (lm == LM_LUT)
            hipLaunchKernelGGL((ecc2d_batch<T, LM_LUT>), dim3(grid), dim3(256), lds, s, fields, items, wg_first, luts);
        else
            hipLaunchKernelGGL((ecc2d_batch<T, LM_IDENTITY>), dim3(grid), dim3(256), lds, s, fields, items, wg_first,
                               luts);
    } else {
        if (lm == LM_AFFINE)
            hipLaunchKernelGGL((ecc2d_batch<T, LM_AFFINE>), dim3(grid), dim3(256), lds, s, fields, items, wg_first,
                               luts);
        else
            hipLaunchKernelGGL((ecc2d_batch<T, LM_SEARCH>), dim3(grid), dim3(256), lds, s, fields, items, wg_first,
                               luts);
    }
    return (int)hipGetLastError();
}

int launch_batch_2d(int dtype, int lm, const BatchField2D *fields, const BatchItem *items,
                    const int32_t *wg_first, int grid, const uint64_t *luts, int max_L, void *stream) {
    const size_t lds = lds_bytes_batch_2d(lm, max_L);
    hipStream_t s = (hipStream_t)stream;
    switch (dtype) {
    case ECC_U8: return launch_batch_t<uint8_t>(lm, fields, items, wg_first, grid, luts, lds, s);
    case ECC_U16: return launch_batch_t<uint16_t>(lm, fields, items, wg_first, grid, luts, lds, s);
    default: return launch_batch_t<float>(lm, fields, items, wg_first, grid, luts, lds, s);
    }
}

int launch_merge(const int32_t *partial, int grid, int nch, int L, int64_t *const out[4],
                 int64_t *totals, unsigned *counter, void *stream) {
    OutPtrs o;
    for (int c = 0; c < 4; ++c) o.p[c] = c < nch ? out[c] : nullptr;
    const int64_t bins = (int64_t)nch * L;
    static const int max_blocks = [] {
        const char *e = std::getenv("ECC_MERGE_BLOCKS");
        const int x = e ? std::atoi(e) : 256;
        return x < 1 ? 1 : (x > 4096 ? 4096 : x);
    }();
    const int blocks = (int)std::min<int64_t>(max_blocks, (bins + 15) / 16);
    hipLaunchKernelGGL(ecc_merge, dim3(blocks), dim3(1024), 0, (hipStream_t)stream, partial, grid, nch, L,
                       o, totals, counter);
    return (int)hipGetLastError();
}

int launch_level_lut(const float *thr, int L, int n_values, uint16_t *lut, void *stream) {
    hipLaunchKernelGGL(ecc_level_lut, dim3((n_values + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, thr, L, n_values, lut);
    return (int)hipGetLastError();
}

}  // namespace ecc
