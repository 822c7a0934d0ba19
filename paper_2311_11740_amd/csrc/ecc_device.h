// Device helpers shared by the field kernels of libecc (gfx950).
//
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
#pragma once

#include <hip/hip_ext.h>
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

// the value the thresholds are compared with: x, or -x for the superlevel
// filtration (neg = the sign bit)
__device__ __forceinline__ float cmp_value(float x, uint32_t neg) {
    return __uint_as_float(__float_as_uint(x) ^ neg);
}

template <int LM, typename TH>
__device__ __forceinline__ uint32_t level_of_float(float xin, const LevelArgs &a, const TH &thr) {
    const int L = a.L;
    if (!(xin == xin)) return (uint32_t)L;  // NaN never enters
    const float x = cmp_value(xin, a.neg);
    if constexpr (LM == LM_AFFINE) {
        const float u = __builtin_fmaf(xin, a.inv_step, a.u0);  // inv_step carries the sign
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

// the bits of one element (float bits, or the integer value)
template <typename T>
__device__ __forceinline__ uint32_t elem_bits(const T *p) {
    if constexpr (sizeof(T) == 4)
        return __float_as_uint(*p);
    else
        return (uint32_t)*p;
}

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
// would make it wait for all outstanding ones).  The loads carry the
// non-temporal hint: without it the line where two strips meet more often
// stays in L2 for the neighbour (an 8192^2 float field then reads 1.041x its
// bytes instead of 1.070x), but the kernel runs about 3 % longer.
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

// The value of the lane below (wave_shr:1) or above (wave_shl:1) this one;
// lanes at the ends of the wave get 0 (bound_ctrl), which callers never use.
__device__ __forceinline__ uint32_t from_lane_below(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x138, 0xf, 0xf, true);
}
__device__ __forceinline__ uint32_t from_lane_above(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x130, 0xf, 0xf, true);
}

// Issue priority of a wave by how far it is through its share of the work:
// 3 in the first quarter down to 0 in the last.  Waves of equal work share a
// SIMD; with equal priorities the oldest issues first and the others finish
// later, one by one, leaving the SIMD with too few waves at the end.  Waves
// that are ahead step down, so the ones behind catch up.
struct ProgressPrio {
    int64_t q1 = 0, q2 = 0, q3 = 0;  // work done at the quarter marks
    int cur = 3;
    bool on = false;
    __device__ void init(bool enable, int64_t total) {
        on = enable;
        q1 = total / 4;
        q2 = total / 2;
        q3 = total - total / 4;
        cur = 3;
        if (on) __builtin_amdgcn_s_setprio(3);
    }
    __device__ __forceinline__ void update(int64_t done) {
        if (!on) return;
        const int p = done < q1 ? 3 : (done < q2 ? 2 : (done < q3 ? 1 : 0));
        if (p == cur) return;
        cur = p;
        if (p == 2)
            __builtin_amdgcn_s_setprio(2);
        else if (p == 1)
            __builtin_amdgcn_s_setprio(1);
        else
            __builtin_amdgcn_s_setprio(0);
    }
};

// (a.hi, b.lo): the 16-bit value just below b's low half
__device__ __forceinline__ uint32_t straddle(uint32_t a, uint32_t b) {
    return __builtin_amdgcn_alignbit(b, a, 16);
}



// ---------------------------------------------------------------------------
// bin indices and LDS addresses of the field kernels
// ---------------------------------------------------------------------------
// A pass histograms the levels [lo, lo + W) into bins kBinOff .. kBinOff + W - 1
// (level l -> bin l - lo + kBinOff; kBinOff in ecc_internal.h).  A cell whose
// level lies below the window takes its lane's own bin `lane` (< kBinOff), a
// cell above it or never entering the bin W + kBinOff + lane; neither range is drained, and the
// per-lane bins keep masses of such cells (the outside of the field, the
// levels of other passes) from piling onto one LDS address.  The bin index is
// also the rank the "entered before" relations compare: below-window values
// are smaller and above-window values larger than every in-window one, which
// is all those relations need for the in-window cells whose deltas count.

// Per-lane constants of the bin convention: a cell
// below the pass window ranks and is binned as `below` (= lane), a cell above
// it or never entering as `never` (= W + kBinOff + lane).
struct LaneBins {
    uint32_t below, never;
};

// level of x mapped to its bin index (kBinOff) by a binary search over the
// staged thresholds [lo - 1, hi)
template <typename TH>
__device__ __forceinline__ uint32_t bin_search(float x, int lo, int hi, const TH &thr, const LaneBins &lb) {
    if (lo > 0 && x <= thr[lo - 1]) return lb.below;
    if (!(x <= thr[hi - 1])) return lb.never;  // also NaN
    int a = lo, b = hi - 1;                    // x <= thr[b]
    while (a < b) {
        const int m = (a + b) >> 1;
        if (x <= thr[m])
            b = m;
        else
            a = m + 1;
    }
    return (uint32_t)(a - lo + kBinOff);
}

typedef __attribute__((address_space(3))) unsigned long long lds_u64;
typedef __attribute__((address_space(3))) unsigned int lds_u32;

// LDS byte address of a shared-memory pointer
__device__ __forceinline__ uint32_t lds_addr(const void *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}

// m * (x & 0xFFFF) + c and m * (x >> 16) + c in one operation each (m < 2^16):
// the LDS address of the bin of the low or high cell of a packed pair
__device__ __forceinline__ uint32_t mad_lo16(uint32_t x, uint32_t m, uint32_t c) {
    uint32_t r;
    asm("v_mad_u32_u16 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(m), "v"(c));
    return r;
}
__device__ __forceinline__ uint32_t mad_hi16(uint32_t x, uint32_t m, uint32_t c) {
    uint32_t r;
    asm("v_mad_u32_u16 %0, %1, %2, %3 op_sel:[1,0,0,0]" : "=v"(r) : "v"(x), "v"(m), "v"(c));
    return r;
}

__device__ __forceinline__ void lds_add64(uint32_t addr, uint64_t v) {
    __hip_atomic_fetch_add((lds_u64 *)(uintptr_t)addr, (unsigned long long)v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add32(uint32_t addr, uint32_t v) {
    __hip_atomic_fetch_add((lds_u32 *)(uintptr_t)addr, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ---------------------------------------------------------------------------
// merge of per-workgroup partials and prefix scan over levels
// ---------------------------------------------------------------------------
struct OutPtrs {
    int64_t *p[4];
};

// the sum of one bin's G workgroup partials (a whole wave; lane 0's result)
__device__ __forceinline__ int64_t sum_bin_wave(const int32_t *__restrict__ src, int G, int lane) {
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
    return s;
}

// Accumulators of the atomic drain (kAccCopies, ecc_internal.h): a workgroup
// adds into the copy of the XCD it runs on (its hardware XCC id), so that at
// most the workgroups of one XCD contend for an address.
__device__ __forceinline__ unsigned xcc_copy() {
    return __builtin_amdgcn_s_getreg(20 | (0 << 6) | ((4 - 1) << 11)) & (kAccCopies - 1);
}
__device__ __forceinline__ void acc_add(int64_t *p, int64_t v) {
    if (v) __hip_atomic_fetch_add((unsigned long long *)p, (unsigned long long)v, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
}

// Fields of a batched launch split over several workgroups: each workgroup
// adds its bins into the field's int32 histogram [nch][L] with device-scope
// atomics, then takes the field's ticket; the workgroup that takes the last
// one scans.  Those adds are atomics, performed where every XCD sees them, so
// a workgroup only waits until its own have completed before it takes the
// ticket (no L2 write-back, which per work item cost more than the item), and
// the elected workgroup reads and clears the histogram with device-scope
// exchanges, which see every completed add.
__device__ __forceinline__ bool take_field_ticket(uint32_t *done, int n_items) {
    __shared__ int s_last;
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);  // this thread's adds have completed
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __syncthreads();
    if (threadIdx.x == 0)
        s_last = __hip_atomic_fetch_add(done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                 (uint32_t)(n_items - 1);
    __syncthreads();
    return s_last != 0;
}

// The elected workgroup (256 threads): the field's histogram [nch][L] ->
// running sums over levels into out[ch] (NULL: skipped), histogram and ticket
// left at zero.  `stage` is LDS for L int64, `part` LDS for 256 int64.
__device__ __forceinline__ void scan_field_hist(int32_t *__restrict__ hist, int nch, int L, int64_t *const *out,
                                                int64_t *stage, int64_t *part, uint32_t *done) {
    const int tid = threadIdx.x;
    const int per = (L + 255) / 256;
    const int beg = tid * per < L ? tid * per : L, end = beg + per < L ? beg + per : L;
    for (int ch = 0; ch < nch; ++ch) {
        int *src = reinterpret_cast<int *>(hist) + (int64_t)ch * L;
        for (int l = tid; l < L; l += 256)
            stage[l] = __hip_atomic_exchange(src + l, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        int64_t *dst = out[ch];
        int64_t s = 0;
        for (int i = beg; i < end; ++i) s += stage[i];
        part[tid] = s;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {  // inclusive scan of the chunk sums
            const int64_t v = tid >= off ? part[tid - off] : 0;
            __syncthreads();
            part[tid] += v;
            __syncthreads();
        }
        int64_t run = part[tid] - s;
        if (dst)  // uniform
            for (int i = beg; i < end; ++i) {
                run += stage[i];
                dst[i] = run;
            }
        __syncthreads();  // stage and part are reused
    }
    if (tid == 0) __hip_atomic_store(done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Running sums over levels of the per-level totals [nch][L] into the caller's
// curves (channels with a NULL output skipped), by one whole workgroup of at
// most 16 waves: each thread sums a chunk of levels, the chunk sums are
// scanned within waves by shuffles, then over the wave totals.
__device__ __forceinline__ void scan_totals_block(const int64_t *__restrict__ totals, int nch, int L,
                                                  const OutPtrs &out) {
    __shared__ int64_t wtot[4][16];
    const int t = threadIdx.x, nt = blockDim.x;
    const int lane = t & 63, wave = t >> 6, waves = nt >> 6;
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
}

}  // namespace ecc
