// 2D kernels: the single-field row-streaming kernel (curves and vertex class
// counts) and the batched persistent kernel, with their launchers.
#include "ecc_device.h"
#include "ecc_levels.h"
#include "ecc_schedule.h"

namespace ecc {

// Bin indices of one row, packed as pairs P[i] = (bin[i-1], bin[i]) of the
// lane's cells with the neighbouring lanes' cells at both ends.
//
// Float fields with (nearly) evenly spaced thresholds: y = fma(x, 1/step, c)
// with c = -t0/step + kBinOff + 0.5 - lo estimates bin - 0.5; adding 1.5*2^23
// rounds y to an integer k in the low mantissa bits of m (exact for |y| <
// 2^22), and r = y - k is the rounding residual.  k is the bin unless |r| is
// within eps of 1/2, i.e. x sits within the host's error bound of a
// threshold; those cells are settled against the thresholds.
template <typename T, int LM, typename TH>
__device__ __forceinline__ void convert_row(const RawRow &raw_in, bool row_ok, bool full, const LevelArgs &lv,
                                            const TH &thr, int lo, int W, float cpass, const LaneBins &lb,
                                            uint32_t (&P)[Elem<T>::VEC + 1]) {
    constexpr int VEC = Elem<T>::VEC;
    const uint32_t never = lb.never;
    if (!row_ok) {  // uniform
#pragma unroll
        for (int i = 0; i <= VEC; ++i) P[i] = never | never << 16;
        return;
    }
    RawRow raw = raw_in;
    if (__any(raw.shift != 0)) unshift_row<T>(raw);  // rare: blocks at the end of the buffer
    if constexpr (LM == LM_IDENTITY) {  // integer values, two per packed operation
        // bin = v - lo + kBinOff, at most `never` (values at or above the
        // window, the field's level count included, rank as never) and, past
        // the first pass, at least `below`
        const uint32_t nv2 = never * 0x10001u;
        uint32_t Q[VEC / 2];  // Q[k] = (bin[2k], bin[2k+1])
        if (lo == 0) {        // uniform
            const u16x2 off = {(unsigned short)kBinOff, (unsigned short)kBinOff};
#pragma unroll
            for (int k = 0; k < VEC / 2; ++k) {
                u16x2 v = __builtin_bit_cast(u16x2, raw_pair<T>(raw.w, 2 * k));
                v = __builtin_elementwise_min(__builtin_elementwise_add_sat(v, off), __builtin_bit_cast(u16x2, nv2));
                Q[k] = __builtin_bit_cast(uint32_t, v);
            }
        } else {
            const unsigned short sub = (unsigned short)(lo - kBinOff);
            const u16x2 off = {sub, sub};
            const uint32_t bl2 = lb.below * 0x10001u;
#pragma unroll
            for (int k = 0; k < VEC / 2; ++k) {
                u16x2 v = __builtin_bit_cast(u16x2, raw_pair<T>(raw.w, 2 * k));
                v = __builtin_elementwise_max(__builtin_elementwise_sub_sat(v, off), __builtin_bit_cast(u16x2, bl2));
                v = __builtin_elementwise_min(v, __builtin_bit_cast(u16x2, nv2));
                Q[k] = __builtin_bit_cast(uint32_t, v);
            }
        }
        if (!full) {  // uniform: cells outside the field never enter
#pragma unroll
            for (int k = 0; k < VEC / 2; ++k) {
                const uint32_t m = ((raw.valid >> (2 * k)) & 1u ? 0u : 0xFFFFu) |
                                   ((raw.valid >> (2 * k + 1)) & 1u ? 0u : 0xFFFF0000u);
                Q[k] = bit_select(m, nv2, Q[k]);
            }
        }
        const uint32_t lq = from_lane_below(Q[VEC / 2 - 1]);
        const uint32_t rq = from_lane_above(Q[0]);
        P[0] = straddle(lq, Q[0]);
#pragma unroll
        for (int k = 0; k < VEC / 2; ++k) {
            P[2 * k + 1] = Q[k];
            P[2 * k + 2] = straddle(Q[k], k + 1 < VEC / 2 ? Q[k + 1] : rq);
        }
        return;
    }
    uint32_t lam[VEC];  // low 16 bits: the bin
    if constexpr (LM == LM_AFFINE) {
        const float hme = 0.5f - lv.eps;
        // estimates clamp to [below, never]; in the first pass to the bin of
        // level 0, since every value at or below t0 (however far) has level 0
        const float mlo = kMagic + (float)(lo == 0 ? (uint32_t)kBinOff : lb.below);
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
                const int k = (int)(lam[i] - kMagicBits);  // clamped bin estimate
                // only estimates of the levels [lo - 1, hi] can matter (the
                // true level is within one of the estimate)
                if (nr[i] && k >= kBinOff - 1 && k <= W + kBinOff) {
                    const int g0 = k + lo - kBinOff < 0 ? 0 : k + lo - kBinOff;
                    const int g = (int)level_settle(__uint_as_float(raw.w[i] ^ lv.neg), (uint32_t)g0, lv.L, thr);
                    lam[i] = g < lo ? lb.below : (g >= lo + W ? never : (uint32_t)(g - lo + kBinOff));
                }
            }
        }
    } else if constexpr (LM == LM_SEARCH) {
#pragma unroll
        for (int i = 0; i < VEC; ++i) lam[i] = bin_search(__uint_as_float(raw.w[i] ^ lv.neg), lo, lo + W, thr, lb);
    } else {
#pragma unroll
        for (int i = 0; i < VEC; ++i) {
            const int l = (int)level_of<T, LM>(as_value<T>(Elem<T>::get(raw.w, i)), lv, thr);
            lam[i] = (uint32_t)min(max(l - lo + kBinOff, (int)lb.below), (int)never);
        }
    }
    if (!full) {  // uniform: some lanes hold cells outside the field
#pragma unroll
        for (int i = 0; i < VEC; ++i)
            if (!(raw.valid >> i & 1u)) lam[i] = never;
    }
    // neighbours from the adjacent lanes by DPP wave shifts (lane 0's left and
    // lane 63's right are never used: those lanes only serve as halo)
    const uint32_t left = from_lane_below(lam[VEC - 1]);
    const uint32_t right = from_lane_above(lam[0]);
    P[0] = pack_lo16(left, lam[0]);
#pragma unroll
    for (int i = 1; i < VEC; ++i) P[i] = pack_lo16(lam[i - 1], lam[i]);
    P[VEC] = pack_lo16(lam[VEC - 1], right);
}

// Partials are stored level-major, [channel][level][workgroup] (int32), so that
// the merge reads the values of one bin contiguously.  `hist` points at the
// bin of level lo.
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

// the same bins added into the XCD's accumulator copy [3][L] (atomic drain)
__device__ __forceinline__ void drain_2d_acc(const uint64_t *hist, int W, int lo, int L, int64_t *__restrict__ acc,
                                             bool pack) {
    int64_t *a = acc + (int64_t)xcc_copy() * 3 * L;
    for (int b = threadIdx.x; b < W; b += blockDim.x) {
        const uint64_t v = hist[b];
        const int64_t n = (int64_t)(v >> kShiftCnt2);
        if (n == 0) continue;
        const int64_t per = (int64_t)((v >> kShiftPer2) & ((1ull << (kShiftCnt2 - kShiftPer2)) - 1)) -
                            kPerBias2 * n;
        const int64_t ec = (int64_t)(v & ((1ull << kShiftPer2) - 1)) - kEcBias2 * n;
        acc_add(a + lo + b, ec);
        if (pack) {  // uniform
            acc_add(a + L + lo + b, per + kPackBias * n + (n << kPackShift));
        } else {
            acc_add(a + L + lo + b, per);
            acc_add(a + 2 * L + lo + b, n);
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

// Where a lane's cells go: the LDS address of bin index b is mb * b + base,
// with mb the bytes per bin and base the LDS address of bin 0 for the lanes
// that own cells; a halo lane (lanes 0 and 63 of a strip only serve as
// neighbours) has mb = 0 and base = its own `never` bin, so its cells land
// there whatever their level.
struct LaneDst {
    uint32_t mb, base;
};

// The deltas of the VEC cells of `mid` into the LDS bins, one 64-bit atomic
// per cell at the address of its bin (two with CLS: the bins then hold two
// words and the tables are dl[0..255] and dl[256..511]).  Cells outside the
// pass window and every cell of a halo lane land in bins that are never
// drained; the atomics stay unconditional, so all table reads of a group are
// issued before its atomics.
//
// The north relation of a pair is the south relation of the pair above it,
// complemented: up - (mid + 1) = ~(mid - up) per 16-bit half.  So `sc` carries
// each pair's south difference from one row to the next and enters the
// pattern in the north position as it is; the tables are indexed with the
// north bit complemented (kNorthFlip2D).
template <int VEC, bool CLS>
__device__ __forceinline__ void emit_row(const uint32_t (&up)[VEC + 1], const uint32_t (&mid)[VEC + 1],
                                         const uint32_t (&dn)[VEC + 1], uint32_t (&sc)[VEC / 2],
                                         const LaneDst &ld, const uint64_t *dl) {
    // groups of up to 4 cell pairs: all table reads of a group are issued
    // before its atomics, so the atomics wait for one LDS round trip, not one each
    constexpr int NP = VEC / 2, GP = CLS ? (NP < 2 ? NP : 2) : (NP < 4 ? NP : 4);
#pragma unroll
    for (int g0 = 0; g0 < NP; g0 += GP) {
        uint64_t dv[2 * GP], dv2[CLS ? 2 * GP : 1];
        uint32_t addr[2 * GP];
#pragma unroll
        for (int q = 0; q < GP; ++q) {
            const int j = 2 * (g0 + q) + 1;
            const uint32_t self = mid[j], self1 = self + 0x00010001u;
            const uint32_t south = pk_diff(dn[j], self);
            const uint32_t acc = gather_offsets<3>(pk_diff(up[j - 1], self1), sc[g0 + q],
                                                   pk_diff(up[j + 1], self1), pk_diff(mid[j - 1], self1),
                                                   pk_diff(mid[j + 1], self), pk_diff(dn[j - 1], self), south,
                                                   pk_diff(dn[j + 1], self));
            sc[g0 + q] = south;
            addr[2 * q] = mad_lo16(self, ld.mb, ld.base);
            addr[2 * q + 1] = mad_hi16(self, ld.mb, ld.base);
            dv[2 * q] = lut_lo<uint64_t, 3>(dl, acc);
            dv[2 * q + 1] = lut_hi<uint64_t, 3>(dl, acc);
            if constexpr (CLS) {
                dv2[2 * q] = lut_lo<uint64_t, 3>(dl + 256, acc);
                dv2[2 * q + 1] = lut_hi<uint64_t, 3>(dl + 256, acc);
            }
        }
#pragma unroll
        for (int q = 0; q < 2 * GP; ++q) {
            lds_add64(addr[q], dv[q]);
            if constexpr (CLS) lds_add64(addr[q] + 8, dv2[q]);
        }
    }
}

// rows [ra, rb) of one strip; three row buffers whose roles rotate with the
// row index (PF is a multiple of 3, so the unrolled loop needs no copies)
template <typename T, int LM, int AL, int PF, bool CLS, typename TH>
__device__ __forceinline__ void stream_run_2d(const T *__restrict__ data, int h, int64_t w,
                                              const LevelArgs &lv, const TH &thr, int32_t lo, int W,
                                              float cpass, const uint64_t *dl, int64_t strip,
                                              int ra, int rb, int lane, const LaneBins &lb, const LaneDst &ld,
                                              ProgressPrio &pp, int64_t done0) {
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
    uint32_t sc[VEC / 2];    // south differences of the row above (see emit_row)
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
        convert_row<T, LM>(r0, ra - 1 >= 0, full, lv, thr, lo, W, cpass, lb, R[2]);
        convert_row<T, LM>(r1, true, full, lv, thr, lo, W, cpass, lb, R[0]);
#pragma unroll
        for (int q = 0; q < VEC / 2; ++q) sc[q] = pk_diff(R[0][2 * q + 1], R[2][2 * q + 1]);
    }
    int r0 = ra;
    // full blocks of PF rows: no conditional loads, so PF loads stay in flight;
    // the field's last row (whose row below is outside the field) is left to
    // the remainder, so that here every row below lies inside the field
    const int rb_full = rb == h ? rb - 1 : rb;
    for (; r0 + PF <= rb_full; r0 += PF) {
        pp.update(done0 + (r0 - ra));
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int r = r0 + k;  // current row (buffer k%3); ring[k] holds row r + 1
            convert_row<T, LM>(ring[k], true, full, lv, thr, lo, W, cpass, lb, R[(k + 1) % 3]);
            const int nx = r + 1 + PF < rb ? r + 1 + PF : rb;
            fetch_row<T, AL>(data, clamp_row(nx), w, x0, last_block, ring[k]);
            emit_row<VEC, CLS>(R[(k + 2) % 3], R[k % 3], R[(k + 1) % 3], sc, ld, dl);
        }
    }
    // remaining rows (at most PF); here r - ra = r0 - ra + k with r0 - ra
    // a multiple of PF, so the buffer roles are those of k again
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        const int r = r0 + k;
        if (r < rb) {
            convert_row<T, LM>(ring[k], r + 1 < h, full, lv, thr, lo, W, cpass, lb, R[(k + 1) % 3]);
            emit_row<VEC, CLS>(R[(k + 2) % 3], R[k % 3], R[(k + 1) % 3], sc, ld, dl);
        }
    }
}

// Work split: the (strip, row) units of rows [row_lo, row_hi) are ordered by
// bands of B rows, then strip, then row, and divided into equal contiguous
// ranges, one per wave (a range may run from one strip of a band into the
// next).  B is the units per wave, so a wave mostly takes one strip of one
// band, and the waves of a workgroup take neighbouring strips of the same
// rows: the cache line where two strips meet (each wave's row load reaches 16
// bytes into the next strip's first line) is fetched once from HBM and then
// found in the XCD's L2 by the neighbour.
template <typename T, int LM, int AL, int PF, bool CLS>
__global__ void __launch_bounds__(64 * kWaves2D)
    ecc2d_stream(const T *__restrict__ data, int64_t h, int64_t w, LevelArgs lv, int32_t lo,
                 int32_t hi, float cpass, const uint64_t *__restrict__ delta_lut, int32_t *__restrict__ partial,
                 int64_t row_lo, int64_t row_hi, int accumulate, int prio, int64_t *acc, int pack) {
    constexpr int VEC = Elem<T>::VEC;
    constexpr int CE = 62 * VEC;
    constexpr int BW = CLS ? 2 : 1;  // words per bin
    extern __shared__ uint64_t smem[];
    __shared__ uint64_t dl[256 * BW];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: keeps loop control scalar
    const int W = hi - lo;
    const int L = lv.L;
    // LDS: bins [0, W + 2 kBinOff) (kBinOff .. kBinOff + W - 1 are the
    // window's levels), then thresholds [lo-2, hi+1)
    const int n_bins = W + 2 * kBinOff;
    uint64_t *hist = smem;
    float *thr_s = reinterpret_cast<float *>(smem + BW * n_bins);
    constexpr bool kThr = LM == LM_AFFINE || LM == LM_SEARCH;
    if (kThr)
        for (int i = tid; i < W + 3; i += 64 * kWaves2D) {
            int k = lo - 2 + i;
            k = k < 0 ? 0 : (k >= L ? L - 1 : k);
            thr_s[i] = lv.thr[k];
        }
#pragma unroll
    for (int k = tid; k < 256 * BW; k += 64 * kWaves2D) dl[k] = delta_lut[k];
    for (int b = tid; b < BW * n_bins; b += 64 * kWaves2D) hist[b] = 0;
    __syncthreads();

    const int G = gridDim.x;
    const int wg = xcd_order(blockIdx.x, G);
    const int64_t gw = (int64_t)wg * kWaves2D + wave, NW = (int64_t)G * kWaves2D;
    const int64_t H = row_hi - row_lo;
    const int64_t n_strips = (w + CE - 1) / CE;
    const int64_t units = n_strips * H;
    const int64_t u_end = units * (gw + 1) / NW;
    const LaneBins lb{(uint32_t)lane, (uint32_t)(W + kBinOff + lane)};
    const bool halo = lane == 0 || lane == 63;
    const uint32_t h0 = lds_addr(hist);
    const LaneDst ld{halo ? 0u : 8u * BW, halo ? h0 + 8u * BW * lb.never : h0};
    const ThrLds thr{thr_s, lo - 2};
    const int64_t u_beg = units * gw / NW;
    const int64_t B = (units + NW - 1) / NW < H ? (units + NW - 1) / NW : H;  // rows per band
    const int64_t BU = n_strips * B;                                         // units per full band
    ProgressPrio pp;
    pp.init(prio != 0, u_end - u_beg);
    for (int64_t u = u_beg; u < u_end;) {
        const int64_t band = u / BU, r0 = band * B;
        const int64_t hb = H - r0 < B ? H - r0 : B;  // rows of this band (the last may be short)
        const int64_t rem = u - band * BU, strip = rem / hb, ra = r0 + rem % hb;
        const int64_t rb = ra + (u_end - u) < r0 + hb ? ra + (u_end - u) : r0 + hb;
        stream_run_2d<T, LM, AL, PF, CLS>(data, (int)h, w, lv, thr, lo, W, cpass, dl, strip, (int)(row_lo + ra),
                                          (int)(row_lo + rb), lane, lb, ld, pp, u - u_beg);
        u += rb - ra;
    }
    __syncthreads();
    if constexpr (CLS)
        drain_cls(hist + 2 * kBinOff, W, lo, L, G, wg, partial, accumulate == 0);
    else if (acc)
        drain_2d_acc(hist + kBinOff, W, lo, L, acc, pack != 0);
    else
        drain_2d(hist + kBinOff, W, lo, L, G, wg, partial, accumulate == 0);
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
        uint64_t *hist = smem;  // bins [0, L + 2 kBinOff): kBinOff + l is level l
        float *thr_s = reinterpret_cast<float *>(smem + L + 2 * kBinOff);
        for (int b = tid; b < L + 2 * kBinOff; b += 256) hist[b] = 0;
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
        lv.eps_far = f.eps;  // one pass window, starting at level 0
        lv.neg = f.neg;
        const ThrLds thr{thr_s, -2};
        const LaneBins lb{(uint32_t)lane, (uint32_t)(L + kBinOff + lane)};
        const uint32_t h0 = lds_addr(hist);
        const LaneDst ld{halo_lane ? 0u : 8u, halo_lane ? h0 + 8u * lb.never : h0};
        ProgressPrio pp;  // (off in the batched kernel)
        const int n = item.u1 - item.u0;
        const int u_end = item.u0 + (int)((int64_t)n * (wave + 1) / kWavesPerWG);
        for (int u = item.u0 + (int)((int64_t)n * wave / kWavesPerWG); u < u_end;) {
            const int strip = u / h, ra = u % h;
            const int rb = ra + (u_end - u) < h ? ra + (u_end - u) : h;
            stream_run_2d<T, LM, kLoadVector, PF, false>((const T *)f.data, h, w, lv, thr, 0, L, f.cpass,
                                                         dl[f.conn_idx], strip, ra, rb, lane, lb, ld, pp, 0);
            u += rb - ra;
        }
        __syncthreads();
        // bins -> the field's global histogram (levels hist[kBinOff .. kBinOff + L))
        for (int b = tid; b < L; b += 256) {
            const uint64_t v = hist[kBinOff + b];
            if (v == 0) continue;
            const int64_t cnt = (int64_t)(v >> kShiftCnt2);
            const int64_t per = (int64_t)((v >> kShiftPer2) & ((1ull << (kShiftCnt2 - kShiftPer2)) - 1)) -
                                kPerBias2 * cnt;
            const int64_t ec = (int64_t)(v & ((1ull << kShiftPer2) - 1)) - kEcBias2 * cnt;
            int32_t *dst = f.hist + b;
            if (ec) atomicAdd(dst, (int32_t)ec);
            if (per) atomicAdd(dst + L, (int32_t)per);
            atomicAdd(dst + 2 * L, (int32_t)cnt);
        }
        // the workgroup that adds last scans the field's histogram into its
        // curves (and clears it)
        if (take_field_ticket(f.done, f.n_items))  // uniform
            scan_field_hist(f.hist, 3, L, f.out, reinterpret_cast<int64_t *>(smem), part, f.done);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
size_t lds_bytes_2d(int window, bool classes) {
    return (size_t)(classes ? 2 : 1) * (window + 2 * kBinOff) * 8 + (size_t)(window + 3) * 4;
}

int load_mode_2d(const void *data, int64_t h, int64_t w, int elem_bytes) {
    (void)h;
    return ((uintptr_t)data % 16 == 0 && (w * elem_bytes) % 16 == 0) ? kLoadAligned : kLoadVector;
}

// cells one workgroup may add to its LDS bins in a launch of `rows` rows
static int64_t max_wg_cells_2d(int64_t rows, int64_t w, int vec, int grid) {
    const int64_t ce = 62 * vec;
    const int64_t units = ((w + ce - 1) / ce) * rows;
    const int64_t NW = (int64_t)grid * kWaves2D;
    return kWaves2D * ((units + NW - 1) / NW + 1) * ce;
}

template <typename T, int LM, int AL, bool CLS>
static int launch_2d_t(const Launch2D &a, hipStream_t s) {
    // rows in flight per wave: fewer for the variants with the most registers
    // per row (the 16-wave workgroup allows 128 VGPRs)
    constexpr int VEC = Elem<T>::VEC, PF = (sizeof(T) == 1 || LM == LM_LUT) ? 3 : 6;
    const int W = a.hi - a.lo;
    // the packed LDS bins of one workgroup may see at most kFlush2D (class
    // counts: kFlushCls) cells: split tall fields into row chunks that respect
    // it (later chunks add to the partials of the first)
    const int64_t flush = CLS ? kFlushCls : kFlush2D;
    int64_t chunk = a.row_hi - a.row_lo;
    while (chunk > 1 && max_wg_cells_2d(chunk, a.w, VEC, a.grid) > flush) chunk = (chunk + 1) / 2;
    if (max_wg_cells_2d(chunk, a.w, VEC, a.grid) > flush) return (int)hipErrorInvalidValue;
    // affine levels: the pass constant -t0/step + kBinOff + 0.5 - lo, rounded
    // once, and the margin that holds for it
    const float cpass = pass_constant(a.lv.u0d, a.lo);
    LevelArgs lv = a.lv;
    if (a.lo != 0) lv.eps = lv.eps_far;
    const size_t lds = lds_bytes_2d(W, CLS);
    for (int64_t r0 = a.row_lo; r0 < a.row_hi; r0 += chunk) {
        const int64_t r1 = r0 + chunk < a.row_hi ? r0 + chunk : a.row_hi;
        const bool acc = a.accumulate || r0 > a.row_lo;
        hipExtLaunchKernelGGL((ecc2d_stream<T, LM, AL, PF, CLS>), dim3(a.grid), dim3(64 * kWaves2D), lds, s,
                              r0 == a.row_lo ? (hipEvent_t)a.ev_start : nullptr,
                              r1 == a.row_hi ? (hipEvent_t)a.ev_stop : nullptr, 0, (const T *)a.data, a.h, a.w,
                              lv, a.lo, a.hi, cpass, a.delta_lut, a.partial, r0, r1, acc ? 1 : 0,
                              progress_prio() ? 1 : 0, CLS ? nullptr : a.acc, !CLS && a.acc && a.pack ? 1 : 0);
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

}  // namespace ecc
