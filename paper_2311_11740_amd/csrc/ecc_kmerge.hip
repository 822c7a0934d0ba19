// Merge of per-workgroup partials with the prefix scan over levels, and the
// value -> level table kernel.
#include "ecc_device.h"

namespace ecc {

// ---------------------------------------------------------------------------
// merge of per-workgroup partials and prefix scan over levels
// ---------------------------------------------------------------------------
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
        const int64_t s = sum_bin_wave(partial + bin * G, G, lane);
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
    scan_totals_block(totals, nch, L, out);
    if (threadIdx.x == 0) *counter = 0u;  // ready for the next merge
}

// Sums the kAccCopies accumulator copies of every bin (and clears them) and
// scans, one block per channel: the block sums the copies of its
// channel's bins in chunks of kMergeChChunk levels (every load of a thread in
// flight at once), clears them, keeps the chunk's per-level totals in LDS and
// writes the running sums, carried from chunk to chunk.  Blocks share nothing,
// so there is no ticket and no device-scope fence.
constexpr int kMergeChChunk = 4096;
constexpr int kMergeChThreads = 1024;
__global__ void __launch_bounds__(kMergeChThreads)
    ecc_merge_acc_ch(int64_t *__restrict__ acc, int nch, int L, OutPtrs out, int64_t *__restrict__ rows) {
    constexpr int PER = kMergeChChunk / kMergeChThreads;  // levels per thread and chunk
    __shared__ int64_t tot[kMergeChChunk];
    __shared__ int64_t wsum[kMergeChThreads / 64];
    const int ch = blockIdx.x, t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const unsigned nb = (unsigned)(nch * L);  // 32-bit offsets from one base: scalar-base loads
    int64_t *a = acc + (int64_t)ch * L;
    int64_t *dst = rows ? rows + (int64_t)ch * L : out.p[ch];
    int64_t carry = 0;  // running sum of the earlier chunks
    for (int l0 = 0; l0 < L; l0 += kMergeChChunk) {
        const int n = L - l0 < kMergeChChunk ? L - l0 : kMergeChChunk;
        // unconditional loads and stores at indices wrapped into the chunk (a
        // conditional load would be waited for before the next one is
        // issued); wrapped duplicates are not counted
        unsigned lc[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i) lc[i] = (unsigned)(l0 + (i * kMergeChThreads + t) % n);
        // (groups i of 1024 levels past the chunk's end are skipped: uniform)
        int64_t v[kAccCopies][PER];
#pragma unroll
        for (int c = 0; c < kAccCopies; ++c)
#pragma unroll
            for (int i = 0; i < PER; ++i)
                v[c][i] = i * kMergeChThreads < n ? __builtin_nontemporal_load(a + c * nb + lc[i]) : 0;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            int64_t s = 0;
#pragma unroll
            for (int c = 0; c < kAccCopies; ++c) s += v[c][i];
            if (i * kMergeChThreads + t < n) tot[i * kMergeChThreads + t] = s;
        }
        __syncthreads();  // every thread has read its copies before any is cleared
#pragma unroll
        for (int c = 0; c < kAccCopies; ++c)
#pragma unroll
            for (int i = 0; i < PER; ++i)
                if (i * kMergeChThreads < n) a[c * nb + lc[i]] = 0;
        // thread t scans the chunk's levels [t * per, (t + 1) * per)
        const int per = (n + kMergeChThreads - 1) / kMergeChThreads;
        const int beg = t * per < n ? t * per : n, end = beg + per < n ? beg + per : n;
        int64_t sum = 0;
        for (int i = beg; i < end; ++i) sum += tot[i];
        int64_t x = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        int64_t run = carry + x - sum;
        for (int k = 0; k < wave; ++k) run += wsum[k];
        if (dst)  // uniform
            for (int i = beg; i < end; ++i) {
                run += tot[i];
                dst[l0 + i] = run;
            }
        for (int k = 0; k < kMergeChThreads / 64; ++k) carry += wsum[k];
        __syncthreads();  // tot and wsum are reused by the next chunk
    }
}

// The same for more than kMergeSplit levels, in two short kernels instead of
// one block walking every chunk of a channel in turn: block (ch, k) sums and
// clears the copies of levels [k kMergeSplit, (k + 1) kMergeSplit), one level
// per thread, writes the chunk's own running sums and its total
// (chunk_tot[ch][k]); ecc_merge_carry then adds to every chunk the totals of
// the chunks before it.
constexpr int kMergeSplit = kMergeChThreads;
// With pack_ch >= 0, channel pack_ch holds the boundary measure and the count
// packed as the atomic drains write them (kPackShift): its block writes both curves (pack_ch and
// pack_ch + 1) and both chunk totals, and the block of pack_ch + 1 has nothing
// to do.
__global__ void __launch_bounds__(kMergeChThreads)
    ecc_merge_acc_split(int64_t *__restrict__ acc, int nch, int L, OutPtrs out, int64_t *__restrict__ chunk_tot,
                        int pack_ch) {
    __shared__ int64_t wsum[kMergeChThreads / 64], wsum2[kMergeChThreads / 64];
    const int ch = blockIdx.x, k = blockIdx.y, t = threadIdx.x, lane = t & 63, wave = t >> 6;
    if (pack_ch >= 0 && ch == pack_ch + 1) return;  // uniform: its curve comes from pack_ch
    const bool packed = ch == pack_ch;
    const unsigned nb = (unsigned)(nch * L);
    int64_t *a = acc + (int64_t)ch * L;
    const int l0 = k * kMergeSplit, n = L - l0 < kMergeSplit ? L - l0 : kMergeSplit;
    const bool in = t < n;
    // unconditional loads; a thread past the chunk's end re-reads level l0 and
    // discards it, and only the thread that owns a level clears it
    const unsigned li = (unsigned)(l0 + (in ? t : 0));
    int64_t v[kAccCopies];
#pragma unroll
    for (int c = 0; c < kAccCopies; ++c) v[c] = __builtin_nontemporal_load(a + c * nb + li);
    uint64_t sum = 0;
#pragma unroll
    for (int c = 0; c < kAccCopies; ++c) sum += (uint64_t)v[c];
    if (!in) sum = 0;
    if (in)
#pragma unroll
        for (int c = 0; c < kAccCopies; ++c) a[c * nb + li] = 0;
    // packed: boundary + kPackBias n in the low kPackShift bits, n above
    const int64_t cnt = packed ? (int64_t)(sum >> kPackShift) : 0;
    int64_t x = packed ? (int64_t)(sum & ((1ull << kPackShift) - 1)) - kPackBias * cnt : (int64_t)sum;
    int64_t x2 = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t y = __shfl_up(x, off), y2 = __shfl_up(x2, off);
        if (lane >= off) {
            x += y;
            x2 += y2;
        }
    }
    if (lane == 63) {
        wsum[wave] = x;
        wsum2[wave] = x2;
    }
    __syncthreads();
    int64_t run = x, tot = 0, run2 = x2, tot2 = 0;
    for (int w = 0; w < kMergeChThreads / 64; ++w) {
        const int64_t ws = wsum[w], ws2 = wsum2[w];
        if (w < wave) {
            run += ws;
            run2 += ws2;
        }
        tot += ws;
        tot2 += ws2;
    }
    int64_t *dst = out.p[ch];
    if (in && dst) dst[l0 + t] = run;
    if (t == 0) chunk_tot[ch * gridDim.y + k] = tot;
    if (packed) {  // uniform
        int64_t *dst2 = out.p[ch + 1];
        if (in && dst2) dst2[l0 + t] = run2;
        if (t == 0) chunk_tot[(ch + 1) * gridDim.y + k] = tot2;
    }
}

__global__ void __launch_bounds__(kMergeChThreads)
    ecc_merge_carry(int L, int n_chunks, OutPtrs out, const int64_t *__restrict__ chunk_tot) {
    const int ch = blockIdx.x, k = blockIdx.y + 1;
    int64_t *dst = out.p[ch];
    if (!dst) return;  // uniform
    int64_t carry = 0;
    for (int j = 0; j < k; ++j) carry += chunk_tot[ch * n_chunks + j];
    const int l = k * kMergeSplit + (int)threadIdx.x;
    if (l < L) dst[l] += carry;
}

__global__ void ecc_zero(u32x4 *__restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = u32x4{0u, 0u, 0u, 0u};
}

// level index of every integer value from the thresholds (integer fields with
// a threshold array; superlevel: the thresholds are -t and the value -v)
__global__ void ecc_level_lut(const float *__restrict__ thr, int L, int n_values, int neg,
                              uint16_t *__restrict__ lut) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n_values) return;
    const float x = neg ? -(float)v : (float)v;
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

int launch_merge_acc(int64_t *acc, int copies, int nch, int L, int64_t *const out[4], int64_t *totals,
                     unsigned *counter, void *stream, int pack_ch) {
    OutPtrs o;
    for (int c = 0; c < 4; ++c) o.p[c] = c < nch ? out[c] : nullptr;
    (void)counter;
    if (copies != kAccCopies || nch > 4) return (int)hipErrorInvalidValue;
    if (pack_ch >= 0 && (!totals || pack_ch + 1 >= nch)) return (int)hipErrorInvalidValue;
    if (!totals) {
        hipLaunchKernelGGL(ecc_merge_acc_ch, dim3(nch), dim3(kMergeChThreads), 0, (hipStream_t)stream, acc, nch, L,
                           o, (int64_t *)nullptr);
        return (int)hipGetLastError();
    }
    // chunks of kMergeSplit levels side by side, then (more than one chunk)
    // the carries; the chunk totals take nch x chunks words of the caller's
    // nch x L totals
    const int n_chunks = (L + kMergeSplit - 1) / kMergeSplit;
    hipLaunchKernelGGL(ecc_merge_acc_split, dim3(nch, n_chunks), dim3(kMergeChThreads), 0, (hipStream_t)stream, acc,
                       nch, L, o, totals, pack_ch);
    int e = (int)hipGetLastError();
    if (e || n_chunks == 1) return e;
    hipLaunchKernelGGL(ecc_merge_carry, dim3(nch, n_chunks - 1), dim3(kMergeChThreads), 0, (hipStream_t)stream, L,
                       n_chunks, o, (const int64_t *)totals);
    return (int)hipGetLastError();
}

int launch_merge_acc_rows(int64_t *acc, int nch, int L, int64_t *rows, void *stream) {
    if (nch > 64) return (int)hipErrorInvalidValue;
    OutPtrs o{{nullptr, nullptr, nullptr, nullptr}};
    hipLaunchKernelGGL(ecc_merge_acc_ch, dim3(nch), dim3(kMergeChThreads), 0, (hipStream_t)stream, acc, nch, L, o,
                       rows);
    return (int)hipGetLastError();
}

int launch_zero(void *p, size_t bytes, void *stream) {
    const int64_t n = (int64_t)(bytes / 16);
    const int blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256));
    hipLaunchKernelGGL(ecc_zero, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (u32x4 *)p, n);
    return (int)hipGetLastError();
}

int launch_level_lut(const float *thr, int L, int n_values, uint16_t *lut, bool neg, void *stream) {
    hipLaunchKernelGGL(ecc_level_lut, dim3((n_values + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, thr, L, n_values, neg ? 1 : 0, lut);
    return (int)hipGetLastError();
}

}  // namespace ecc
