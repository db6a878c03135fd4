// Plain failure-less scan: the paper's own kernel design (Section 2.3) on gfx950.
//
// One lane per start position walks the goto-only trie held in HBM (through L2) with
// Eq. 1, and a second pass writes the matches. Each block owns kPlainRows rows of 256
// consecutive start positions; pass 1 counts matches per block, a one-block kernel turns
// the block counts into offsets, and pass 2 recounts row by row, scans the row's counts
// across the block, and writes each start's keys at its place, so the output is sorted
// without a global sort.
//
// This path is kept as the in-library baseline the optimized scan is measured against
// (same output, bit for bit); it is selected with PFAC_ALGO_PLAIN.
#include <algorithm>

#include "pfac_impl.h"
#include "kernels.h"

namespace pfac {

namespace {

constexpr int kPlainThreads = 256;
constexpr int kPlainRows = 16;  // positions per block = 256 * 16

// Child of q on symbol c, or -1 when the bit for c is clear (Eq. 1); term: whether the
// child is terminal.
template <int LAYOUT>
__device__ __forceinline__ int64_t step(const DevTable &t, uint32_t q, uint32_t c, bool &term) {
    if (LAYOUT == LAYOUT_NARROW) {
        uint64_t w = t.nodes[q];
        uint32_t bm = (uint32_t)w;
        if (!((bm >> c) & 1u)) return -1;
        uint32_t child = (uint32_t)(w >> 32) & kNarrowIndexMask;
        child += __builtin_popcount(bm & ((1u << c) - 1u));
        term = (t.nodes[child] >> 63) != 0;
        return child;
    } else {
        uint32_t w = c >> 6, b = c & 63;
        uint64_t word = t.bm[((size_t)q << t.nw_log2) + w];
        if (!((word >> b) & 1ull)) return -1;
        uint64_t meta = t.nodes[q];
        uint32_t child = (uint32_t)meta;
        if (w) child += (uint32_t)(meta >> (32 + 8 * (w - 1))) & 0xffu;
        child += __builtin_popcountll(word & ((1ull << b) - 1ull));
        term = (t.nodes[child] >> 63) != 0;
        return child;
    }
}

// The plain table stores a unary path below a tail head as one record (its nodes are
// not stored); the walk here still takes it one symbol per step: the number of path
// symbols text[p ..] matches, and its record.
__device__ __forceinline__ uint4 tail_of(const DevTable &t, uint64_t w, int layout) {
    const uint32_t x = layout == LAYOUT_NARROW ? (uint32_t)(w >> 32) & kNarrowIndexMask : (uint32_t)w;
    return reinterpret_cast<const uint4 *>(t.tails)[x];
}
__device__ __forceinline__ uint32_t tail_match(const DevTable &t, uint4 tr, const uint8_t *text, uint64_t p,
                                               uint64_t end) {
    uint32_t k = 0;
    while (k < tr.y && p + k < end && text[p + k] == t.tail_bytes[tr.x + k]) k++;
    return k;
}

// Number of pattern ids on the walk from start s (every terminal the walk passes).
template <int LAYOUT>
__device__ uint32_t count_at(const DevTable &t, const uint8_t *text, uint64_t s, uint64_t end) {
    uint32_t q = 0, cnt = 0;
    for (uint64_t p = s; p < end; p++) {
        const uint64_t w = t.nodes[q];
        if (w & kTailBit) {
            const uint4 tr = tail_of(t, w, LAYOUT);
            if (tail_match(t, tr, text, p, end) == tr.y) cnt += tr.w;
            break;
        }
        uint32_t c = text[p];
        if (c >= t.alphabet) break;
        bool term = false;
        int64_t nq = step<LAYOUT>(t, q, c, term);
        if (nq < 0) break;
        q = (uint32_t)nq;
        if (term) cnt += t.out_first[q + 1] - t.out_first[q];
    }
    return cnt;
}

// Write the keys of start s to keys[o .. o + cnt) in (start, id) order, if they all fit.
template <int LAYOUT>
__device__ void emit_at(const DevTable &t, const uint8_t *text, uint64_t s, uint64_t end,
                        uint64_t *keys, uint64_t o, uint32_t cnt, uint64_t cap) {
    if (o + cnt > cap) return;  // capacity overflow: content unspecified, count still right
    uint32_t q = 0, k = 0, nterm = 0;
    const uint64_t hi = s << 32;
    for (uint64_t p = s; p < end && k < cnt; p++) {
        const uint64_t w = t.nodes[q];
        if (w & kTailBit) {
            const uint4 tr = tail_of(t, w, LAYOUT);
            if (tail_match(t, tr, text, p, end) == tr.y) {
                nterm++;
                if (tr.w == 1) keys[o + k++] = hi | tr.z;  // the record holds the id itself
                else
                    for (uint32_t i = tr.z; i < tr.z + tr.w; i++) keys[o + k++] = hi | t.out_ids[i];
            }
            break;
        }
        uint32_t c = text[p];
        if (c >= t.alphabet) break;
        bool term = false;
        int64_t nq = step<LAYOUT>(t, q, c, term);
        if (nq < 0) break;
        q = (uint32_t)nq;
        if (term) {
            nterm++;
            for (uint32_t i = t.out_first[q]; i < t.out_first[q + 1]; i++) keys[o + k++] = hi | t.out_ids[i];
        }
    }
    if (nterm > 1) {  // ids of several nested patterns: order them (each list is sorted)
        for (uint32_t i = 1; i < cnt; i++) {
            uint64_t v = keys[o + i];
            uint32_t j = i;
            while (j > 0 && keys[o + j - 1] > v) {
                keys[o + j] = keys[o + j - 1];
                j--;
            }
            keys[o + j] = v;
        }
    }
}

__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// Exclusive scan over the block (256 threads = 4 waves); returns the total in *total.
__device__ uint64_t block_excl_scan(uint64_t v, uint64_t *total, uint64_t *sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t inc = wave_incl_scan(v);
    if (lane == 63) sh[wave] = inc;
    __syncthreads();
    uint64_t before = 0, tot = 0;
    for (int w = 0; w < kPlainThreads / 64; w++) {
        if (w < wave) before += sh[w];
        tot += sh[w];
    }
    __syncthreads();
    *total = tot;
    return before + inc - v;
}

template <int LAYOUT>
__global__ __launch_bounds__(kPlainThreads) void plain_count(DevTable t, const uint8_t *text,
                                                             uint64_t n, uint64_t *block_counts) {
    __shared__ uint64_t sh[kPlainThreads / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kPlainThreads * kPlainRows;
    uint64_t cnt = 0;
    for (int r = 0; r < kPlainRows; r++) {
        uint64_t s = base + (uint64_t)r * kPlainThreads + threadIdx.x;
        if (s < n) cnt += count_at<LAYOUT>(t, text, s, n);
    }
    uint64_t tot;
    block_excl_scan(cnt, &tot, sh);
    if (threadIdx.x == 0) block_counts[blockIdx.x] = tot;
}

// One block turns per-block counts into exclusive offsets and writes the total.
__global__ __launch_bounds__(1024) void plain_offsets(const uint64_t *counts, uint64_t nb,
                                                     uint64_t *offsets, uint64_t *d_count) {
    __shared__ uint64_t sh[16];
    __shared__ uint64_t carry;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint64_t a = 0; a < nb; a += 1024) {
        uint64_t i = a + threadIdx.x;
        uint64_t v = i < nb ? counts[i] : 0;
        uint64_t inc = wave_incl_scan(v);
        if (lane == 63) sh[wave] = inc;
        __syncthreads();
        uint64_t before = carry, tot = 0;
        for (int w = 0; w < 16; w++) {
            if (w < wave) before += sh[w];
            tot += sh[w];
        }
        if (i < nb) offsets[i] = before + inc - v;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *d_count = carry;
}

template <int LAYOUT>
__global__ __launch_bounds__(kPlainThreads) void plain_emit(DevTable t, const uint8_t *text,
                                                            uint64_t n, const uint64_t *offsets,
                                                            uint64_t *keys, uint64_t cap) {
    __shared__ uint64_t sh[kPlainThreads / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kPlainThreads * kPlainRows;
    uint64_t o = offsets[blockIdx.x];
    for (int r = 0; r < kPlainRows; r++) {
        uint64_t s = base + (uint64_t)r * kPlainThreads + threadIdx.x;
        uint32_t c = s < n ? count_at<LAYOUT>(t, text, s, n) : 0;
        uint64_t row_total;
        uint64_t mine = block_excl_scan(c, &row_total, sh);
        if (c) emit_at<LAYOUT>(t, text, s, n, keys, o + mine, c, cap);
        o += row_total;
    }
}

// Prefix depths (Section 2.4's truncated trie, Section 4.2's study): for every start the
// number of Eq. 1 steps the walk takes before a transition is missing, capped at `cap`,
// gathered into hist[0 .. cap] (the last bin: depth cap or more). One lane per start,
// grid-stride; each workgroup keeps its bins in LDS and adds them to hist once.
constexpr uint32_t kHistMaxBins = 64;

__global__ void hist_zero(uint64_t *hist, uint32_t bins) {
    for (uint32_t i = threadIdx.x; i < bins; i += blockDim.x) hist[i] = 0;
}

template <int LAYOUT>
__global__ __launch_bounds__(kPlainThreads) void prefix_hist(DevTable t, const uint8_t *text, uint64_t n,
                                                             uint32_t cap, uint64_t *hist) {
    __shared__ uint32_t bins[kHistMaxBins];
    for (uint32_t i = threadIdx.x; i < kHistMaxBins; i += kPlainThreads) bins[i] = 0;
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * kPlainThreads;
    for (uint64_t s = (uint64_t)blockIdx.x * kPlainThreads + threadIdx.x; s < n; s += stride) {
        uint32_t q = 0, d = 0;
        for (uint64_t p = s; p < n && d < cap; p++) {
            const uint64_t w = t.nodes[q];
            if (w & kTailBit) {  // the rest of a unary path, symbol by symbol
                const uint4 tr = tail_of(t, w, LAYOUT);
                const uint32_t m = tail_match(t, tr, text, p, n);
                d = d + m < cap ? d + m : cap;
                break;
            }
            const uint32_t c = text[p];
            if (c >= t.alphabet) break;
            bool term = false;
            const int64_t nq = step<LAYOUT>(t, q, c, term);
            if (nq < 0) break;
            q = (uint32_t)nq;
            d++;
        }
        atomicAdd(&bins[d], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i <= cap; i += kPlainThreads)
        if (bins[i]) atomicAdd((unsigned long long *)&hist[i], (unsigned long long)bins[i]);
}

}  // namespace

int launch_plain(const DevTable &t, const uint8_t *text, uint64_t n, uint64_t *keys,
                 uint64_t cap, uint64_t *d_count, uint64_t *block_counts,
                 uint64_t *block_offsets, hipStream_t s) {
    const uint64_t per = (uint64_t)kPlainThreads * kPlainRows;
    const uint64_t nb = (n + per - 1) / per;
    if (t.layout == LAYOUT_NARROW)
        plain_count<LAYOUT_NARROW><<<(unsigned)nb, kPlainThreads, 0, s>>>(t, text, n, block_counts);
    else
        plain_count<LAYOUT_WIDE><<<(unsigned)nb, kPlainThreads, 0, s>>>(t, text, n, block_counts);
    plain_offsets<<<1, 1024, 0, s>>>(block_counts, nb, block_offsets, d_count);
    if (t.layout == LAYOUT_NARROW)
        plain_emit<LAYOUT_NARROW><<<(unsigned)nb, kPlainThreads, 0, s>>>(t, text, n, block_offsets, keys, cap);
    else
        plain_emit<LAYOUT_WIDE><<<(unsigned)nb, kPlainThreads, 0, s>>>(t, text, n, block_offsets, keys, cap);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_prefix_hist(const DevTable &t, const uint8_t *text, uint64_t n, uint32_t cap, uint64_t *hist,
                       uint32_t cus, hipStream_t s) {
    if (cap == 0 || cap >= kHistMaxBins) return -1;
    hist_zero<<<1, 64, 0, s>>>(hist, cap + 1);
    const uint64_t want = (n + kPlainThreads - 1) / kPlainThreads;
    const uint64_t grid = std::min<uint64_t>(want ? want : 1, (uint64_t)cus * 8);
    if (n) {
        if (t.layout == LAYOUT_NARROW)
            prefix_hist<LAYOUT_NARROW><<<(unsigned)grid, kPlainThreads, 0, s>>>(t, text, n, cap, hist);
        else
            prefix_hist<LAYOUT_WIDE><<<(unsigned)grid, kPlainThreads, 0, s>>>(t, text, n, cap, hist);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

uint64_t plain_blocks(uint64_t n) {
    const uint64_t per = (uint64_t)kPlainThreads * kPlainRows;
    return (n + per - 1) / per;
}

}  // namespace pfac
