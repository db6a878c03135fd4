// Tiled failure-less scan for gfx950: one persistent kernel per scan.
//
// The method is Section 2.3's: every start position walks the goto-only trie until a
// transition is missing, reporting every pattern whose final state it reaches; nodes
// are found with Eq. 1. What changes on this GPU is how the positions reach the walk.
//
//  * Tiles. Persistent workgroups take kTile-byte tiles in increasing order from an
//    atomic ticket. A tile and a halo after it are staged into LDS with 16-byte loads,
//    so a walk never re-reads HBM for text it has already fetched.
//  * LDS prefilter. No pattern is shorter than min_len, so a start can only match if its
//    first k = min(min_len, kmax) symbols are the first k symbols of some pattern. Every
//    position is tested against an LDS bitmap: either a hashed k-gram bitmap, or the
//    root image itself. A clear bit proves there is no match at that start; a set bit
//    sends the start to the walk, which decides exactly.
//  * Root image. The top D levels of the trie are folded into one direct-indexed bitmap
//    over D-symbol keys (lexicographic), with a rank word per 32 bits. The rank of a key
//    is the breadth-first index of its depth-D node minus the first depth-D index: Eq. 1's
//    popcount rule applied to a D-symbol root. Survivors start their walk there.
//  * Survivors are compacted (popcount prefix over the tile's survivor bitmap) into
//    batches of one start per lane, so the deep, divergent part of the walk runs on
//    dense waves. Walks read nodes from HBM through L2.
//  * Output. The tile's match count is published and the tile's output offset is found
//    by decoupled look-back over earlier tiles; matching starts are revisited in
//    position order and their keys written at their final place, sorted by (start, id)
//    without any global sort.
#include <mutex>

#include "kernels.h"
#include "pfac_impl.h"
#include "scan_internal.h"

namespace pfac {
namespace {

constexpr uint64_t kFlagAgg = 1, kFlagInc = 2;
constexpr uint32_t kSpinLimit = 1u << 24;

struct Lds {
    uint32_t *img;       // root bitmap | rank (u16) | filter
    uint8_t *text;       // kTile + kHalo bytes
    uint16_t *surv;      // survivor bits, 16 positions per entry, position order
    uint16_t *hits;      // starts with at least one match, same layout
    uint16_t *queue;     // one batch of local positions (kThreads)
    uint32_t *red;       // per-wave partial sums (kWaves * 2 words)
    uint32_t *misc;      // [0] ticket, [1] next ticket, [2] epoch, [3] flags
    uint64_t *red64;     // per-wave 64-bit partials
};

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t u = __shfl_up(v, d, 64);
        if (lane >= (uint32_t)d) v += u;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Exclusive scan of v over the workgroup; *total gets the sum. Two barriers.
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t *total, uint32_t *red) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) red[wave] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (uint32_t w = 0; w < kWaves; w++) {
        uint32_t x = red[w];
        before += w < wave ? x : 0;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return before + inc - v;
}

__device__ uint64_t block_sum64(uint64_t v, uint64_t *red64) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_sum64(v);
    if (lane == 0) red64[wave] = v;
    __syncthreads();
    uint64_t tot = 0;
#pragma unroll
    for (uint32_t w = 0; w < kWaves; w++) tot += red64[w];
    __syncthreads();
    return tot;
}

// ------------------------------------------------------------------------ the walk
template <int LAYOUT, bool PACK2, bool SEG>
struct Walk {
    const DevTable &t;
    const uint8_t *__restrict__ gtext;
    const uint32_t *img;   // LDS image
    const uint8_t *ltext;  // LDS text tile
    uint64_t base;         // global index of local position 0

    __device__ __forceinline__ uint32_t sym(uint64_t i) const {
        uint64_t li = i - base;
        return li < kTile + kHalo ? (uint32_t)ltext[li] : (uint32_t)gtext[i];
    }

    // Node reached from the root image by the D symbols at s, or -1.
    __device__ __forceinline__ int64_t root(uint64_t s, uint64_t end) const {
        const uint32_t D = t.root_depth;
        if (s + D > end) return -1;
        uint32_t key = 0;
        if (PACK2) {
            for (uint32_t i = 0; i < D; i++) {
                uint32_t c = sym(s + i);
                if (c > 3) return -1;  // a byte outside the 2-bit code space
                key = (key << 2) | c;
            }
        } else {
            for (uint32_t i = 0; i < D; i++) key = (key << 8) | sym(s + i);
        }
        const uint32_t w = key >> 5, b = key & 31;
        const uint32_t word = img[w];
        if (!((word >> b) & 1u)) return -1;
        const uint16_t *rank = reinterpret_cast<const uint16_t *>(img + t.rank_word);
        return (int64_t)t.root_base + rank[w] + __builtin_popcount(word & ((1u << b) - 1u));
    }

    __device__ __forceinline__ bool is_term(uint32_t q) const { return (t.nodes[q] >> 63) != 0; }

    // Child of q on c (Eq. 1), or -1.
    __device__ __forceinline__ int64_t child(uint32_t q, uint32_t c) const {
        if (c >= t.alphabet) return -1;
        if (LAYOUT == LAYOUT_NARROW) {
            const uint64_t w = t.nodes[q];
            const uint32_t bm = (uint32_t)w;
            if (!((bm >> c) & 1u)) return -1;
            return (int64_t)(((uint32_t)(w >> 32) & 0x7fffffffu) + __builtin_popcount(bm & ((1u << c) - 1u)));
        } else {
            const uint32_t wi = c >> 6, b = c & 63;
            const uint64_t word = t.bm[((size_t)q << t.nw_log2) + wi];
            if (!((word >> b) & 1ull)) return -1;
            const uint64_t meta = t.nodes[q];
            uint32_t r = (uint32_t)meta;
            if (wi) r += (uint32_t)(meta >> (24 + 8 * wi)) & 0xffu;
            return (int64_t)(r + __builtin_popcountll(word & ((1ull << b) - 1ull)));
        }
    }

    // Number of pattern ids on the walk from s; *nterm gets the number of terminal
    // nodes passed.
    __device__ uint32_t count(uint64_t s, uint64_t end, uint32_t *nterm) const {
        int64_t r = root(s, end);
        *nterm = 0;
        if (r < 0) return 0;
        uint32_t q = (uint32_t)r, cnt = 0, nt = 0;
        uint64_t i = s + t.root_depth;
        for (;;) {
            if (is_term(q)) {
                cnt += t.out_first[q + 1] - t.out_first[q];
                nt++;
            }
            if (i >= end) break;
            int64_t nq = child(q, sym(i));
            if (nq < 0) break;
            q = (uint32_t)nq;
            i++;
        }
        *nterm = nt;
        return cnt;
    }

    // Write the cnt keys of start s at keys[o ..), sorted by id.
    __device__ void emit(uint64_t s, uint64_t end, uint64_t *keys, uint64_t o, uint32_t cnt,
                         uint32_t nterm) const {
        int64_t r = root(s, end);
        if (r < 0) return;
        uint32_t q = (uint32_t)r, k = 0;
        uint64_t i = s + t.root_depth;
        const uint64_t hi = s << 32;
        for (;;) {
            if (is_term(q)) {
                for (uint32_t x = t.out_first[q]; x < t.out_first[q + 1]; x++) keys[o + k++] = hi | t.out_ids[x];
                if (k >= cnt) break;
            }
            if (i >= end) break;
            int64_t nq = child(q, sym(i));
            if (nq < 0) break;
            q = (uint32_t)nq;
            i++;
        }
        if (nterm > 1) {  // several nested patterns: merge their (sorted) id lists
            for (uint32_t a = 1; a < cnt; a++) {
                uint64_t v = keys[o + a];
                uint32_t b = a;
                while (b > 0 && keys[o + b - 1] > v) {
                    keys[o + b] = keys[o + b - 1];
                    b--;
                }
                keys[o + b] = v;
            }
        }
    }
};

// End of the packet holding global position s (SEG), by binary search.
__device__ __forceinline__ uint64_t packet_end(const uint64_t *__restrict__ offsets,
                                               uint32_t n_packets, uint64_t s) {
    uint32_t lo = 0, hi = n_packets;  // find first i with offsets[i+1] > s
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (offsets[mid + 1] > s) hi = mid;
        else lo = mid + 1;
    }
    return offsets[lo + 1];
}

// ------------------------------------------------------------------ prefilter keys
// Survivor mask of the 16 starts base + 16*tid + j (j = 0..15) whose first symbols
// pass the LDS test. Byte symbols: x_j = the four bytes at j as a little-endian word.
template <bool PACK2>
__device__ __forceinline__ uint32_t prefilter16(const DevTable &t, const Lds &L, uint32_t lpos) {
    const uint32_t *tw = reinterpret_cast<const uint32_t *>(L.text + lpos);
    uint32_t d[8];
#pragma unroll
    for (int i = 0; i < 8; i++) d[i] = tw[i];
    uint32_t mask = 0;
    if (!PACK2) {
        if (t.filter_k) {
            const uint32_t kmask = t.filter_k >= 4 ? 0xffffffffu : ((1u << (8 * t.filter_k)) - 1u);
            const uint32_t sh = 32 - t.filter_log2;
            const uint32_t *F = L.img + t.filter_word;
#pragma unroll
            for (int j = 0; j < 16; j++) {
                uint32_t x = (j & 3) ? __builtin_amdgcn_alignbyte(d[(j >> 2) + 1], d[j >> 2], j & 3) : d[j >> 2];
                uint32_t h = ((x & kmask) * kFilterMul) >> sh;
                mask |= ((F[h >> 5] >> (h & 31)) & 1u) << j;
            }
        } else {
            // root image as the filter: D-byte key, first byte most significant
#pragma unroll
            for (int j = 0; j < 16; j++) {
                uint32_t x = (j & 3) ? __builtin_amdgcn_alignbyte(d[(j >> 2) + 1], d[j >> 2], j & 3) : d[j >> 2];
                uint32_t key = t.root_depth == 2 ? (((x & 0xffu) << 8) | ((x >> 8) & 0xffu)) : (x & 0xffu);
                mask |= ((L.img[key >> 5] >> (key & 31)) & 1u) << j;
            }
        }
    } else {
        // two-bit codes, first symbol most significant: c[i] holds 4 symbols
        uint32_t code[8];
#pragma unroll
        for (int i = 0; i < 8; i++) {
            uint32_t y = d[i] & 0x03030303u;
            code[i] = ((y & 0xffu) << 6) | ((y >> 4) & 0x30u) | ((y >> 14) & 0x0cu) | (y >> 24);
        }
        const uint32_t c0 = (code[0] << 24) | (code[1] << 16) | (code[2] << 8) | code[3];
        const uint32_t c1 = (code[4] << 24) | (code[5] << 16) | (code[6] << 8) | code[7];
        const uint32_t K = t.filter_k ? t.filter_k : t.root_depth;
        const uint32_t kbits = 2 * K;
        const uint32_t kmask = kbits >= 32 ? 0xffffffffu : ((1u << kbits) - 1u);
        const uint32_t *F = t.filter_k ? L.img + t.filter_word : L.img;
        const uint32_t sh = 32 - t.filter_log2;
#pragma unroll
        for (int j = 0; j < 16; j++) {
            // window of K symbols at j: bits (63-2j) .. (64-2j-2K) of c0:c1
            uint32_t top = j ? __builtin_amdgcn_alignbit(c0, c1, 32 - 2 * j) : c0;  // symbols j..j+15
            uint32_t key = kbits >= 32 ? top : (top >> (32 - kbits)) & kmask;
            uint32_t h = t.filter_k ? (key * kFilterMul) >> sh : key;
            mask |= ((F[h >> 5] >> (h & 31)) & 1u) << j;
        }
    }
    return mask;
}

// ------------------------------------------------------------------------ kernel
template <int LAYOUT, bool PACK2, bool SEG>
__global__ __launch_bounds__(kThreads) void scan_tiled(DevTable t, const uint8_t *__restrict__ text,
                                                      uint64_t n, const uint64_t *__restrict__ offsets,
                                                      uint32_t n_packets, uint64_t *__restrict__ keys,
                                                      uint64_t cap, uint64_t *__restrict__ d_count,
                                                      TileState ts, uint32_t n_tiles) {
    extern __shared__ __align__(16) uint8_t smem[];
    Lds L;
    L.img = reinterpret_cast<uint32_t *>(smem);
    uint8_t *p = smem + ((t.lds_words * 4 + 15) & ~15u);
    L.text = p;
    p += kTile + kHalo + 32;
    L.surv = reinterpret_cast<uint16_t *>(p);
    p += kTile / 8;
    L.hits = reinterpret_cast<uint16_t *>(p);
    p += kTile / 8;
    L.queue = reinterpret_cast<uint16_t *>(p);
    p += kThreads * 2;
    L.red = reinterpret_cast<uint32_t *>(p);
    p += kWaves * 8;
    L.misc = reinterpret_cast<uint32_t *>(p);
    p += 16 * 4;
    L.red64 = reinterpret_cast<uint64_t *>(p);

    const uint32_t tid = threadIdx.x;
    // LDS image (root bitmap, rank, filter), once per workgroup
    for (uint32_t i = tid; i < t.lds_words; i += kThreads) L.img[i] = t.lds_image[i];
    if (tid == 0) {
        L.misc[2] = __hip_atomic_load(&ts.ctrl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        L.misc[0] = __hip_atomic_fetch_add(&ts.ctrl[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const uint32_t epoch = L.misc[2];
    const bool aligned = (((uintptr_t)text) & 15) == 0;
    Walk<LAYOUT, PACK2, SEG> W{t, text, L.img, L.text, 0};

    for (;;) {
        const uint32_t tile = L.misc[0];
        if (tile >= n_tiles) break;
        const uint64_t base = (uint64_t)tile * kTile;
        const uint64_t tile_end = base + kTile < n ? base + kTile : n;
        W.base = base;
        // ---- stage tile + halo into LDS (zero past the end of the text)
        for (uint32_t c = tid; c < (kTile + kHalo + 32) / 16; c += kThreads) {
            const uint64_t g = base + (uint64_t)c * 16;
            uint4 v;
            if (aligned && g + 16 <= n) {
                v = *reinterpret_cast<const uint4 *>(text + g);
            } else {
                uint32_t b[16];
#pragma unroll
                for (int i = 0; i < 16; i++) b[i] = g + i < n ? text[g + i] : 0u;
                v.x = b[0] | (b[1] << 8) | (b[2] << 16) | (b[3] << 24);
                v.y = b[4] | (b[5] << 8) | (b[6] << 16) | (b[7] << 24);
                v.z = b[8] | (b[9] << 8) | (b[10] << 16) | (b[11] << 24);
                v.w = b[12] | (b[13] << 8) | (b[14] << 16) | (b[15] << 24);
            }
            *reinterpret_cast<uint4 *>(L.text + c * 16) = v;
        }
        for (uint32_t i = tid; i < kTile / 16; i += kThreads) L.hits[i] = 0;
        __syncthreads();

        // ---- prefilter: 16 consecutive starts per lane, survivor bitmap in LDS
        for (uint32_t r = 0; r < kTile / (16 * kThreads); r++) {
            const uint32_t e = r * kThreads + tid;   // entry: starts 16e .. 16e+15
            const uint32_t lpos = e * 16;
            uint32_t m = prefilter16<PACK2>(t, L, lpos);
            // starts at or past the tile end, or with too little text left for the
            // shortest pattern, cannot match
            const uint64_t s0 = base + lpos;
            const uint64_t lim = n >= t.min_len ? n - t.min_len + 1 : 0;  // starts < lim
            if (s0 + 16 > lim) m &= s0 >= lim ? 0u : ((1u << (uint32_t)(lim - s0)) - 1u);
            L.surv[e] = (uint16_t)m;
        }
        __syncthreads();

        // ---- walk the survivors, one per lane per batch, in position order
        const uint32_t *sv32 = reinterpret_cast<const uint32_t *>(L.surv);
        uint32_t sw[kTile / 32 / kThreads];
        uint32_t mycnt = 0;
#pragma unroll
        for (uint32_t i = 0; i < kTile / 32 / kThreads; i++) {
            sw[i] = sv32[tid * (kTile / 32 / kThreads) + i];
            mycnt += __builtin_popcount(sw[i]);
        }
        uint32_t nsurv;
        const uint32_t myrank = block_excl_scan(mycnt, &nsurv, L.red);
        uint64_t tile_total = 0;
        for (uint32_t b0 = 0; b0 < nsurv; b0 += kThreads) {
            // write the survivors with rank in [b0, b0 + kThreads) into the queue
            if (myrank < b0 + kThreads && myrank + mycnt > b0) {
                uint32_t rk = myrank;
#pragma unroll
                for (uint32_t i = 0; i < kTile / 32 / kThreads; i++) {
                    uint32_t bits = sw[i];
                    while (bits) {
                        uint32_t j = __builtin_ctz(bits);
                        bits &= bits - 1;
                        if (rk >= b0 && rk < b0 + kThreads)
                            L.queue[rk - b0] = (uint16_t)((tid * (kTile / 32 / kThreads) + i) * 32 + j);
                        rk++;
                    }
                }
            }
            __syncthreads();
            uint64_t c = 0;
            if (b0 + tid < nsurv) {
                const uint32_t ls = L.queue[tid];
                const uint64_t s = base + ls;
                const uint64_t end = SEG ? packet_end(offsets, n_packets, s) : n;
                uint32_t nterm;
                c = W.count(s, end, &nterm);
                if (c) atomicOr(reinterpret_cast<uint32_t *>(L.hits) + (ls >> 5), 1u << (ls & 31));
            }
            tile_total += block_sum64(c, L.red64);  // also orders queue reuse
        }

        // ---- publish the tile's count; find its output offset by decoupled look-back
        if (tid < 64) {
            const uint64_t tagE = (uint64_t)epoch << 44;
            uint64_t excl = 0;
            if (tid == 0) {
                const uint64_t v = tile_total > kValueMask ? kValueMask : tile_total;
                __hip_atomic_store(&ts.word[tile], tagE | ((tile == 0 ? kFlagInc : kFlagAgg) * (1ull << 42)) | v,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                // next ticket now: its latency hides behind the look-back and the emit
                L.misc[1] = __hip_atomic_fetch_add(&ts.ctrl[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (tile > 0) {
                int64_t j = (int64_t)tile - 1;
                uint32_t spins = 0;
                for (;;) {
                    const int64_t idx = j - (int64_t)tid;
                    uint64_t wd = tagE | ((uint64_t)kFlagInc << 42);  // before tile 0: prefix 0
                    if (idx >= 0) wd = __hip_atomic_load(&ts.word[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t flag = (uint32_t)(wd >> 42) & 3u;
                    const bool ready = (wd >> 44) == epoch && flag != 0;
                    const bool isinc = ready && flag == kFlagInc;
                    const uint64_t incm = __ballot(isinc);
                    const uint32_t first = incm ? (uint32_t)__builtin_ctzll(incm) : 64u;
                    const uint64_t need = first >= 63 ? ~0ull : ((2ull << first) - 1ull);
                    const uint64_t notready = __ballot(!ready) & need;
                    if (notready) {
                        if (++spins > kSpinLimit) {  // never expected; report, don't hang
                            if (tid == 0) {
                                __hip_atomic_fetch_or(&ts.ctrl[3], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                            }
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                        continue;
                    }
                    const uint64_t v = (tid <= first) ? (wd & kValueMask) : 0;
                    excl += wave_sum64(v);
                    if (first < 64) break;
                    j -= 64;
                }
                if (tid == 0) {
                    uint64_t inc = excl + tile_total;
                    if (inc > kValueMask) {
                        __hip_atomic_fetch_or(&ts.ctrl[3], 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                        inc = kValueMask;
                    }
                    __hip_atomic_store(&ts.word[tile], tagE | ((uint64_t)kFlagInc << 42) | inc,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            if (tid == 0) L.red64[kWaves] = excl;
        }
        __syncthreads();
        const uint64_t out_base = L.red64[kWaves];

        // ---- emit: matching starts in position order, one per lane per batch
        if (tile_total) {
            const uint32_t *hv = reinterpret_cast<const uint32_t *>(L.hits);
            uint32_t hw[kTile / 32 / kThreads];
            uint32_t hcnt = 0;
#pragma unroll
            for (uint32_t i = 0; i < kTile / 32 / kThreads; i++) {
                hw[i] = hv[tid * (kTile / 32 / kThreads) + i];
                hcnt += __builtin_popcount(hw[i]);
            }
            uint32_t nhits;
            const uint32_t hrank = block_excl_scan(hcnt, &nhits, L.red);
            uint64_t run = out_base;
            for (uint32_t b0 = 0; b0 < nhits; b0 += kThreads) {
                if (hrank < b0 + kThreads && hrank + hcnt > b0) {
                    uint32_t rk = hrank;
#pragma unroll
                    for (uint32_t i = 0; i < kTile / 32 / kThreads; i++) {
                        uint32_t bits = hw[i];
                        while (bits) {
                            uint32_t j = __builtin_ctz(bits);
                            bits &= bits - 1;
                            if (rk >= b0 && rk < b0 + kThreads)
                                L.queue[rk - b0] = (uint16_t)((tid * (kTile / 32 / kThreads) + i) * 32 + j);
                            rk++;
                        }
                    }
                }
                __syncthreads();
                uint32_t c = 0, nterm = 0;
                uint64_t s = 0, end = 0;
                if (b0 + tid < nhits) {
                    s = base + L.queue[tid];
                    end = SEG ? packet_end(offsets, n_packets, s) : n;
                    c = W.count(s, end, &nterm);
                }
                uint32_t btot;
                const uint32_t off = block_excl_scan(c, &btot, L.red);
                if (c && run + off + c <= cap) W.emit(s, end, keys, run + off, c, nterm);
                run += btot;
            }
        }
        __syncthreads();
        if (tid == 0) L.misc[0] = L.misc[1];
        __syncthreads();
    }

    // ---- last workgroup out: writes the count, resets the ticket, advances the epoch
    if (tid == 0) {
        const uint32_t done = __hip_atomic_fetch_add(&ts.ctrl[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (done == gridDim.x - 1) {
            uint64_t total = 0;
            if (n_tiles) {
                // the last tile's inclusive prefix; every tile is published by now, so
                // this wait ends as soon as the word is visible
                const uint64_t want = ((uint64_t)epoch << 44) | ((uint64_t)kFlagInc << 42);
                uint32_t spins = 0;
                for (;;) {
                    const uint64_t wd = __hip_atomic_load(&ts.word[n_tiles - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if ((wd & ~kValueMask) == want) {
                        total = wd & kValueMask;
                        break;
                    }
                    if (++spins > kSpinLimit) {
                        __hip_atomic_fetch_or(&ts.ctrl[3], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // once per launch
            const uint32_t err = __hip_atomic_load(&ts.ctrl[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            *d_count = (err & 1u) ? kCountTimeout : (err & 2u) ? kCountOverflow : total;
            uint32_t ne = epoch + 1;
            if (ne >= (1u << kEpochBits)) ne = 1;
            __hip_atomic_store(&ts.ctrl[3], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ts.ctrl[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ts.ctrl[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ts.ctrl[2], ne, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int LAYOUT, bool PACK2, bool SEG>
int launch_one(const DevTable &t, const uint8_t *text, uint64_t n, const uint64_t *offsets,
               uint32_t n_packets, uint64_t *keys, uint64_t cap, uint64_t *d_count,
               const TileState &ts, uint32_t grid, hipStream_t s) {
    const uint32_t n_tiles = (uint32_t)((n + kTile - 1) / kTile);
    const size_t lds = scan_lds_bytes(t);
    auto k = scan_tiled<LAYOUT, PACK2, SEG>;
    // allow up to the whole 160 KiB of LDS once per kernel (an attribute call per launch
    // costs far more than the launch itself)
    static std::once_flag once;
    std::call_once(once, [&] {
        hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    });
    k<<<grid, kThreads, lds, s>>>(t, text, n, offsets, n_packets, keys, cap, d_count, ts, n_tiles);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

uint32_t scan_grid(const DevTable &t, uint64_t n_tiles) {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (cus <= 0) cus = 256;
    }
    // workgroups per CU: as many as the LDS allows, at most 4 (32 waves)
    const size_t lds = scan_lds_bytes(t);
    uint32_t per_cu = (uint32_t)((160 * 1024) / (lds ? lds : 1));
    if (per_cu < 1) per_cu = 1;
    if (per_cu > 4) per_cu = 4;
    uint64_t g = (uint64_t)cus * per_cu;
    if (g > n_tiles) g = n_tiles;
    return (uint32_t)(g ? g : 1);
}

size_t scan_lds_bytes(const DevTable &t) {
    return ((t.lds_words * 4 + 15) & ~15u) + kTile + kHalo + 32 + kTile / 8 + kTile / 8 +
           kThreads * 2 + kWaves * 8 + 16 * 4 + (kWaves + 1) * 8;
}

int launch_tiled(const DevTable &t, const uint8_t *text, uint64_t n, const uint64_t *offsets,
                 uint32_t n_packets, uint64_t *keys, uint64_t cap, uint64_t *d_count,
                 const TileState &ts, uint32_t grid, hipStream_t s) {
    const bool seg = offsets != nullptr;
    const bool narrow = t.layout == LAYOUT_NARROW;
    const bool pack2 = t.pack2 != 0;
#define PFAC_L(LA, P2, SG) return launch_one<LA, P2, SG>(t, text, n, offsets, n_packets, keys, cap, d_count, ts, grid, s)
    if (narrow) {
        if (pack2) { if (seg) PFAC_L(LAYOUT_NARROW, true, true); else PFAC_L(LAYOUT_NARROW, true, false); }
        else { if (seg) PFAC_L(LAYOUT_NARROW, false, true); else PFAC_L(LAYOUT_NARROW, false, false); }
    } else {
        if (seg) PFAC_L(LAYOUT_WIDE, false, true);
        PFAC_L(LAYOUT_WIDE, false, false);
    }
#undef PFAC_L
}

}  // namespace pfac
