// Streaming failure-less scan for gfx950: one persistent kernel per scan, every wave on
// its own.
//
// The method is Section 2.3's: every start position walks the goto-only trie until a
// transition is missing, and reports every pattern whose final state it reaches; nodes
// are found with Eq. 1. What is particular to this GPU is how positions reach the walk.
//
//  * Spans. Each wavefront takes kSpan-byte spans of the text in increasing order from
//    an atomic ticket and streams them in 1 KiB steps: 64 lanes x 16 bytes, one 16-byte
//    load per lane, the next steps' loads already in flight. No workgroup barrier is
//    used after the LDS image is loaded, so the waves of a CU overlap each other's
//    memory latency freely.
//  * LDS prefilter. No pattern is shorter than min_len, so a start can only match if its
//    first k = min(min_len, kmax) symbols begin some pattern. Each lane tests its 16
//    starts against an LDS bitmap: a blocked Bloom filter (two bits of one 32-bit word
//    per k-gram), or the root image itself. A clear bit proves there is no match there;
//    a set bit sends the start to the walk, which decides exactly.
//  * Root image. The top D trie levels are folded into one direct-indexed bitmap over
//    D-symbol keys (lexicographic), with a rank per 32-bit word: the rank of a key is
//    its depth-D node's breadth-first index minus the first depth-D index, i.e. Eq. 1's
//    popcount rule applied to a D-symbol root. Walks start at that node.
//  * Survivors go to a wave-private LDS queue in position order and are walked 64 at a
//    time, one per lane, so the dependent node loads of a walk are paid once per 64
//    survivors. Walks read nodes and text through L2.
//  * Output. A span's match count is published and its output offset found by
//    decoupled look-back over earlier spans (one 64-bit word per span, relaxed atomics).
//    Starts that matched were kept in a wave-private hit queue in position order; they
//    are walked again and their keys written at their final place, so the output is
//    sorted by (start, id) with no global sort. When a span has more matching starts
//    than the hit queue holds, the rest of the span is streamed again in emit mode.
#include <mutex>

#include "kernels.h"
#include "pfac_impl.h"
#include "scan_internal.h"

namespace pfac {
namespace {

constexpr uint64_t kFlagAgg = 1, kFlagInc = 2;
constexpr uint32_t kSpinLimit = 1u << 24;
constexpr uint32_t kNone = 0xffffffffu;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t bcast(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Inclusive prefix sum over the wave.
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

// ------------------------------------------------------------------------ the walk
template <int LAYOUT, bool PACK2, bool SEG>
struct Walk {
    const DevTable &t;
    const uint8_t *__restrict__ text;
    const uint32_t *img;  // LDS image

    // Node reached from the root image by the D symbols at s, or -1.
    __device__ __forceinline__ int64_t root(uint64_t s, uint64_t end) const {
        const uint32_t D = t.root_depth;
        if (s + D > end) return -1;
        uint32_t key = 0;
        if (PACK2) {
            for (uint32_t i = 0; i < D; i++) {
                uint32_t c = text[s + i];
                if (c > 3) return -1;  // a byte outside the 2-bit code space
                key = (key << 2) | c;
            }
        } else {
            for (uint32_t i = 0; i < D; i++) key = (key << 8) | text[s + i];
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

    // Pattern ids on the walk from s (every terminal passed); *nterm = terminals passed.
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
            int64_t nq = child(q, text[i]);
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
            int64_t nq = child(q, text[i]);
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

// End of the packet holding global position s (packet batches), by binary search.
__device__ __forceinline__ uint64_t packet_end(const uint64_t *__restrict__ offsets,
                                               uint32_t n_packets, uint64_t s) {
    uint32_t lo = 0, hi = n_packets;  // first i with offsets[i+1] > s
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (offsets[mid + 1] > s) hi = mid;
        else lo = mid + 1;
    }
    return offsets[lo + 1];
}

// 16 bytes at p (zero past n); vector load when it is whole and aligned.
__device__ __forceinline__ uint4 load16(const uint8_t *__restrict__ text, uint64_t p, uint64_t n, bool aligned) {
    uint4 v;
    if (aligned && p + 16 <= n) {
        v = *reinterpret_cast<const uint4 *>(text + p);
    } else {
        uint32_t b[16];
#pragma unroll
        for (int i = 0; i < 16; i++) b[i] = p + i < n ? text[p + i] : 0u;
        v.x = b[0] | (b[1] << 8) | (b[2] << 16) | (b[3] << 24);
        v.y = b[4] | (b[5] << 8) | (b[6] << 16) | (b[7] << 24);
        v.z = b[8] | (b[9] << 8) | (b[10] << 16) | (b[11] << 24);
        v.w = b[12] | (b[13] << 8) | (b[14] << 16) | (b[15] << 24);
    }
    return v;
}

// Two-bit codes of 16 bytes, first byte in the top bits.
__device__ __forceinline__ uint32_t pack2x16(uint4 v) {
    uint32_t d[4] = {v.x, v.y, v.z, v.w};
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        uint32_t y = d[i] & 0x03030303u;
        uint32_t code = ((y & 0xffu) << 6) | ((y >> 4) & 0x30u) | ((y >> 14) & 0x0cu) | (y >> 24);
        c = (c << 8) | code;
    }
    return c;
}

// LDS test of one prefilter key in the blocked Bloom filter: two bits of one word.
__device__ __forceinline__ uint32_t bloom2(const uint32_t *F, uint32_t key, uint32_t wshift) {
    const uint32_t h = key * kFilterMul;
    const uint32_t w = F[h >> wshift];
    return (w >> ((h >> 6) & 31)) & (w >> ((h >> 11) & 31)) & 1u;
}

// Survivor mask of this lane's 16 starts (bit j = start 16*lane + j of the step).
// cur: this lane's 16 bytes; next_d0: the 4 bytes after them; c0/c1: two-bit codes of
// this lane's and the next 16 bytes.
template <bool PACK2>
__device__ __forceinline__ uint32_t prefilter16(const DevTable &t, const uint32_t *img, uint4 cur,
                                                uint32_t next_d0, uint32_t c0, uint32_t c1) {
    uint32_t mask = 0;
    if (!PACK2) {
        const uint32_t d[5] = {cur.x, cur.y, cur.z, cur.w, next_d0};
        if (t.filter_k) {
            const uint32_t kmask = t.filter_k >= 4 ? 0xffffffffu : ((1u << (8 * t.filter_k)) - 1u);
            const uint32_t wshift = 37 - t.filter_log2;
            const uint32_t *F = img + t.filter_word;
#pragma unroll
            for (int j = 0; j < 16; j++) {
                uint32_t x = (j & 3) ? __builtin_amdgcn_alignbyte(d[(j >> 2) + 1], d[j >> 2], j & 3) : d[j >> 2];
                mask |= bloom2(F, x & kmask, wshift) << j;
            }
        } else {
            // root image as the filter: D-byte key, first byte most significant
            const bool two = t.root_depth == 2;
#pragma unroll
            for (int j = 0; j < 16; j++) {
                uint32_t x = (j & 3) ? __builtin_amdgcn_alignbyte(d[(j >> 2) + 1], d[j >> 2], j & 3) : d[j >> 2];
                uint32_t key = two ? (((x & 0xffu) << 8) | ((x >> 8) & 0xffu)) : (x & 0xffu);
                mask |= ((img[key >> 5] >> (key & 31)) & 1u) << j;
            }
        }
    } else {
        const uint32_t K = t.filter_k ? t.filter_k : t.root_depth;
        const uint32_t kbits = 2 * K;
        const uint32_t kmask = kbits >= 32 ? 0xffffffffu : ((1u << kbits) - 1u);
        const uint32_t rs = kbits >= 32 ? 0 : 32 - kbits;
        if (t.filter_k) {
            const uint32_t wshift = 37 - t.filter_log2;
            const uint32_t *F = img + t.filter_word;
#pragma unroll
            for (int j = 0; j < 16; j++) {
                uint32_t top = j ? __builtin_amdgcn_alignbit(c0, c1, 32 - 2 * j) : c0;  // symbols j..j+15
                mask |= bloom2(F, (top >> rs) & kmask, wshift) << j;
            }
        } else {
#pragma unroll
            for (int j = 0; j < 16; j++) {
                uint32_t top = j ? __builtin_amdgcn_alignbit(c0, c1, 32 - 2 * j) : c0;
                uint32_t key = (top >> rs) & kmask;
                mask |= ((img[key >> 5] >> (key & 31)) & 1u) << j;
            }
        }
    }
    return mask;
}

enum Mode { kCount = 0, kEmit = 1 };

// Per-wave state of one span (wave-uniform values).
struct SpanState {
    uint64_t a;          // first byte of the span
    uint32_t qlen;       // survivors queued
    uint32_t nh;         // hits stored
    uint32_t ovf;        // span-local start of the first hit not stored, or kNone
    uint64_t my_cnt;     // this lane's share of the span's match count
    uint64_t run;        // emit: output index of the next key
};

template <int LAYOUT, bool PACK2, bool SEG>
struct Scanner {
    const DevTable &t;
    Walk<LAYOUT, PACK2, SEG> W;
    const uint8_t *__restrict__ text;
    uint64_t n, lim;  // starts >= lim cannot match (too little text left)
    const uint64_t *__restrict__ offsets;
    uint32_t n_packets;
    uint64_t *__restrict__ keys;
    uint64_t cap;
    uint16_t *q;   // survivor queue (span-local starts), kQCap entries
    uint16_t *hq;  // hit queue, kHCap entries
    bool aligned;

    __device__ __forceinline__ uint64_t end_of(uint64_t s) const {
        return SEG ? packet_end(offsets, n_packets, s) : n;
    }

    // Walk `cnt` queued survivors from q[first], one per lane.
    template <int MODE>
    __device__ void walk_batch(SpanState &S, uint32_t first, uint32_t cnt) {
        const uint32_t lane = lane_id();
        const bool on = lane < cnt;
        const uint32_t sl = on ? q[first + lane] : 0u;
        const uint64_t s = S.a + sl;
        uint32_t c = 0, nterm = 0;
        uint64_t end = 0;
        if (on) {
            end = end_of(s);
            c = W.count(s, end, &nterm);
        }
        if (MODE == kCount) {
            S.my_cnt += c;
            const uint64_t hb = __ballot(c > 0);
            if (hb && S.ovf == kNone) {
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(hb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)hb, 0u));
                const bool store = c > 0 && S.nh + rank < kHCap;
                if (store) hq[S.nh + rank] = (uint16_t)sl;
                const uint64_t lost = __ballot(c > 0 && !store);
                if (lost) S.ovf = bcast(__shfl(sl, (int)__builtin_ctzll(lost), 64));
                const uint32_t nh = S.nh + (uint32_t)__builtin_popcountll(hb);
                S.nh = nh < kHCap ? nh : kHCap;
            }
        } else {
            const uint32_t inc = wave_incl_scan(c);
            const uint32_t tot = __shfl(inc, 63, 64);
            const uint64_t o = S.run + inc - c;
            if (c && o + c <= cap) W.emit(s, end, keys, o, c, nterm);
            S.run += tot;
        }
    }

    // Stream starts [lo, hi) of the span (lo >= S.a); survivors are walked in MODE.
    template <int MODE>
    __device__ void stream(SpanState &S, uint64_t lo, uint64_t hi) {
        const uint32_t lane = lane_id();
        uint64_t step = lo & ~(uint64_t)(kStep - 1);
        uint4 cur = load16(text, step + 16 * lane, n, aligned);
        uint4 nx1 = load16(text, step + kStep + 16 * lane, n, aligned);
        uint32_t pc = PACK2 ? pack2x16(cur) : 0u;
        const uint64_t top = hi < lim ? hi : lim;
        for (; step < hi; step += kStep) {
            const uint4 nx2 = load16(text, step + 2 * kStep + 16 * lane, n, aligned);
            // bytes just after this lane's 16: the next lane's, or the next step's lane 0
            const uint32_t dn = __shfl_down(cur.x, 1, 64);
            const uint32_t d0n = bcast(__shfl(nx1.x, 0, 64));
            const uint32_t next_d0 = lane == 63 ? d0n : dn;
            uint32_t pn = 0, c1 = 0;
            if (PACK2) {
                pn = pack2x16(nx1);
                const uint32_t cn = __shfl_down(pc, 1, 64);
                const uint32_t p0n = bcast(__shfl(pn, 0, 64));
                c1 = lane == 63 ? p0n : cn;
            }
            uint32_t m = prefilter16<PACK2>(t, W.img, cur, next_d0, pc, c1);
            // keep starts in [lo, min(hi, lim))
            const uint64_t s0 = step + 16 * lane;
            if (s0 + 16 > top) m &= s0 >= top ? 0u : ((1u << (uint32_t)(top - s0)) - 1u);
            if (s0 < lo) m &= lo >= s0 + 16 ? 0u : ~((1u << (uint32_t)(lo - s0)) - 1u);
            if (__ballot(m != 0)) {
                const uint32_t c = __builtin_popcount(m);
                const uint32_t inc = wave_incl_scan(c);
                const uint32_t tot = bcast(__shfl(inc, 63, 64));
                uint32_t at = S.qlen + inc - c;
                const uint32_t base_local = (uint32_t)(s0 - S.a);
                while (m) {
                    const uint32_t j = __builtin_ctz(m);
                    m &= m - 1;
                    q[at++] = (uint16_t)(base_local + j);
                }
                S.qlen += tot;
                __builtin_amdgcn_wave_barrier();
                if (S.qlen >= 64) {
                    uint32_t done = 0;
                    while (S.qlen - done >= 64) {
                        walk_batch<MODE>(S, done, 64);
                        done += 64;
                    }
                    const uint32_t rest = S.qlen - done;
                    const uint16_t v = lane < rest ? q[done + lane] : 0;
                    __builtin_amdgcn_wave_barrier();
                    if (lane < rest) q[lane] = v;
                    __builtin_amdgcn_wave_barrier();
                    S.qlen = rest;
                }
            }
            cur = nx1;
            nx1 = nx2;
            pc = pn;
        }
        if (S.qlen) {
            walk_batch<MODE>(S, 0, S.qlen);
            S.qlen = 0;
        }
    }
};

// ------------------------------------------------------------------------ kernel
template <int LAYOUT, bool PACK2, bool SEG>
__global__ __launch_bounds__(kThreads) void scan_stream(DevTable t, const uint8_t *__restrict__ text,
                                                       uint64_t n, const uint64_t *__restrict__ offsets,
                                                       uint32_t n_packets, uint64_t *__restrict__ keys,
                                                       uint64_t cap, uint64_t *__restrict__ d_count,
                                                       TileState ts, uint32_t n_spans) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint32_t *img = reinterpret_cast<uint32_t *>(smem);
    for (uint32_t i = threadIdx.x; i < t.lds_words; i += kThreads) img[i] = t.lds_image[i];
    __syncthreads();  // the only workgroup barrier: waves run independently from here

    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    uint16_t *wq = reinterpret_cast<uint16_t *>(smem + image_bytes(t) + wave * kWaveLds);
    Scanner<LAYOUT, PACK2, SEG> sc{t, {t, text, img}, text, n,
                                   n >= t.min_len ? n - t.min_len + 1 : 0,
                                   offsets, n_packets, keys, cap, wq, wq + kQCap,
                                   (((uintptr_t)text) & 15) == 0};
    uint32_t epoch = 0;
    if (lane == 0) epoch = __hip_atomic_load(&ts.ctrl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    epoch = bcast(epoch);
    const uint64_t tagE = (uint64_t)epoch << 44;

    for (;;) {
        uint32_t span = 0;
        if (lane == 0) span = __hip_atomic_fetch_add(&ts.ctrl[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        span = bcast(span);
        if (span >= n_spans) break;
        SpanState S{(uint64_t)span * kSpan, 0, 0, kNone, 0, 0};
        const uint64_t b = S.a + kSpan < n ? S.a + kSpan : n;
        sc.template stream<kCount>(S, S.a, b);
        const uint64_t total = wave_sum64(S.my_cnt);

        // publish the span's count; find its output offset by decoupled look-back
        if (lane == 0) {
            const uint64_t v = total > kValueMask ? kValueMask : total;
            __hip_atomic_store(&ts.word[span], tagE | ((span == 0 ? kFlagInc : kFlagAgg) << 42) | v,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        uint64_t excl = 0;
        if (span > 0) {
            int64_t j = (int64_t)span - 1;
            uint32_t spins = 0;
            for (;;) {
                const int64_t idx = j - (int64_t)lane;
                uint64_t wd = tagE | (kFlagInc << 42);  // before span 0: prefix 0
                if (idx >= 0) wd = __hip_atomic_load(&ts.word[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t flag = (uint32_t)(wd >> 42) & 3u;
                const bool ready = (wd >> 44) == epoch && flag != 0;
                const bool isinc = ready && flag == kFlagInc;
                const uint64_t incm = __ballot(isinc);
                const uint32_t first = incm ? (uint32_t)__builtin_ctzll(incm) : 64u;
                const uint64_t need = first >= 63 ? ~0ull : ((2ull << first) - 1ull);
                if (__ballot(!ready) & need) {
                    if (++spins > kSpinLimit) {  // never expected; report, don't hang
                        if (lane == 0) {
                            __hip_atomic_fetch_or(&ts.ctrl[3], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                        }
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += wave_sum64(lane <= first ? (wd & kValueMask) : 0);
                if (first < 64) break;
                j -= 64;
            }
            if (lane == 0) {
                uint64_t inc = excl + total;
                if (inc > kValueMask) {
                    __hip_atomic_fetch_or(&ts.ctrl[3], 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    inc = kValueMask;
                }
                __hip_atomic_store(&ts.word[span], tagE | (kFlagInc << 42) | inc, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
        }

        // emit: stored hits in position order, then (if the hit queue overflowed) the
        // rest of the span streamed again in emit mode
        if (total) {
            S.run = excl;
            for (uint32_t h0 = 0; h0 < S.nh; h0 += 64) {
                const uint32_t cnt = S.nh - h0 < 64 ? S.nh - h0 : 64;
                // walk_batch reads its starts from q: move this batch of hits there
                const uint16_t v = lane < cnt ? sc.hq[h0 + lane] : 0;
                __builtin_amdgcn_wave_barrier();
                if (lane < cnt) sc.q[lane] = v;
                __builtin_amdgcn_wave_barrier();
                sc.template walk_batch<kEmit>(S, 0, cnt);
                __builtin_amdgcn_wave_barrier();
            }
            if (S.ovf != kNone) sc.template stream<kEmit>(S, S.a + S.ovf, b);
        }
    }

    // last wave out: writes the count, resets the ticket, advances the epoch
    if (lane == 0) {
        const uint32_t waves = gridDim.x * (kThreads / 64);
        const uint32_t done = __hip_atomic_fetch_add(&ts.ctrl[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (done == waves - 1) {
            uint64_t total = 0;
            if (n_spans) {
                // the last span's inclusive prefix: every span is published by now, so
                // this wait ends as soon as the word is visible
                const uint64_t want = tagE | (kFlagInc << 42);
                uint32_t spins = 0;
                for (;;) {
                    const uint64_t wd = __hip_atomic_load(&ts.word[n_spans - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    const uint32_t n_spans = (uint32_t)((n + kSpan - 1) / kSpan);
    const size_t lds = scan_lds_bytes(t);
    auto k = scan_stream<LAYOUT, PACK2, SEG>;
    // allow up to the whole 160 KiB of LDS, once per kernel (an attribute call per launch
    // costs far more than the launch itself)
    static std::once_flag once;
    static int cus = 0;
    std::call_once(once, [&] {
        (void)hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        int dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (cus <= 0) cus = 256;
    });
    if (grid == 0) {
        // as many workgroups as can be resident at once, and no more than it takes to
        // give every wave a span
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kThreads, lds) != hipSuccess || per_cu < 1)
            per_cu = 1;
        uint64_t g = (uint64_t)cus * (uint32_t)per_cu;
        const uint64_t need = (n_spans + kWaves - 1) / kWaves;
        grid = (uint32_t)(g < need ? g : need);
        if (grid == 0) grid = 1;
    }
    k<<<grid, kThreads, lds, s>>>(t, text, n, offsets, n_packets, keys, cap, d_count, ts, n_spans);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace

size_t scan_lds_bytes(const DevTable &t) { return image_bytes(t) + (size_t)kWaves * kWaveLds; }

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
