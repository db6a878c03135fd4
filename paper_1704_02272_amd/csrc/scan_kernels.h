// Failure-less scan for gfx950: a streaming count kernel and a placement kernel.
// (Device code; instantiated for the plain trie in kernels_scan.hip and for the
// compressed trie of Section 3.2 in kernels_scan_merged.hip.)
//
// The method is Section 2.3's: every start position walks the goto-only trie until a
// transition is missing, and reports every pattern whose final state it reaches; nodes
// are found with Eq. 1. What is particular to this GPU is how positions reach the walk
// and how the matches reach their place in the output.
//
// Count kernel (scan_count), one persistent wave per span at a time, no wave ever
// waiting on another:
//  * Spans. The text is cut into spans of 2^span_log2 bytes (2-64 KiB, a tuning choice);
//    wave g of G takes spans g, g+G, ... and streams each in 2 KiB steps: 64 lanes x 32
//    bytes, two 16-byte buffer loads per lane, the next two steps' loads in flight.
//  * LDS prefilter. No pattern is shorter than min_len, so a start can only match if its
//    first symbols begin some pattern. Bytes with every pattern four or longer take the
//    sampled form: every second start is probed with its 3-gram (a pattern starting
//    there or one byte earlier has that 3-gram at offset 0 or 1), and the lane holding
//    the bytes of a start that passes checks its 4-grams against a two-probe 4-gram
//    filter. Other sets probe every start's k-gram in a
//    two-probe Bloom filter, or the root image itself. A clear bit proves there is no
//    match there; a start that passes is walked, which decides exactly.
//  * Root image. The top D trie levels are folded into one direct-indexed bitmap over
//    D-symbol keys (lexicographic), with a rank per 32-bit word: the rank of a key is
//    its depth-D node's breadth-first index minus the first depth-D index, i.e. Eq. 1's
//    popcount rule applied to a D-symbol root. Walks start at that node.
//  * Survivors go to a wave-private LDS queue in position order and are walked 64 at a
//    time, one per lane, mostly at the end of the span so walks seldom stall the stream
//    of text loads. Walks read nodes and text through L2.
//  * Per span the kernel stores the match count and one record per matching start
//    (start, and the id, or the first terminal node, or nothing), up to span / 64
//    records (at least 256).
//
// Placement kernel (place_emit): blocks of kBlockSpans spans. A block finds its output
// offset (the matches of all spans before it: summed by the block itself up to
// kDirectMaxSpans spans, else by decoupled look-back over earlier blocks taken by
// ticket) and writes every match key at its final place from the records, so the output
// is sorted by (start, id) with no global sort. A start that passed several terminals,
// and any start of a span with more matching starts than records, is walked again in
// HBM.
#pragma once
#include <mutex>

#include "kernels.h"
#include "pfac_impl.h"
#include "scan_internal.h"

namespace pfac {
namespace {

constexpr uint64_t kFlagAgg = 1, kFlagInc = 2;
// Bound on any device-side wait, in ticks of the 100 MHz real-time counter (2 s).
constexpr uint64_t kWaitTicks = 200000000ull;
constexpr uint32_t kNone = 0xffffffffu;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t bcast(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// DPP lane moves (register to register, no LDS round trip). Lanes with no source keep 0.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143, kDppWaveShl1 = 0x130;

// Inclusive prefix sum over the wave: shifts within each 16-lane row, then the row
// totals carried into the rows above.
// The row shifts read 0 where the source lane is outside the row (bound control), so
// they need no zeroed register and fold into the adds.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppRowShr1, 0xf, 0xf, true);
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppRowShr2, 0xf, 0xf, true);
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppRowShr4, 0xf, 0xf, true);
    v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, kDppRowShr8, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0u, v, kDppRowBcast15, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0u, v, kDppRowBcast31, 0xc, 0xf, false);
    return v;
}

// (m << 2) | b as one instruction: written out so the compiler keeps one shift-or per
// bit instead of regrouping the chain into separate shifts and three-way ors.
__device__ __forceinline__ uint32_t shl2_or(uint32_t m, uint32_t b) {
    uint32_t r;
    asm("v_lshl_or_b32 %0, %1, 2, %2" : "=v"(r) : "v"(m), "v"(b));
    return r;
}

// Value of lane + 1 (lane 63 gets 0).
__device__ __forceinline__ uint32_t from_next_lane(uint32_t v) {
    return __builtin_amdgcn_update_dpp(0u, v, kDppWaveShl1, 0xf, 0xf, false);
}

// 64-bit forms: the same lane moves on both halves, then a 64-bit add.
__device__ __forceinline__ uint64_t dpp_pair(uint64_t v, uint32_t lo_moved, uint32_t hi_moved) {
    return v + (((uint64_t)hi_moved << 32) | lo_moved);
}
#define PFAC_DPP64(v, ctrl, rm)                                                                          \
    dpp_pair(v, __builtin_amdgcn_update_dpp(0u, (uint32_t)(v), ctrl, rm, 0xf, false),                  \
             __builtin_amdgcn_update_dpp(0u, (uint32_t)((v) >> 32), ctrl, rm, 0xf, false))
__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v) {
    v = PFAC_DPP64(v, kDppRowShr1, 0xf);
    v = PFAC_DPP64(v, kDppRowShr2, 0xf);
    v = PFAC_DPP64(v, kDppRowShr4, 0xf);
    v = PFAC_DPP64(v, kDppRowShr8, 0xf);
    v = PFAC_DPP64(v, kDppRowBcast15, 0xa);
    v = PFAC_DPP64(v, kDppRowBcast31, 0xc);
    return v;
}
#undef PFAC_DPP64

// Sum over the wave, in every lane.
__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
    const uint64_t s = wave_incl_scan64(v);
    return ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(s >> 32), 63) << 32) |
           __builtin_amdgcn_readlane((uint32_t)s, 63);
}

// ------------------------------------------------------------------------ the walk
// Result of one walk: how many pattern ids it passed, how many terminals, the first one.
// A walk's pattern-id count, the number of terminals it passed, and the ids of the first
// one: out_ids[f0 .. f0 + k0) (id0 = out_ids[f0] when k0 == 1).
struct WalkResult {
    uint32_t cnt, nterm, f0, k0, id0, q0, d0;  // q0, d0: node and depth of the first terminal
    uint32_t k1, id1;                          // second terminal: its id count, its id when one
};

// Where a walk over a compressed table (Section 3.2) stands for the ids: the last record
// below shared_base it passed and the sum of rank words added since (see reduce.cpp).
// The plain trie keeps ids per node and never reads it.
struct RankState {
    uint32_t u, add;
};

template <int LAYOUT, bool MERGED>
struct Trie {
    const DevTable &t;

    __device__ __forceinline__ bool is_term(uint32_t q) const { return (t.nodes[q] >> 63) != 0; }
    // Index of terminal q's ids in out_first: q itself, or for a compressed table the
    // rank of the string the walk spelled.
    __device__ __forceinline__ uint32_t id_index(uint32_t q, const RankState &rs) const {
        if (!MERGED) return q;
        return q < t.shared_base ? t.rk[q] : t.rk[rs.u] + rs.add;
    }

    // Child of q on c (Eq. 1), or -1.
    __device__ __forceinline__ int64_t child(uint32_t q, uint32_t c) const {
        if (c >= t.alphabet) return -1;
        if (LAYOUT == LAYOUT_NARROW) {
            const uint64_t w = t.nodes[q];
            const uint32_t bm = (uint32_t)w;
            if (!((bm >> c) & 1u)) return -1;
            return (int64_t)(((uint32_t)(w >> 32) & kNarrowIndexMask) + __builtin_popcount(bm & ((1u << c) - 1u)));
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

    // Plain table: the node word's tail flag, its first-child (or tail) index, and the
    // child of q on c from its word w already loaded (Eq. 1), or -1.
    __device__ __forceinline__ static bool w_tail(uint64_t w) { return (w & kTailBit) != 0; }
    __device__ __forceinline__ static uint32_t w_index(uint64_t w) {
        return LAYOUT == LAYOUT_NARROW ? (uint32_t)(w >> 32) & kNarrowIndexMask : (uint32_t)w;
    }
    __device__ __forceinline__ int64_t child_w(uint32_t q, uint64_t w, uint32_t c) const {
        if (c >= t.alphabet) return -1;
        if (LAYOUT == LAYOUT_NARROW) {
            const uint32_t bm = (uint32_t)w;
            if (!((bm >> c) & 1u)) return -1;
            return (int64_t)(w_index(w) + __builtin_popcount(bm & ((1u << c) - 1u)));
        } else {
            const uint32_t wi = c >> 6, b = c & 63;
            const uint64_t word = t.bm[((size_t)q << t.nw_log2) + wi];
            if (!((word >> b) & 1ull)) return -1;
            uint32_t r = (uint32_t)w;
            if (wi) r += (uint32_t)(w >> (24 + 8 * wi)) & 0xffu;
            return (int64_t)(r + __builtin_popcountll(word & ((1ull << b) - 1ull)));
        }
    }
    // Plain table: tail records {offset in tail_bytes, length, first id index, id count},
    // read by tail_match.

    // Plain table: ids of terminal q (word w): the count, and the first id (one = true:
    // read from the word) or the index of the ids in out_ids.
    __device__ __forceinline__ uint32_t term_ids(uint32_t q, uint64_t w, uint32_t &fi, bool &one) const {
        if (LAYOUT == LAYOUT_NARROW && t.alphabet <= 4 && (w & kOneIdBit)) {
            fi = (uint32_t)w >> kOneIdShift;
            one = true;
            return 1;
        }
        fi = t.out_first[q];
        one = false;
        return t.out_first[q + 1] - fi;
    }

    // Compressed table: path tail of q: x = offset in tail_bytes, y = length (0: none),
    // z = end record.
    __device__ __forceinline__ uint4 tail(uint32_t q) const { return reinterpret_cast<const uint4 *>(t.tails)[q]; }

    // Whether text[i .. i+len) spells tail_bytes[off .. off+len). Both runs are read as
    // aligned dwords (5 per side per 16 bytes, all issued before any compare) and lined
    // up with alignbyte. Only dwords that hold at least one compared byte are loaded, so
    // no load leaves the page of a byte inside the runs.
    __device__ __forceinline__ bool tail_equal(const uint8_t *__restrict__ text, uint64_t i, uint32_t off,
                                               uint32_t len) const {
        const uintptr_t ta = (uintptr_t)(text + i), pa = (uintptr_t)(t.tail_bytes + off);
        const uint32_t *tw = reinterpret_cast<const uint32_t *>(ta & ~(uintptr_t)3);
        const uint32_t *pw = reinterpret_cast<const uint32_t *>(pa & ~(uintptr_t)3);
        const uint32_t ts = (uint32_t)(ta & 3), ps = (uint32_t)(pa & 3);
        const uint32_t nt = (ts + len + 3) >> 2, np = (ps + len + 3) >> 2;  // dwords holding compared bytes
        for (uint32_t o = 0; o < len; o += 16) {
            const uint32_t k0 = o >> 2;  // dword of byte o on both sides (o is a multiple of 16)
            uint32_t x[5], y[5];
#pragma unroll
            for (uint32_t k = 0; k < 5; k++) {
                x[k] = k0 + k < nt ? tw[k0 + k] : 0u;
                y[k] = k0 + k < np ? pw[k0 + k] : 0u;
            }
            uint32_t diff = 0;
#pragma unroll
            for (uint32_t k = 0; k < 4; k++) {
                const uint32_t b = o + 4 * k;  // first compared byte of this group
                if (b < len) {
                    const uint32_t m = b + 4 <= len ? 0xffffffffu : (1u << (8 * (len - b))) - 1u;
                    const uint32_t xt = __builtin_amdgcn_alignbyte(x[k + 1], x[k], ts);
                    const uint32_t yp = __builtin_amdgcn_alignbyte(y[k + 1], y[k], ps);
                    diff |= (xt ^ yp) & m;
                }
            }
            if (diff) return false;
        }
        return true;
    }

    // Plain table, at the tail head whose word is w and text position i (end exclusive):
    // whether the text from i spells the head's path, with its record in tr. The record,
    // the copy of the path's first kHeadBytes bytes kept beside it and the text dwords
    // those bytes cover (never past end) are all loaded before any compare, so the walk
    // pays one memory round trip here; a longer path compares the rest after.
    __device__ __forceinline__ bool tail_match(uint64_t w, const uint8_t *__restrict__ text, uint64_t i,
                                               uint64_t end, uint4 &tr) const {
        static_assert(kHeadBytes == 16, "one 16-byte load of path bytes");
        const uint32_t x = w_index(w);
        tr = reinterpret_cast<const uint4 *>(t.tails)[x];
        const uint4 h0 = t.tail_head[x];
        const uint64_t lim = i + kHeadBytes < end ? i + kHeadBytes : end;
        const uintptr_t ta = (uintptr_t)(text + i);
        const uint32_t *tw = reinterpret_cast<const uint32_t *>(ta & ~(uintptr_t)3);
        const uint32_t ts = (uint32_t)(ta & 3);
        const uint32_t nt = (uint32_t)((ts + (lim - i) + 3) >> 2);  // dwords holding text bytes below lim
        uint32_t xw[kHeadBytes / 4 + 1];
#pragma unroll
        for (uint32_t k = 0; k <= kHeadBytes / 4; k++) xw[k] = k < nt ? tw[k] : 0u;
        if (i + tr.y > end) return false;
        const uint32_t len = tr.y, hl = len < kHeadBytes ? len : kHeadBytes;
        const uint32_t pw[kHeadBytes / 4] = {h0.x, h0.y, h0.z, h0.w};
        uint32_t diff = 0;
#pragma unroll
        for (uint32_t g = 0; g < kHeadBytes / 4; g++) {
            const uint32_t b = 4 * g;  // first compared byte of this group
            if (b < hl) {
                const uint32_t m = b + 4 <= hl ? 0xffffffffu : (1u << (8 * (hl - b))) - 1u;
                diff |= (__builtin_amdgcn_alignbyte(xw[g + 1], xw[g], ts) ^ pw[g]) & m;
            }
        }
        if (diff) return false;
        return len <= kHeadBytes || tail_equal(text, i + kHeadBytes, tr.x + kHeadBytes, len - kHeadBytes);
    }

    // One move of a walk at node q, text position i < end: the next symbol by Eq. 1, and
    // when q has a path tail and that symbol starts it, the rest of the tail at once. A
    // mismatch on the first symbol thus costs no more than a plain step. False when the
    // walk ends here.
    // qterm: whether q is terminal (a compressed table's rank counts it).
    __device__ __forceinline__ bool advance(uint32_t &q, uint64_t &i, uint4 tl, const uint8_t *__restrict__ text,
                                            uint32_t c, uint64_t end, RankState &rs, bool qterm) const {
        const int64_t nq = child(q, c);
        if (nq < 0) return false;
        if (MERGED) {
            // into a shared record: add what sorts before it; the rest of a path tail adds
            // nothing (one child each, no terminal before its end)
            if ((uint32_t)nq < t.shared_base) rs.u = (uint32_t)nq;
            else rs.add += (qterm ? 1u : 0u) + t.rk[nq];
        }
        if (tl.y > 1) {
            if (i + tl.y > end || !tail_equal(text, i + 1, tl.x + 1, tl.y - 1)) return false;
            q = tl.z;
            i += tl.y;
            return true;
        }
        q = (uint32_t)nq;
        i++;
        return true;
    }

    // Walk from node q at text position i (end exclusive): count ids of every terminal,
    // including q itself.
    // (q: the root, or for a compressed table a record below shared_base.)
    __device__ WalkResult walk_from(uint32_t q, const uint8_t *__restrict__ text, uint64_t i, uint64_t end) const {
        WalkResult r{0, 0, 0, 0, 0, 0, 0, 0, 0};
        if constexpr (!MERGED) {
            // plain table: one node word per step; a tail head ends the walk with one
            // comparison of the rest of its path
            for (;;) {
                const uint64_t w = t.nodes[q];
                if (w & kTermBit) {
                    uint32_t f;
                    bool one;
                    const uint32_t k = term_ids(q, w, f, one);
                    r.cnt += k;
                    if (r.nterm == 0) {
                        r.f0 = f;
                        r.k0 = k;
                    }
                    r.nterm++;
                }
                if (i >= end) break;
                if (w_tail(w)) {
                    uint4 tr;
                    if (tail_match(w, text, i, end, tr)) {
                        r.cnt += tr.w;
                        if (r.nterm == 0) {
                            r.f0 = tr.z;
                            r.k0 = tr.w;
                        }
                        r.nterm++;
                    }
                    break;
                }
                const int64_t nq = child_w(q, w, text[i]);
                if (nq < 0) break;
                q = (uint32_t)nq;
                i++;
            }
            return r;
        }
        RankState rs{q, 0};
        for (;;) {
            const uint4 tl = tail(q);
            const bool tq = is_term(q);
            if (tq) {
                const uint32_t x = id_index(q, rs);
                const uint32_t f = t.out_first[x], k = t.out_first[x + 1] - f;
                r.cnt += k;
                if (r.nterm == 0) {
                    r.f0 = f;
                    r.k0 = k;
                }
                r.nterm++;
            }
            if (i >= end) break;
            if (!advance(q, i, tl, text, text[i], end, rs, tq)) break;
        }
        return r;
    }

    // Keys of start s (walk from the root node 0 in HBM) written at keys[o ..), sorted by
    // id; cnt is the walk's id count. Ids of one terminal are sorted; those of nested
    // terminals are merged by insertion.
    __device__ void emit_walk(const uint8_t *__restrict__ text, uint64_t s, uint64_t end, uint64_t *keys,
                              uint64_t o, uint32_t cnt, uint32_t q = 0, uint64_t i0 = ~0ull) const {
        const uint64_t hi = s << 32;
        uint32_t k = 0, nterm = 0;
        uint64_t i = i0 == ~0ull ? s : i0;
        RankState rs{q, 0};
        if constexpr (!MERGED) {
            for (;;) {
                const uint64_t w = t.nodes[q];
                if (w & kTermBit) {
                    nterm++;
                    uint32_t f;
                    bool one;
                    const uint32_t kk = term_ids(q, w, f, one);
                    if (one) keys[o + k++] = hi | f;
                    else
                        for (uint32_t x = f; x < f + kk; x++) keys[o + k++] = hi | t.out_ids[x];
                    if (k >= cnt) break;
                }
                if (i >= end) break;
                if (w_tail(w)) {
                    uint4 tr;
                    if (tail_match(w, text, i, end, tr)) {
                        nterm++;
                        if (tr.w == 1) keys[o + k++] = hi | tr.z;  // the id itself
                        else
                            for (uint32_t x = tr.z; x < tr.z + tr.w; x++) keys[o + k++] = hi | t.out_ids[x];
                    }
                    break;
                }
                const int64_t nq = child_w(q, w, text[i]);
                if (nq < 0) break;
                q = (uint32_t)nq;
                i++;
            }
        } else
        for (;;) {
            const uint4 tl = tail(q);
            const bool tq = is_term(q);
            if (tq) {
                nterm++;
                const uint32_t xi = id_index(q, rs);
                for (uint32_t x = t.out_first[xi]; x < t.out_first[xi + 1]; x++) keys[o + k++] = hi | t.out_ids[x];
                if (k >= cnt) break;
            }
            if (i >= end) break;
            if (!advance(q, i, tl, text, text[i], end, rs, tq)) break;
        }
        if (nterm > 1) {
            for (uint32_t a = 1; a < cnt; a++) {
                const uint64_t v = keys[o + a];
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

// Walk of a survivor in the count kernel: the first D symbols through the LDS root
// image, the rest through the trie in HBM. The first eight text bytes come from one
// round of independent loads.
template <int LAYOUT, bool PACK2, int FORM, bool MERGED>
struct RootWalk {
    const DevTable &t;
    const uint8_t *__restrict__ text;
    const uint32_t *img;  // LDS image

    __device__ WalkResult count(uint64_t s, uint64_t end) const {
        const uint32_t D = t.root_depth;
        if (s + D > end) return WalkResult{0, 0, 0, 0, 0, 0, 0, 0, 0};
        // the first eight bytes: three aligned dwords when they lie inside the walk's
        // bounds (bytes past `end` are read but never used), else byte by byte
        uint64_t w8 = 0;
        const uint64_t b4 = s & ~3ull;
        if (b4 + 12 <= end) {
            const uint32_t *p = reinterpret_cast<const uint32_t *>(text + b4);
            const uint32_t x0 = p[0], x1 = p[1], x2 = p[2], sh = (uint32_t)(s & 3);
            w8 = ((uint64_t)__builtin_amdgcn_alignbyte(x2, x1, sh) << 32) | __builtin_amdgcn_alignbyte(x1, x0, sh);
        } else {
#pragma unroll
            for (int i = 0; i < 8; i++)
                if (s + i < end) w8 |= (uint64_t)text[s + i] << (8 * i);
        }
        uint32_t key = 0;
        if constexpr (PACK2) {
            // the first D bytes (D <= 8) must all be 2-bit codes; the key packs them two
            // bits each, the first symbol highest, with word-wide operations
            const uint64_t dm = D >= 8 ? ~0ull : (1ull << (8 * D)) - 1ull;
            if (w8 & dm & 0xfcfcfcfcfcfcfcfcull) return WalkResult{0, 0, 0, 0, 0, 0, 0, 0, 0};
            auto code4 = [](uint32_t x) {  // bytes b0..b3 (each < 4) -> b0 b1 b2 b3, two bits each
                return ((x & 0xffu) << 6) | ((x >> 4) & 0x30u) | ((x >> 14) & 0x0cu) | (x >> 24);
            };
            const uint32_t c8 = (code4((uint32_t)(w8 & dm)) << 8) | code4((uint32_t)((w8 & dm) >> 32));
            key = c8 >> (2 * (8 - D));
        } else {
            for (uint32_t i = 0; i < D; i++) key = (key << 8) | ((uint32_t)(w8 >> (8 * i)) & 0xffu);
        }
        const uint32_t wi = key >> 5, b = key & 31;
        const uint32_t word = img[Lds<FORM>::root + wi];
        if (!((word >> b) & 1u)) return WalkResult{0, 0, 0, 0, 0, 0, 0, 0, 0};
        const uint16_t *rank = reinterpret_cast<const uint16_t *>(img + Lds<FORM>::rank);
        uint32_t q = t.root_base + rank[wi] + __builtin_popcount(word & ((1u << b) - 1u));
        // continue with the bytes already loaded, then one load per level
        const Trie<LAYOUT, MERGED> T{t};
        WalkResult r{0, 0, 0, 0, 0, 0, 0, 0, 0};
        RankState rs{q, 0};  // the depth-D records lie below shared_base
        uint64_t i = s + D;
        if constexpr (!MERGED) {
            // plain table: one node word per step; a tail head ends the walk with one
            // comparison of the rest of its path (its end is not a node: q0 = kNone)
            // f: index of the ids, or (one) the single id itself
            auto note = [&](uint32_t f, uint32_t k, bool one, uint32_t qn, uint32_t depth) {
                r.cnt += k;
                if (r.nterm == 0) {
                    r.f0 = f;
                    r.k0 = k;
                    if (k == 1) r.id0 = one ? f : t.out_ids[f];  // used only when k == 1
                    r.q0 = qn;
                    r.d0 = depth;
                } else if (r.nterm == 1) {
                    r.k1 = k;
                    if (k == 1) r.id1 = one ? f : t.out_ids[f];
                }
                r.nterm++;
            };
            for (;;) {
                const uint64_t w = t.nodes[q];
                if (w & kTermBit) {
                    uint32_t f;
                    bool one;
                    const uint32_t k = T.term_ids(q, w, f, one);
                    note(f, k, one, q, (uint32_t)(i - s));
                }
                if (i >= end) break;
                if (T.w_tail(w)) {
                    uint4 tr;
                    if (T.tail_match(w, text, i, end, tr))
                        note(tr.z, tr.w, tr.w == 1, kNone, (uint32_t)(i - s) + tr.y);
                    break;
                }
                const uint32_t d = (uint32_t)(i - s);
                const uint32_t c = d < 8 ? (uint32_t)(w8 >> (8 * d)) & 0xffu : (uint32_t)text[i];
                const int64_t nq = T.child_w(q, w, c);
                if (nq < 0) break;
                q = (uint32_t)nq;
                i++;
            }
            return r;
        }
        for (;;) {
            const uint4 tl = T.tail(q);
            const bool tq = T.is_term(q);
            if (tq) {
                const uint32_t x = T.id_index(q, rs);
                const uint32_t f = t.out_first[x], k = t.out_first[x + 1] - f;
                r.cnt += k;
                if (r.nterm == 0) {
                    r.f0 = f;
                    r.k0 = k;
                    r.id0 = t.out_ids[f];  // used only when k == 1; overlaps the rest of the walk
                    r.q0 = q;
                    r.d0 = (uint32_t)(i - s);
                } else if (r.nterm == 1) {
                    r.k1 = k;
                    r.id1 = t.out_ids[f];
                }
                r.nterm++;
            }
            if (i >= end) break;
            const uint32_t d = (uint32_t)(i - s);
            const uint32_t c = d < 8 ? (uint32_t)(w8 >> (8 * d)) & 0xffu : (uint32_t)text[i];
            if (!T.advance(q, i, tl, text, c, end, rs, tq)) break;
        }
        return r;
    }
};

// Text stream loads through a buffer resource over the text: the per-step offset is a
// scalar (wave-uniform) register and the lane's 16-byte slot a fixed vector offset, so a
// load costs no vector address arithmetic. 0x20000: the raw-buffer word 3 of gfx9.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t text_rsrc(const uint8_t *text, uint64_t n) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(text), (short)0,
                                             (int)(n < 0xffffffffull ? n : 0xffffffffull), 0x00020000);
}
__device__ __forceinline__ uint4 stream16(__amdgpu_buffer_rsrc_t rs, uint32_t lane_off, uint32_t step_off) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, lane_off, __builtin_amdgcn_readfirstlane(step_off), 0);
    return make_uint4(v.x, v.y, v.z, v.w);
}

// 16 bytes at p; bytes at or past `lim` read as zero (no load at all when p >= lim).
// Vector load when the 16 bytes are whole and aligned.
__device__ __forceinline__ uint4 load16(const uint8_t *__restrict__ text, uint64_t p, uint64_t lim, bool aligned) {
    uint4 v;
    if (aligned && p + 16 <= lim) {
        v = *reinterpret_cast<const uint4 *>(text + p);
    } else if (p >= lim) {
        v = make_uint4(0u, 0u, 0u, 0u);
    } else {
        uint32_t b[16];
#pragma unroll
        for (int i = 0; i < 16; i++) b[i] = p + i < lim ? text[p + i] : 0u;
        v.x = b[0] | (b[1] << 8) | (b[2] << 16) | (b[3] << 24);
        v.y = b[4] | (b[5] << 8) | (b[6] << 16) | (b[7] << 24);
        v.z = b[8] | (b[9] << 8) | (b[10] << 16) | (b[11] << 24);
        v.w = b[12] | (b[13] << 8) | (b[14] << 16) | (b[15] << 24);
    }
    return v;
}

// Two-bit codes of 16 bytes, first byte in the top bits.
__device__ __forceinline__ uint32_t pack2x16(uint4 v) {
    // Per dword, bytes b0..b3 keep their low two bits (y). One 24-bit multiply-add puts
    // b0 b1 b2 b3 (two bits each, b0 highest) in byte 2 of p: y's low three bytes times
    // 2^22 + 2^12 + 2^2 land b0, b1, b2 at bits 22, 20, 18 (the other partial products
    // stay below bit 14 or start at bit 28), and the added byte-permute of y puts b3 at
    // bit 16. Two permutes and an or then gather the four code bytes, first dword highest.
    const uint32_t d[4] = {v.x, v.y, v.z, v.w};
    uint32_t p[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const uint32_t y = d[i] & 0x03030303u;
        p[i] = __umul24(y, 0x401004u) + __builtin_amdgcn_perm(y, y, 0x0c030c0cu);  // low 24 bits of y
    }
    return __builtin_amdgcn_perm(p[0], p[1], 0x06020c0cu) | __builtin_amdgcn_perm(p[2], p[3], 0x0c0c0602u);
}

// First prefilter probe of a key: the word at the masked high half of key * kFilterMul
// in the first-probe region, bit key & 31.
__device__ __forceinline__ uint32_t probe(const uint32_t *img, uint32_t key) {
    const uint32_t off = (__umulhi(key, kFilterMul) & kAmask1) + kLdsF1 * 4;
    const uint32_t w = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const uint8_t *>(img) + off);
    return __builtin_amdgcn_ubfe(w, key, 1);
}

// Second probe, for a key that passed the first: the second-probe region, bit = the top
// five bits of the high half of key * kFilterMul2.
__device__ __forceinline__ uint32_t probe2(const uint32_t *img, uint32_t key) {
    const uint32_t h = __umulhi(key, kFilterMul2);
    const uint32_t w = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const uint8_t *>(img) + (h & kAmask2));
    return (w >> (h >> 27)) & 1u;
}

// Sampled layout: the 3-gram probe (bytes j..j+2 of x, its top byte ignored by the
// 24-bit multiply) and the two probes of a candidate start's 4-gram.
__device__ __forceinline__ uint32_t probe3(const uint32_t *img, uint32_t x) {
    const uint32_t h = (x & 0xffffffu) * kFilterMul3;  // low half of a 24 x 24-bit product
    const uint32_t w = *reinterpret_cast<const uint32_t *>(reinterpret_cast<const uint8_t *>(img) + kLdsS3 * 4 +
                                                          ((h >> 16) & ((kS3Words - 1u) << 2)));
    return __builtin_amdgcn_ubfe(w, x, 1);
}
// Both 4-gram probes of one key, given key >> 8 as well (bytes 1..3: probe 1's hash
// input, and its low five bits are probe 2's bit).
__device__ __forceinline__ uint32_t probe4s(const uint32_t *img, uint32_t key, uint32_t key_hi) {
    const uint8_t *b = reinterpret_cast<const uint8_t *>(img);
    const uint32_t o1 = (((key_hi & 0xffffffu) * kS1Mul) >> 16) & ((kS1Words - 1u) << 2);
    const uint32_t o2 = (s2_hash(key) >> 16) & ((kS2Words - 1u) << 2);
    const uint32_t w1 = *reinterpret_cast<const uint32_t *>(b + kLdsS1 * 4 + o1);
    const uint32_t w2 = *reinterpret_cast<const uint32_t *>(b + kLdsS2 * 4 + o2);
    return __builtin_amdgcn_ubfe(w1, key, 1) & __builtin_amdgcn_ubfe(w2, key_hi, 1);
}

// Four bytes starting at byte j (0..15) of the 20 bytes v, d4 (little-endian words).
__device__ __forceinline__ uint32_t bytes4_at(uint4 v, uint32_t d4, uint32_t j) {
    const uint32_t qd = j >> 2;
    const uint32_t lo = qd == 0 ? v.x : qd == 1 ? v.y : qd == 2 ? v.z : v.w;
    const uint32_t hi = qd == 0 ? v.y : qd == 1 ? v.z : qd == 2 ? v.w : d4;
    return __builtin_amdgcn_alignbyte(hi, lo, j & 3);
}

// One direct probe of the root bitmap: bit `key` of the bitmap at `root`.
__device__ __forceinline__ uint32_t probe_root(const uint32_t *root, uint32_t key) {
    return __builtin_amdgcn_ubfe(root[key >> 5], key, 1);
}

// Prefilter forms, fixed per kernel instance: FM_K4 four-byte keys and no pattern shorter
// than four (the sampled layout); FM_GEN any key length, with the short-pattern bitmap;
// FM_ROOT no hashed filter (the root image's D-gram bitmap is the test); FM_EXACT two-bit
// symbols, the exact bitmap of the first D + 1 trie levels (the exact layout).
enum FilterMode : int { FM_K4 = 0, FM_GEN = 1, FM_ROOT = 2, FM_EXACT = 3 };

// LDS layout of a kernel instance.
template <bool PACK2, int FM>
struct FormOf {
    static constexpr int value = (FM == FM_K4 && !PACK2) ? kFormSampled : (FM == FM_EXACT && PACK2) ? kFormExact
                                                                                                   : kFormGeneral;
};

// Prefilter mask of 16 starts of a lane (bit j = the start at byte j of cur): the
// survivors, or for FM_K4 the candidates (odd j only; see sample_step). cur: the 16
// bytes; next_d0: the 4 bytes after them; c0/c1: two-bit codes of these and the next
// 16 bytes.
template <bool PACK2, int FM>
__device__ __forceinline__ uint32_t prefilter16(const DevTable &t, const uint32_t *img, uint4 cur,
                                                uint32_t next_d0, uint32_t c0, uint32_t c1) {
    uint32_t mask = 0;
    if (!PACK2) {
        const uint32_t d[5] = {cur.x, cur.y, cur.z, cur.w, next_d0};
        if (FM == FM_K4) {
            // sampled: probe the 3-gram at every odd start j; a pattern (four bytes or
            // more) starting at j or j-1 puts its 3-gram at offset 0 or 1 there. The
            // mask holds the odd starts that pass: candidates, each standing for the
            // starts j-1 and j, which the lane then checks (sample_step).
            // bits gathered two positions at a time (one shift-or each), then moved up
            // by one to their odd positions
#pragma unroll
            for (int j = 15; j >= 1; j -= 2) {
                const uint32_t x = __builtin_amdgcn_alignbyte(d[(j >> 2) + 1], d[j >> 2], j & 3);
                mask = shl2_or(mask, probe3(img, x));
            }
            mask <<= 1;
        } else if (FM == FM_GEN) {
            // k-gram filter, plus the short bitmap for patterns shorter than k
            const uint32_t kmask = t.filter_k >= 4 ? 0xffffffffu : (1u << (8 * t.filter_k)) - 1u;
            const uint32_t *shrt = img + Lds<kFormGeneral>::shrt;
            const bool two = t.root_depth == 2, sh = t.has_short;
            uint32_t ms = 0;
#pragma unroll
            for (int j = 15; j >= 0; j--) {
                const uint32_t x = (j & 3) ? __builtin_amdgcn_alignbyte(d[(j >> 2) + 1], d[j >> 2], j & 3) : d[j >> 2];
                mask = (mask << 1) | probe(img, x & kmask);
                if (sh) {
                    const uint32_t key = two ? (((x & 0xffu) << 8) | ((x >> 8) & 0xffu)) : (x & 0xffu);
                    ms = (ms << 1) | probe_root(shrt, key);
                }
            }
            uint32_t rem = mask & ~ms;
            while (rem) {
                const uint32_t j = __builtin_ctz(rem);
                rem &= rem - 1;
                mask &= ~((probe2(img, bytes4_at(cur, next_d0, j) & kmask) ^ 1u) << j);
            }
            mask |= ms;
        } else {
            // root image as the filter: D-byte key, first byte most significant
            const uint32_t *root = img + Lds<kFormGeneral>::root;
            const bool two = t.root_depth == 2;
#pragma unroll
            for (int j = 15; j >= 0; j--) {
                const uint32_t x = (j & 3) ? __builtin_amdgcn_alignbyte(d[(j >> 2) + 1], d[j >> 2], j & 3) : d[j >> 2];
                const uint32_t key = two ? (((x & 0xffu) << 8) | ((x >> 8) & 0xffu)) : (x & 0xffu);
                mask = (mask << 1) | probe_root(root, key);
            }
        }
    } else {
        // window of K symbols at j: the top 2K bits of symbols j..j+15
        const uint32_t K = FM != FM_ROOT ? t.filter_k : t.root_depth;
        const uint32_t rs = 32 - 2 * K;
        if (FM == FM_EXACT) {
            // one probe per start: bit (symbols j .. j+K-1) of the exact bitmap at offset 0
#pragma unroll
            for (int j = 15; j >= 0; j--) {
                const uint32_t top = j ? __builtin_amdgcn_alignbit(c0, c1, 32 - 2 * j) : c0;
                mask = (mask << 1) | probe_root(img, top >> rs);
            }
        } else if (FM != FM_ROOT) {
            // k-gram filter, plus the short bitmap (D-grams) for patterns shorter than k
            const uint32_t *shrt = img + Lds<kFormGeneral>::shrt;
            const uint32_t rsd = 32 - 2 * t.root_depth;
            const bool sh = t.has_short;
            uint32_t ms = 0;
#pragma unroll
            for (int j = 15; j >= 0; j--) {
                const uint32_t top = j ? __builtin_amdgcn_alignbit(c0, c1, 32 - 2 * j) : c0;
                mask = (mask << 1) | probe(img, rs >= 32 ? top : top >> rs);
                if (sh) ms = (ms << 1) | probe_root(shrt, top >> rsd);
            }
            uint32_t rem = mask & ~ms;
            while (rem) {
                const uint32_t j = __builtin_ctz(rem);
                rem &= rem - 1;
                const uint32_t top = j ? __builtin_amdgcn_alignbit(c0, c1, 32 - 2 * j) : c0;
                mask &= ~((probe2(img, rs >= 32 ? top : top >> rs) ^ 1u) << j);
            }
            mask |= ms;
        } else {
            const uint32_t *root = img + Lds<kFormGeneral>::root;
#pragma unroll
            for (int j = 15; j >= 0; j--) {
                const uint32_t top = j ? __builtin_amdgcn_alignbit(c0, c1, 32 - 2 * j) : c0;
                mask = (mask << 1) | probe_root(root, top >> rs);
            }
        }
    }
    return mask;
}

// Per-wave state of one span (wave-uniform values).
struct SpanState {
    uint64_t a;       // first byte of the span
    uint32_t span;    // span index
    uint32_t qlen;    // survivors queued
    uint32_t nh;      // records stored
    uint32_t ovf;     // span-local start of the first matching start not recorded, or kNone
    uint64_t my_cnt;  // this lane's share of the span's match count
    uint64_t top;     // starts at or past top are not counted here
};

template <int LAYOUT, bool PACK2, bool SEG, int FM, bool MERGED, uint32_t LB>
struct Scanner {
    static constexpr uint32_t kLB = LB, kSt = Lanes<LB>::step, kPf = Lanes<LB>::prefetch;
    const DevTable &t;
    static constexpr bool kSampled = FM == FM_K4 && !PACK2;
    static constexpr int kForm = FormOf<PACK2, FM>::value;
    static constexpr uint32_t kQ = Lds<kForm>::qcap;  // survivor queue entries
    RootWalk<LAYOUT, PACK2, kForm, MERGED> W;
    const uint8_t *__restrict__ text;
    uint64_t n, lim;  // starts >= lim cannot match (too little text left)
    const uint64_t *__restrict__ offsets;
    uint32_t n_packets;
    SpanOut so;
    uint16_t *q;  // survivor queue (span-local starts), kQ entries
    bool aligned;
    uint32_t *stg;  // sampled form: this wave's step staging words (kStageWords)

    // A lane's bytes of one step: kLB (16 or 32) consecutive text bytes, with the
    // two-bit codes of each 16 when symbols are two-bit codes.
    struct Chunk {
        uint4 v[kLB / 16];
    };

    __device__ __forceinline__ uint64_t end_of(uint64_t s) const {
        if (!SEG) return n;
        const uint64_t e = packet_end(offsets, n_packets, s);
        return e < n ? e : n;
    }

    // Walk `cnt` queued survivors from q[first], one per lane; record the matching ones.
    __device__ __forceinline__ void walk_batch(SpanState &S, uint32_t first, uint32_t cnt) {
        const uint32_t lane = lane_id();
        const bool on = lane < cnt;
        const uint32_t sl = on ? q[first + lane] : 0u;
        const uint64_t s = S.a + sl;
        WalkResult r{0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (on) r = W.count(s, end_of(s));
        S.my_cnt += r.cnt;
        const uint64_t hb = __ballot(r.cnt > 0);
        if (hb && S.ovf == kNone) {
            // records per start: one; two (one per id, in id order) for a start that
            // passed exactly two terminals with one id each
            const bool two = r.nterm == 2 && r.k0 == 1 && r.k1 == 1;
            const uint32_t rc = r.cnt > 0 ? (two ? 2u : 1u) : 0u;
            const uint32_t incl = wave_incl_scan(rc);
            const uint32_t pos = S.nh + incl - rc;
            const uint32_t hcap = 1u << so.rec_log2;
            const bool store = rc > 0 && pos + rc <= hcap;
            if (store) {
                uint64_t *rec = so.rec + ((size_t)S.span << so.rec_log2) + pos;
                if (two) {
                    const uint32_t a = r.id0 < r.id1 ? r.id0 : r.id1, b = r.id0 < r.id1 ? r.id1 : r.id0;
                    rec[0] = ((uint64_t)a << 32) | (1u << 16) | sl;
                    rec[1] = ((uint64_t)b << 32) | (1u << 16) | sl;
                } else {
                    // one terminal: its id itself when it has one, else where its ids are;
                    // several: the first one's node and depth, where the placement resumes
                    uint32_t k, hi;
                    if (r.nterm == 1 && r.k0 < kRecMulti) {
                        k = r.k0;
                        hi = k == 1 ? r.id0 : r.f0;
                    } else if (r.nterm > 1 && r.d0 < kRecMulti - 1 && (!MERGED || r.q0 < t.shared_base)) {
                        // (a compressed table resumes only from a record whose own rank
                        // word is its rank)
                        k = kRecMulti | r.d0;
                        hi = r.q0;
                    } else {
                        k = 0;  // walk again from the root
                        hi = 0;
                    }
                    rec[0] = ((uint64_t)hi << 32) | (k << 16) | sl;
                }
            }
            const uint64_t lost = __ballot(rc > 0 && !store);
            if (lost) {
                // records end where the first start that did not fit would have begun
                const int f = (int)__builtin_ctzll(lost);
                S.ovf = __builtin_amdgcn_readlane(sl, f);
                S.nh = __builtin_amdgcn_readlane(pos, f);
            } else {
                S.nh += __builtin_amdgcn_readlane(incl, 63);
            }
        }
    }

    // Walk every full batch of 64 queued survivors; keep the rest (< 64) at the front.
    __device__ __forceinline__ void drain(SpanState &S) {
        const uint32_t lane = lane_id();
        uint32_t done = 0;
        while (S.qlen - done >= 64) {
            walk_batch(S, done, 64);
            done += 64;
        }
        if (!done) return;
        const uint32_t rest = S.qlen - done;
        const uint16_t v = lane < rest ? q[done + lane] : 0;
        __builtin_amdgcn_wave_barrier();
        if (lane < rest) q[lane] = v;
        __builtin_amdgcn_wave_barrier();
        S.qlen = rest;
    }

    // Append the positions sl0 + j of the set bits j of every lane's m to the queue qq
    // (len entries, room for cap), in position order. flush() leaves fewer than 64
    // entries; it runs when a step's positions might not fit, and between windows when
    // they do not fit at all (position k of the step is the k-th in position order).
    template <class Flush>
    __device__ __forceinline__ void push(uint16_t *qq, uint32_t &len, uint32_t cap, uint32_t m, uint32_t sl0,
                                         Flush flush) {
        if (!__ballot(m != 0)) return;
        const uint32_t c = __builtin_popcount(m);
        const uint32_t inc = wave_incl_scan(c);
        const uint32_t tot = __builtin_amdgcn_readlane(inc, 63);
        if (len + tot > cap) flush();  // now len < 64
        if (len + tot <= cap) {
            uint32_t at = len + inc - c;
            while (m) {
                const uint32_t j = __builtin_ctz(m);
                m &= m - 1;
                qq[at++] = (uint16_t)(sl0 + j);
            }
            len += tot;
            __builtin_amdgcn_wave_barrier();
            return;
        }
        for (uint32_t done = 0; done < tot;) {
            const uint32_t room = cap - len;
            const uint32_t w = room < tot - done ? room : tot - done;
            uint32_t mm = m, k = inc - c;
            while (mm) {
                const uint32_t j = __builtin_ctz(mm);
                mm &= mm - 1;
                if (k >= done && k < done + w) qq[len + (k - done)] = (uint16_t)(sl0 + j);
                k++;
            }
            __builtin_amdgcn_wave_barrier();
            len += w;
            done += w;
            if (done < tot) flush();
        }
    }

    // Survivors of one step to the survivor queue. Walks wait until the queue might not
    // hold another step (or the span ends).
    __device__ __forceinline__ void take(SpanState &S, uint32_t m, uint32_t sl0) {
        push(q, S.qlen, kQ, m, sl0, [&] { drain(S); });
    }

    // Both 4-gram probes of the starts j-1 and j (bits j-1 and j of the result). The two
    // words holding bytes j-1 .. j+3 (j odd, so j-1 is even and the five bytes never span
    // three words) are read back from the lane's staged step bytes: words q and q + 1,
    // q = (j - 1) >> 2, one LDS read for a choice a register file cannot index per lane.
    __device__ __forceinline__ uint32_t check2(const uint32_t *my, uint32_t j) const {
        const uint32_t q = (j - 1) >> 2;
        const uint32_t lo = my[q], hi = my[q + 1];
        // k0 = bytes j-1..j+2, k1 = bytes j..j+3: k0 >> 8 equals k1 in the 24 bits a
        // 24-bit multiply reads (and in its low byte), so k1 stands in for it
        const uint32_t k0 = __builtin_amdgcn_alignbyte(hi, lo, (j - 1) & 3u);
        const uint32_t k1 = __builtin_amdgcn_alignbyte(hi, lo, j & 3u);
        const uint32_t p0 = probe4s(W.img, k0, k1);
        const uint32_t p1 = probe4s(W.img, k1, k1 >> 8);
        return ((p1 << 1) | p0) << (j - 1);
    }

    // Sampled prefilter, one step: m holds this lane's candidates (bit j, j odd: the
    // starts j-1 and j of the lane's bytes). Each lane checks its own: the first two
    // candidates of every lane together (all their LDS probes in flight at once), then
    // any further ones (rare). Starts whose 4-gram passes join the survivor queue.
    __device__ __forceinline__ void sample_step(SpanState &S, uint64_t step, const Chunk &cur, uint32_t nd,
                                                uint32_t m, uint32_t sl0) {
        static_assert(kLB == 32, "the sampled check reads a lane's 32 bytes");
        if (!__ballot(m != 0)) return;
        // the lane's 36 bytes to its staging words (read back only by this lane; the
        // wave's LDS operations complete in order, so no barrier is needed either way)
        uint32_t *my = stg + kStageLaneWords * lane_id();
        my[0] = cur.v[0].x;
        my[1] = cur.v[0].y;
        my[2] = cur.v[0].z;
        my[3] = cur.v[0].w;
        my[4] = cur.v[1].x;
        my[5] = cur.v[1].y;
        my[6] = cur.v[1].z;
        my[7] = cur.v[1].w;
        my[8] = nd;
        const uint32_t m2 = m & (m - 1), m3 = m2 & (m2 - 1);
        uint32_t sm = 0;
        if (m) {  // only lanes with candidates probe (fewer LDS bank conflicts)
            sm = check2(my, (uint32_t)__builtin_ctz(m));
            if (m2) sm |= check2(my, (uint32_t)__builtin_ctz(m2));
        }
        for (uint32_t r = m3; __ballot(r != 0);) {
            const uint32_t j = r ? (uint32_t)__builtin_ctz(r) : 1u;
            const uint32_t s = check2(my, j);
            sm |= r ? s : 0u;
            r &= r - 1;
        }
        // the span's last step: keep starts below top
        // span-local and 32-bit (scalar); top can lie before the span start
        if ((uint32_t)(step - S.a) + kSt > (S.top > S.a ? (uint32_t)(S.top - S.a) : 0u)) {
            const uint64_t s0 = S.a + sl0;
            if (s0 + kLB > S.top) sm &= s0 >= S.top ? 0u : (uint32_t)((1ull << (uint32_t)(S.top - s0)) - 1ull);
        }
        take(S, sm, sl0);
    }

    // One step's prefilter mask: candidates (sampled prefilter, checked here) or survivors.
    __device__ __forceinline__ void step_body(SpanState &S, uint64_t step, uint64_t top, const Chunk &cur, uint32_t nd,
                                              uint32_t nc, uint32_t pc) {
        uint32_t sl0;
        const uint32_t m = mask_step(S, step, top, cur, nd, nc, pc, &sl0);
        if constexpr (kSampled)
            sample_step(S, step, cur, nd, m, sl0);
        else
            take(S, m, sl0);
    }

    __device__ __forceinline__ Chunk chunk_buffer(__amdgpu_buffer_rsrc_t rs, uint32_t loff, uint32_t soff) const {
        Chunk c;
#pragma unroll
        for (uint32_t h = 0; h < kLB / 16; h++) c.v[h] = stream16(rs, loff + 16 * h, soff);
        return c;
    }
    __device__ __forceinline__ Chunk chunk_guarded(uint64_t p, uint64_t ld) const {
        Chunk c;
#pragma unroll
        for (uint32_t h = 0; h < kLB / 16; h++) c.v[h] = load16(text, p + 16 * h, ld, aligned);
        return c;
    }

    // Survivor mask of this lane's kLB starts at `step` (bit j = start
    // step + kLB * lane + j), cut to [S.a, top). next_d0 / next_c: first word / first
    // two-bit codes of the bytes after this lane's; pc: two-bit codes of the lane's first
    // 16 bytes.
    __device__ __forceinline__ uint32_t mask_step(const SpanState &S, uint64_t step, uint64_t top, const Chunk &cur,
                                                  uint32_t next_d0, uint32_t next_c, uint32_t pc,
                                                  uint32_t *sl0_out) const {
        const uint32_t lane = lane_id();
        uint32_t m = 0;
#pragma unroll
        for (uint32_t h = 0; h < kLB / 16; h++) {
            const bool lasth = h + 1 == kLB / 16;
            const uint32_t nd = lasth ? next_d0 : cur.v[h + 1].x;
            const uint32_t c0 = PACK2 ? (h == 0 ? pc : pack2x16(cur.v[h])) : 0u;
            const uint32_t c1 = PACK2 ? (lasth ? next_c : pack2x16(cur.v[h + 1])) : 0u;
            m |= prefilter16<PACK2, FM>(t, W.img, cur.v[h], nd, c0, c1) << (16 * h);
        }
        const uint32_t sl0 = (uint32_t)(step - S.a) + kLB * lane;  // span-local start of bit 0
        // last step: keep starts below top (a candidate j while j-1 is below it)
        const uint64_t cut = FM == FM_K4 && !PACK2 ? top + 1 : top;
        // span-local and 32-bit (scalar); cut can lie before the span start
        if ((uint32_t)(step - S.a) + kSt > (cut > S.a ? (uint32_t)(cut - S.a) : 0u)) {
            const uint64_t s0 = S.a + sl0;
            if (s0 + kLB > cut) m &= s0 >= cut ? 0u : (uint32_t)((1ull << (uint32_t)(cut - s0)) - 1ull);
        }
        *sl0_out = sl0;
        return m;
    }

    // First word and first two-bit codes of the next lane's chunk (the last lane takes
    // them from the next step's lane 0, or from `after` past the span's last step). pc /
    // pn: two-bit codes of the first 16 bytes of this lane's chunk and of its next step's.
    __device__ __forceinline__ void next_lane_head(const Chunk &cur, const Chunk &nxt, bool last, uint4 after,
                                                   uint32_t pc, uint32_t pn, uint32_t *d0, uint32_t *c0) const {
        const uint32_t lane = lane_id();
        const uint32_t dn = from_next_lane(cur.v[0].x);
        const uint32_t d0n = last ? after.x : __builtin_amdgcn_readfirstlane(nxt.v[0].x);
        *d0 = lane == 63 ? d0n : dn;
        if (PACK2) {
            const uint32_t cn = from_next_lane(pc);
            const uint32_t c0n = last ? pack2x16(after) : __builtin_amdgcn_readfirstlane(pn);
            *c0 = lane == 63 ? c0n : cn;
        } else {
            *c0 = 0;
        }
    }

    // Count the span [S.a, hi).
    __device__ __forceinline__ void stream(SpanState &S, uint64_t hi) {
        const uint32_t lane = lane_id();
        uint64_t step = S.a;
        const uint64_t hiR = (hi + kSt - 1) & ~(uint64_t)(kSt - 1);  // end of the last step
        const uint64_t top = hi < lim ? hi : lim;
        S.top = top;
        if (aligned && hiR + 16 <= n) {
            // Steady state: every load is an unconditional 16-byte load with no per-lane
            // test, kPf steps ahead; addresses past the span are clamped to its last
            // step (a repeated load, no bytes past the span). Only the 16 bytes right
            // after the span are read for the last starts' windows.
            const uint64_t lastst = hiR - kSt;
            const uint4 after = *reinterpret_cast<const uint4 *>(text + hiR);  // uniform address
            const __amdgpu_buffer_rsrc_t rs = text_rsrc(text, n);
            const uint32_t loff = kLB * lane;
            Chunk buf[kPf];  // buf[0]: this step; buf[i]: i steps ahead
#pragma unroll
            for (uint32_t i = 0; i < kPf; i++)
                buf[i] = chunk_buffer(rs, loff, (uint32_t)(step + i * kSt < lastst ? step + i * kSt : lastst));
            const uint32_t last32 = (uint32_t)lastst;  // the text is below 4 GiB
            // two-bit codes of the first 16 bytes of this step's chunk, carried over from
            // the step before (it needs the next step's for its last lane)
            uint32_t pc = PACK2 ? pack2x16(buf[0].v[0]) : 0u;
            for (; step < hiR; step += kSt) {
                // kPf steps ahead, clamped to the last step (32-bit scalar arithmetic;
                // step <= lastst here, so the difference does not wrap)
                const uint32_t st32 = (uint32_t)step;
                const uint32_t ak = last32 - st32 > kPf * kSt ? st32 + kPf * kSt : last32;
                const Chunk nxk = chunk_buffer(rs, loff, ak);
                uint32_t nd, nc;
                const uint32_t pn = PACK2 ? pack2x16(buf[1 % kPf].v[0]) : 0u;
                next_lane_head(buf[0], buf[1 % kPf], step == lastst, after, pc, pn, &nd, &nc);
                step_body(S, step, top, buf[0], nd, nc, pc);
                pc = pn;
#pragma unroll
                for (uint32_t i = 0; i + 1 < kPf; i++) buf[i] = buf[i + 1];
                buf[kPf - 1] = nxk;
            }
        } else {
            // End of the text, or an unaligned text: guarded loads, zero past the end.
            const uint64_t need = hi + (PACK2 ? 16 : 4);
            const uint64_t ld = need < n ? need : n;
            Chunk cur = chunk_guarded(step + kLB * lane, ld);
            Chunk nx1 = chunk_guarded(step + kSt + kLB * lane, ld);
            for (; step < hi; step += kSt) {
                const Chunk nx2 = chunk_guarded(step + 2 * kSt + kLB * lane, ld);
                uint32_t nd, nc;
                const uint32_t pc = PACK2 ? pack2x16(cur.v[0]) : 0u, pn = PACK2 ? pack2x16(nx1.v[0]) : 0u;
                next_lane_head(cur, nx1, false, make_uint4(0u, 0u, 0u, 0u), pc, pn, &nd, &nc);
                step_body(S, step, top, cur, nd, nc, pc);
                cur = nx1;
                nx1 = nx2;
            }
        }
        drain(S);
        if (S.qlen) {
            walk_batch(S, 0, S.qlen);
            S.qlen = 0;
        }
    }
};

// ------------------------------------------------------------------ count kernel
template <int LAYOUT, bool PACK2, bool SEG, int FM, bool MERGED, uint32_t LB>
__global__ __launch_bounds__(kThreads, PFAC_SCAN_MIN_WG) void scan_count(DevTable t, const uint8_t *__restrict__ text, uint64_t n,
                                                      const uint64_t *__restrict__ offsets, uint32_t n_packets,
                                                      SpanOut so, const uint64_t *__restrict__ sizes,
                                                      uint32_t span_log2) {
    using L = Lds<FormOf<PACK2, FM>::value>;
    __shared__ __align__(16) uint32_t img[L::words];
    if (sizes) {  // sizes of this batch, bounded by those the launch was set up for
        n = sizes[0] < n ? sizes[0] : n;
        n_packets = sizes[1] < n_packets ? (uint32_t)sizes[1] : n_packets;
    }
    const uint64_t span_len = 1ull << span_log2;
    const uint32_t n_spans = (uint32_t)((n + span_len - 1) >> span_log2);
    {
        // filter words to offset 0 (16 bytes a load), root bitmap, rank table and short
        // bitmap (one run in the image) to their fixed places. A thread issues all its
        // loads of a round before its first store: one memory round trip per round,
        // not one per word.
        const uint32_t f4 = t.root_word / 4, rw = t.rank_word - t.root_word, kw = t.short_word - t.rank_word,
                       small = t.lds_words - t.root_word;
        const uint4 *__restrict__ fsrc = reinterpret_cast<const uint4 *>(t.lds_image);
        const uint32_t *__restrict__ ssrc = t.lds_image + t.root_word;
        constexpr uint32_t kF = 8, kS = 6;
        for (uint32_t base = 0; base < f4 || base < small; base += kF * kThreads) {
            uint4 fv[kF];
            uint32_t sv[kS];
#pragma unroll
            for (uint32_t u = 0; u < kF; u++) {
                const uint32_t i = base + u * kThreads + threadIdx.x;
                fv[u] = i < f4 ? fsrc[i] : make_uint4(0u, 0u, 0u, 0u);
            }
#pragma unroll
            for (uint32_t u = 0; u < kS; u++) {
                const uint32_t i = base + u * kThreads + threadIdx.x;
                sv[u] = i < small ? ssrc[i] : 0u;
            }
#pragma unroll
            for (uint32_t u = 0; u < kF; u++) {
                const uint32_t i = base + u * kThreads + threadIdx.x;
                if (i < f4) reinterpret_cast<uint4 *>(img)[i] = fv[u];
            }
#pragma unroll
            for (uint32_t u = 0; u < kS; u++) {
                const uint32_t i = base + u * kThreads + threadIdx.x;
                if (i < small) img[i < rw ? L::root + i : i < rw + kw ? L::rank + (i - rw) : L::shrt + (i - rw - kw)] = sv[u];
            }
            // words kS * kThreads and up of the small run (none at the shapes allowed)
            for (uint32_t i = base + kS * kThreads + threadIdx.x; i < small && i < base + kF * kThreads; i += kThreads)
                img[i < rw ? L::root + i : i < rw + kw ? L::rank + (i - rw) : L::shrt + (i - rw - kw)] = ssrc[i];
        }
    }
    __syncthreads();  // the only barrier: waves run independently from here

    // the wave index through a scalar register: everything derived from it (span, step,
    // load offsets) then stays in scalar registers
    const uint32_t lane = lane_id(), wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint16_t *wq = reinterpret_cast<uint16_t *>(img + L::queues) + wave * L::qcap;
    uint32_t *stg = nullptr;
    if constexpr (FormOf<PACK2, FM>::value == kFormSampled) stg = img + L::stage + wave * kStageWords;
    Scanner<LAYOUT, PACK2, SEG, FM, MERGED, LB> sc{t, {t, text, img}, text, n, n >= t.min_len ? n - t.min_len + 1 : 0,
                                   offsets, n_packets, so, wq, (((uintptr_t)text) & 15) == 0, stg};
    const uint32_t waves = gridDim.x * kWaves;
    for (uint32_t span = blockIdx.x * kWaves + wave; span < n_spans; span += waves) {
        SpanState S{(uint64_t)span << span_log2, span, 0, 0, kNone, 0};
        const uint64_t hi = S.a + span_len < n ? S.a + span_len : n;
        sc.stream(S, hi);
        const uint64_t total = wave_sum64(S.my_cnt);
        if (lane == 0) {
            so.cnt[span] = total;
            so.nh[span] = S.nh;
            so.ovf[span] = S.ovf;
        }
    }
}

// ------------------------------------------------------------------ placement kernel
// Persistent: each workgroup takes block tickets until they run out, and finishes one
// block (sum, look-back, keys) before it takes the next, so a look-back only ever waits
// on blocks that running workgroups are working on.
template <int LAYOUT, bool SEG, bool MERGED>
__global__ __launch_bounds__(kPlaceThreads) void place_emit(DevTable t, const uint8_t *__restrict__ text, uint64_t n,
                                                           const uint64_t *__restrict__ offsets, uint32_t n_packets,
                                                           uint64_t *__restrict__ keys, uint64_t cap,
                                                           uint64_t *__restrict__ d_count, SpanOut so, TileState ts,
                                                           const uint64_t *__restrict__ sizes, uint32_t span_log2) {
    __shared__ uint64_t span_off[kBlockSpans];
    __shared__ uint32_t span_nh[kBlockSpans];
    __shared__ uint32_t span_cls[kBlockSpans];  // 0: no match, 1: one lane writes it, 2: a wave does
    __shared__ uint32_t span_ovf[kBlockSpans];
    __shared__ uint32_t sh[4];
    __shared__ uint64_t pre[kPlaceWaves];
    if (sizes) {
        n = sizes[0] < n ? sizes[0] : n;
        n_packets = sizes[1] < n_packets ? (uint32_t)sizes[1] : n_packets;
    }
    const uint64_t span_len = 1ull << span_log2;
    const uint32_t n_spans = (uint32_t)((n + span_len - 1) >> span_log2);
    const uint32_t n_blocks = (n_spans + kBlockSpans - 1) / kBlockSpans;
    // Up to kDirectMaxSpans spans, each block sums the counts of all spans before it
    // itself: no block waits on another, so blocks go by workgroup index, with no ticket,
    // look-back or last-workgroup step; the last block writes the count. Beyond that,
    // blocks are taken by ticket and placed by decoupled look-back.
    const bool direct = n_spans <= kDirectMaxSpans;
    uint32_t next_blk = blockIdx.x;
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const Trie<LAYOUT, MERGED> T{t};
    uint32_t epoch = 0;  // look-back words' epoch (not used by direct placement)
    if (!direct) {
        if (threadIdx.x == 0) sh[1] = __hip_atomic_load(&ts.ctrl[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        epoch = sh[1];
    }
    const uint64_t tagE = (uint64_t)epoch << 44;
    auto end_of = [&](uint64_t s) -> uint64_t {
        if (!SEG) return n;
        const uint64_t e = packet_end(offsets, n_packets, s);
        return e < n ? e : n;
    };
    for (;;) {
        uint32_t blk;
        if (direct) {
            blk = next_blk;
            next_blk += gridDim.x;
        } else {
            if (threadIdx.x == 0) sh[0] = __hip_atomic_fetch_add(&ts.ctrl[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            blk = sh[0];
            __syncthreads();  // sh[0] is rewritten by the next take
        }
        if (blk >= n_blocks) break;
        // wave 0, lane i: span i of the block; its count, record count, overflow and first
        // records, all loaded at once (records past the stored ones are read and ignored)
        // Loads go out unconditionally from clamped indices (no branch around any of them),
        // so every one of a lane's loads is in flight at once; the selects come after.
        const uint32_t my_sp = blk * kBlockSpans + lane;
        const bool my_in = wave == 0 && my_sp < n_spans;
        const uint32_t sp_c = my_in ? my_sp : 0u;
        const uint64_t c_ld = so.cnt[sp_c];
        const uint32_t nh_ld = so.nh[sp_c], ovf_ld = so.ovf[sp_c];
        uint64_t my_rec[kFastRecs];
#pragma unroll
        for (uint32_t k = 0; k < kFastRecs; k++) my_rec[k] = so.rec[((size_t)sp_c << so.rec_log2) + k];
        uint64_t before = 0;  // matches in spans before this block (direct mode)
        if (direct) {
            uint64_t part = 0;
            const uint32_t lim_s = blk * kBlockSpans;
            for (uint32_t s0 = 0; s0 < lim_s; s0 += kSumLoads * kPlaceThreads) {
                uint64_t v[kSumLoads];
#pragma unroll
                for (uint32_t u = 0; u < kSumLoads; u++) {
                    const uint32_t s = s0 + u * kPlaceThreads + threadIdx.x;
                    v[u] = so.cnt[s < lim_s ? s : 0u];
                }
#pragma unroll
                for (uint32_t u = 0; u < kSumLoads; u++) part += s0 + u * kPlaceThreads + threadIdx.x < lim_s ? v[u] : 0u;
            }
            part = wave_sum64(part);
            if (lane == 0) pre[wave] = part;
            __syncthreads();
#pragma unroll
            for (uint32_t w = 0; w < kPlaceWaves; w++) before += pre[w];
            __syncthreads();  // pre[] is rewritten by the next block
        }
        const uint64_t my_c = my_in ? c_ld : 0u;
        const uint32_t my_nh = my_in ? nh_ld : 0u, my_ovf = my_in ? ovf_ld : kNone;
        if (wave == 0) {
            // the block's span counts, their prefix, and the block's place by look-back
            const uint64_t c = my_c;
            const uint32_t nh = my_nh, ovf = my_ovf;
            span_nh[lane] = nh;
            span_ovf[lane] = ovf;
            span_cls[lane] = c == 0 ? 0u : (ovf == kNone && nh <= kFastRecs) ? 1u : 2u;
            const uint64_t inc = wave_incl_scan64(c);
            const uint64_t total = ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(inc >> 32), 63) << 32) |
                                   __builtin_amdgcn_readlane((uint32_t)inc, 63);
            if (direct && lane == 0 && blk == n_blocks - 1) *d_count = before + total;
            if (!direct && lane == 0) {
                const uint64_t v = total > kValueMask ? kValueMask : total;
                __hip_atomic_store(&ts.word[blk], tagE | ((blk == 0 ? kFlagInc : kFlagAgg) << 42) | v,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            uint64_t excl = before;
            if (!direct && blk > 0) {
                int64_t j = (int64_t)blk - 1;
                const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
                for (;;) {
                    const int64_t idx = j - (int64_t)lane;
                    uint64_t wd = tagE | (kFlagInc << 42);  // before block 0: prefix 0
                    if (idx >= 0) wd = __hip_atomic_load(&ts.word[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t flag = (uint32_t)(wd >> 42) & 3u;
                    const bool ready = (wd >> 44) == epoch && flag != 0;
                    const bool isinc = ready && flag == kFlagInc;
                    const uint64_t incm = __ballot(isinc);
                    const uint32_t first = incm ? (uint32_t)__builtin_ctzll(incm) : 64u;
                    const uint64_t need = first >= 63 ? ~0ull : ((2ull << first) - 1ull);
                    if (__ballot(!ready) & need) {
                        if (__builtin_amdgcn_s_memrealtime() - t0 > kWaitTicks) {  // never expected
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
                    uint64_t v = excl + total;
                    if (v > kValueMask) {
                        __hip_atomic_fetch_or(&ts.ctrl[3], 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                        v = kValueMask;
                    }
                    __hip_atomic_store(&ts.word[blk], tagE | (kFlagInc << 42) | v, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            span_off[lane] = excl + inc - c;
        }
        __syncthreads();
        if (wave == 0) {
            // spans with a few records and no overflow: one lane each, all records'
            // loads in flight at once
            if (span_cls[lane] == 1) {
                const uint64_t a = (uint64_t)my_sp << span_log2;
                const uint32_t nh = my_nh;
                uint64_t o = span_off[lane];
#pragma unroll
                for (uint32_t k = 0; k < kFastRecs; k++) {
                    if (k >= nh) break;
                    const uint64_t s = a + (my_rec[k] & 0xffffu);
                    const uint32_t ki = (uint32_t)(my_rec[k] >> 16) & 0xffffu, f = (uint32_t)(my_rec[k] >> 32);
                    if (ki == 1) {  // one terminal with one id: the record holds the id
                        if (o + 1 <= cap) keys[o] = (s << 32) | f;
                        o += 1;
                    } else if (ki && ki < kRecMulti) {  // one terminal: its ids, in order
                        if (o + ki <= cap)
                            for (uint32_t x = 0; x < ki; x++) keys[o + x] = (s << 32) | t.out_ids[f + x];
                        o += ki;
                    } else {  // several terminals: walk again from the first one (or the root)
                        const uint64_t end = end_of(s);
                        const uint32_t q0 = ki ? f : 0u;
                        const uint64_t i0 = s + (ki ? (ki & (kRecMulti - 1)) : 0u);
                        const uint32_t c = T.walk_from(q0, text, i0, end).cnt;
                        if (c && o + c <= cap) T.emit_walk(text, s, end, keys, o, c, q0, i0);
                        o += c;
                    }
                }
            }
        }
        // the other spans: every wave takes every kPlaceWaves-th (wave 0 after its lanes'
        // spans above)
        for (uint32_t i = wave; i < kBlockSpans; i += kPlaceWaves) {
            const uint32_t sp = blk * kBlockSpans + i;
            if (span_cls[i] != 2) continue;
            uint64_t run = span_off[i];
            const uint64_t a = (uint64_t)sp << span_log2;
            const uint64_t b = a + span_len < n ? a + span_len : n;
            const uint32_t nh = span_nh[i], ovf = span_ovf[i];
            // records kRecRounds x 64 at a time: every load of a round is issued before
            // any of its results is used, so a span with many records pays a few memory
            // latencies per 256 records rather than per 64
            for (uint32_t h0 = 0; h0 < nh; h0 += 64 * kRecRounds) {
                uint64_t rec[kRecRounds];
#pragma unroll
                for (uint32_t u = 0; u < kRecRounds; u++) {
                    const uint32_t h = h0 + 64 * u + lane;
                    rec[u] = h < nh ? so.rec[((size_t)sp << so.rec_log2) + h] : 0;
                }
#pragma unroll
                for (uint32_t u = 0; u < kRecRounds; u++) {
                    if (h0 + 64 * u >= nh) break;  // wave-uniform
                    const bool on = h0 + 64 * u + lane < nh;
                    const uint64_t s = a + (rec[u] & 0xffffu);
                    const uint32_t ki = (uint32_t)(rec[u] >> 16) & 0xffffu, f = (uint32_t)(rec[u] >> 32);
                    uint64_t end = 0;
                    const bool multi = ki == 0 || ki >= kRecMulti;
                    const uint32_t q0 = ki ? f : 0u;
                    const uint64_t i0 = s + (ki ? (ki & (kRecMulti - 1)) : 0u);
                    uint32_t c = on ? ki : 0u;
                    if (on && multi) {  // several terminals: walk again from the first one (or the root)
                        end = end_of(s);
                        c = T.walk_from(q0, text, i0, end).cnt;
                    }
                    const uint32_t incl = wave_incl_scan(c);
                    const uint64_t o = run + incl - c;
                    if (c && o + c <= cap) {
                        if (ki == 1) {
                            keys[o] = (s << 32) | f;
                        } else if (!multi) {
                            const uint64_t hi = s << 32;
                            for (uint32_t x = 0; x < c; x++) keys[o + x] = hi | t.out_ids[f + x];
                        } else {
                            T.emit_walk(text, s, end, keys, o, c, q0, i0);
                        }
                    }
                    run += __builtin_amdgcn_readlane(incl, 63);
                }
            }
            if (ovf != kNone) {
                // more matching starts than records: walk every start from the first one
                // not recorded, 64 at a time, from the root in HBM
                const uint64_t lim = n >= t.min_len ? n - t.min_len + 1 : 0;
                const uint64_t top = b < lim ? b : lim;
                for (uint64_t s0 = a + ovf; s0 < top; s0 += 64) {
                    const uint64_t s = s0 + lane;
                    const bool on = s < top;
                    const uint64_t end = on ? end_of(s) : 0;
                    const uint32_t c = on ? T.walk_from(0, text, s, end).cnt : 0;
                    const uint32_t incl = wave_incl_scan(c);
                    const uint64_t o = run + incl - c;
                    if (c && o + c <= cap) T.emit_walk(text, s, end, keys, o, c);
                    run += __builtin_amdgcn_readlane(incl, 63);
                }
            }
        }
        __syncthreads();  // span_off is rewritten by the next block
    }
    if (direct) {
        if (n_blocks == 0 && blockIdx.x == 0 && threadIdx.x == 0) *d_count = 0;
        return;
    }
    // last workgroup out: writes the count, resets the ticket, advances the epoch
    if (threadIdx.x == 0) {
        const uint32_t done = __hip_atomic_fetch_add(&ts.ctrl[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (done == gridDim.x - 1) {
            uint64_t total = 0;
            if (n_blocks) {
                // the last block's inclusive prefix: every block is published by now, so
                // this wait ends as soon as the word is visible
                const uint64_t want = tagE | (kFlagInc << 42);
                const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
                for (;;) {
                    const uint64_t wd = __hip_atomic_load(&ts.word[n_blocks - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if ((wd & ~kValueMask) == want) {
                        total = wd & kValueMask;
                        break;
                    }
                    if (__builtin_amdgcn_s_memrealtime() - t0 > kWaitTicks) {
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

template <int LAYOUT, bool PACK2, bool SEG, int FM, bool MERGED, uint32_t LB>
int launch_one(const DevTable &t, const uint8_t *text, uint64_t n, const uint64_t *offsets, uint32_t n_packets,
               uint64_t *keys, uint64_t cap, uint64_t *d_count, const SpanOut &so, const TileState &ts,
               const uint64_t *sizes, uint32_t grid, uint32_t span_log2, hipStream_t s) {
    const uint64_t n_spans = (n + (1ull << span_log2) - 1) >> span_log2;
    const uint64_t n_blocks = (n_spans + kBlockSpans - 1) / kBlockSpans;
    auto kc = scan_count<LAYOUT, PACK2, SEG, FM, MERGED, LB>;
    auto kp = place_emit<LAYOUT, SEG, MERGED>;
    static std::once_flag once;
    static int cus = 0, per_cu = 1, per_cu_p = 1;
    std::call_once(once, [&] {
        int dev = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (cus <= 0) cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kc, kThreads, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu_p, kp, kPlaceThreads, 0) != hipSuccess || per_cu_p < 1)
            per_cu_p = 1;
    });
    // count: as many workgroups as are resident at once, no more than it takes to give
    // every wave a span (n is the upper bound when sizes come from device memory)
    uint64_t gc = grid ? grid : (uint64_t)cus * (uint32_t)per_cu;
    const uint64_t need = (n_spans + kWaves - 1) / kWaves;
    if (gc > need) gc = need;
    if (gc == 0) gc = 1;
    uint64_t gp = (uint64_t)cus * (uint32_t)per_cu_p;
    if (gp > n_blocks) gp = n_blocks;
    if (gp == 0) gp = 1;
    SpanOut o = so;
    if (!o.rec_log2) o.rec_log2 = rec_cap_log2(span_log2);  // a caller may fix fewer records per span
    kc<<<(uint32_t)gc, kThreads, 0, s>>>(t, text, n, offsets, n_packets, o, sizes, span_log2);
    kp<<<(uint32_t)gp, kPlaceThreads, 0, s>>>(t, text, n, offsets, n_packets, keys, cap, d_count, o, ts, sizes,
                                               span_log2);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Positions per thread: 16 bytes a lane and step when asked for and the form allows it
// (the sampled form reads a lane's 32 bytes), else 32.
template <int LAYOUT, bool PACK2, bool SEG, int FM, bool MERGED>
int launch_lanes(uint32_t lane_bytes, const DevTable &t, const uint8_t *text, uint64_t n, const uint64_t *offsets,
                 uint32_t n_packets, uint64_t *keys, uint64_t cap, uint64_t *d_count, const SpanOut &so,
                 const TileState &ts, const uint64_t *sizes, uint32_t grid, uint32_t span_log2, hipStream_t s) {
    if constexpr (!(FM == FM_K4 && !PACK2)) {
        if (lane_bytes == 16)
            return launch_one<LAYOUT, PACK2, SEG, FM, MERGED, 16>(t, text, n, offsets, n_packets, keys, cap, d_count,
                                                                  so, ts, sizes, grid, span_log2, s);
    }
    return launch_one<LAYOUT, PACK2, SEG, FM, MERGED, 32>(t, text, n, offsets, n_packets, keys, cap, d_count, so, ts,
                                                          sizes, grid, span_log2, s);
}

// Every kernel instance for one kind of table (plain or compressed).
template <bool MERGED>
int launch_tiled_t(const DevTable &t, const uint8_t *text, uint64_t n, const uint64_t *offsets, uint32_t n_packets,
                   uint64_t *keys, uint64_t cap, uint64_t *d_count, const SpanOut &so, const TileState &ts,
                   const uint64_t *sizes, uint32_t grid, uint32_t span_log2, uint32_t lane_bytes, hipStream_t s) {
    if (span_log2 < kMinSpanLog2 || span_log2 > kMaxSpanLog2) return -1;
    const bool seg = offsets != nullptr;
    const bool narrow = t.layout == LAYOUT_NARROW;
    const bool pack2 = t.pack2 != 0;
    const int fm = t.filter_k == 0 ? FM_ROOT : t.sampled ? FM_K4 : t.exact ? FM_EXACT : FM_GEN;
#define PFAC_L(LA, P2, SG, F) \
    return launch_lanes<LA, P2, SG, F, MERGED>(lane_bytes, t, text, n, offsets, n_packets, keys, cap, d_count, so, ts, \
                                               sizes, grid, span_log2, s)
    // two-bit symbols: the exact, hashed and root-only forms; bytes: sampled, hashed, root-only
#define PFAC_FM2(LA, SG)                                       \
    do {                                                       \
        if (fm == FM_ROOT) PFAC_L(LA, true, SG, FM_ROOT);      \
        if (fm == FM_EXACT) PFAC_L(LA, true, SG, FM_EXACT);    \
        PFAC_L(LA, true, SG, FM_GEN);                          \
    } while (0)
#define PFAC_FM(LA, SG)                                        \
    do {                                                       \
        if (fm == FM_ROOT) PFAC_L(LA, false, SG, FM_ROOT);     \
        if (fm == FM_GEN) PFAC_L(LA, false, SG, FM_GEN);       \
        PFAC_L(LA, false, SG, FM_K4);                          \
    } while (0)
    if (narrow) {
        if (pack2) { if (seg) PFAC_FM2(LAYOUT_NARROW, true); else PFAC_FM2(LAYOUT_NARROW, false); }
        else { if (seg) PFAC_FM(LAYOUT_NARROW, true); else PFAC_FM(LAYOUT_NARROW, false); }
    } else {
        if (seg) PFAC_FM(LAYOUT_WIDE, true);
        PFAC_FM(LAYOUT_WIDE, false);
    }
#undef PFAC_FM
#undef PFAC_FM2
#undef PFAC_L
}

}  // namespace

}  // namespace pfac
