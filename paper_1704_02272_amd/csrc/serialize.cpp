// Serialized automata (pfac_save / pfac_load) and the key-to-packet map of batch keys.
//
// A saved automaton is the table of Section 3.1 (first-child offset and child bitmap per
// node, breadth-first), the pattern ids ending at each node, the patterns themselves and
// the tuning in force, behind a fixed header:
//
//   offset  size  field
//        0     8  magic "PFACAUT1"
//        8     4  format version (1)
//       12     4  header bytes (64)
//       16     4  alphabet              20  4  patterns
//       24     4  nodes                 28  4  longest pattern
//       32     4  shortest pattern      36  4  merge levels of the table (pfac_build_ex)
//       40     4  tuning: algo | span log2 << 8 | root depth << 16 | filter key << 24
//       44     4  tuning: grid | positions per thread << 24 (lane bytes 16 or 32; 0 = 32)
//       48     8  payload bytes
//       56     8  FNV-1a 64 of bytes 0..55 and of the payload
//
// then, each section padded to 8 bytes: pattern offsets (u64, patterns + 1), pattern
// bytes, first-child offsets (u32, nodes), bitmaps (u64, nodes x words), id offsets
// (u32, nodes + 1), ids (u32, patterns). All little-endian.
//
// The table the scans walk (plain or compressed, Section 3.2) is derived again on load.
// Loading checks sizes and the checksum, then that the arrays are the breadth-first
// trie of the stored patterns: every first-child offset is 1 + the children of all
// earlier nodes (0 for a node without children), every leaf ends a pattern, every id
// appears once, and each pattern's path under Eq. 1 ends at the node that lists it.
// A table that passes is the one pfac_build makes from those patterns, so every scan
// over it stays inside its arrays. Anything else is PFAC_EFORMAT.
#include <string.h>

#include <algorithm>
#include <new>
#include <stdexcept>
#include <vector>

#include "pfac.h"
#include "pfac_impl.h"
#include "scan_internal.h"

namespace {

constexpr char kMagic[8] = {'P', 'F', 'A', 'C', 'A', 'U', 'T', '1'};
constexpr uint32_t kVersion = 1;
constexpr uint32_t kHeader = 64;

uint64_t fnv1a(uint64_t h, const uint8_t *p, uint64_t n) {
    for (uint64_t i = 0; i < n; i++) {
        h ^= p[i];
        h *= 0x100000001b3ull;
    }
    return h;
}
constexpr uint64_t kFnvBasis = 0xcbf29ce484222325ull;

inline uint64_t pad8(uint64_t n) { return (n + 7) & ~7ull; }

template <typename T>
void put(uint8_t *b, uint64_t at, T v) {
    memcpy(b + at, &v, sizeof(T));
}
template <typename T>
T get(const uint8_t *b, uint64_t at) {
    T v;
    memcpy(&v, b + at, sizeof(T));
    return v;
}

struct Sizes {
    uint64_t pat_off, pat_bytes, first, bitmap, out_first, out_ids, total;
};

Sizes section_sizes(uint64_t n_pats, uint64_t n_nodes, uint64_t nbw, uint64_t pat_bytes) {
    Sizes z;
    z.pat_off = (n_pats + 1) * 8;
    z.pat_bytes = pad8(pat_bytes);
    z.first = pad8(n_nodes * 4);
    z.bitmap = n_nodes * nbw * 8;
    z.out_first = pad8((n_nodes + 1) * 4);
    z.out_ids = pad8(n_pats * 4);
    z.total = z.pat_off + z.pat_bytes + z.first + z.bitmap + z.out_first + z.out_ids;
    return z;
}

inline uint32_t popc64(uint64_t x) { return (uint32_t)__builtin_popcountll(x); }

// The structural checks described at the top; fills depth_start. True when they hold.
bool valid_trie(pfac_automaton *a) {
    const uint32_t Q = a->n_nodes, N = a->n_pats, W = a->nbw;
    if (Q == 0) return false;
    // bits at or past the alphabet must be clear
    for (uint32_t q = 0; q < Q; q++)
        for (uint32_t w = 0; w < W; w++) {
            const uint32_t lo = 64 * w;
            const uint64_t b = a->bitmap[(size_t)q * W + w];
            if (lo >= a->alphabet ? b != 0 : (a->alphabet - lo < 64 && (b >> (a->alphabet - lo)) != 0))
                return false;
        }
    // breadth-first offsets: children of node q start right after those of nodes < q
    uint64_t next = 1;
    std::vector<uint32_t> depth(Q, 0);
    for (uint32_t q = 0; q < Q; q++) {
        uint32_t deg = 0;
        for (uint32_t w = 0; w < W; w++) deg += popc64(a->bitmap[(size_t)q * W + w]);
        if (deg == 0) {
            if (a->first_child[q] != 0) return false;
        } else {
            if (a->first_child[q] != next || next + deg > Q) return false;
            for (uint32_t k = 0; k < deg; k++) depth[next + k] = depth[q] + 1;
        }
        next += deg;
        if (q + 1 < Q && next <= q + 1) return false;  // node q+1 must be someone's child
    }
    if (next != Q) return false;
    // ids: out_first non-decreasing from 0 to N, every id once
    if (a->out_first[0] != 0 || a->out_first[Q] != N) return false;
    for (uint32_t q = 0; q < Q; q++)
        if (a->out_first[q + 1] < a->out_first[q]) return false;
    std::vector<uint32_t> node_of(N, UINT32_MAX);
    for (uint32_t q = 0; q < Q; q++) {
        const uint32_t f = a->out_first[q], e = a->out_first[q + 1];
        for (uint32_t x = f; x < e; x++) {
            const uint32_t id = a->out_ids[x];
            if (id >= N || node_of[id] != UINT32_MAX) return false;
            if (x > f && a->out_ids[x - 1] >= id) return false;  // ascending per node
            node_of[id] = q;
        }
        // a node without children must end a pattern (the root only when nothing is stored)
        if (a->first_child[q] == 0 && f == e && !(q == 0 && N == 0)) return false;
    }
    if (N == 0) {
        if (Q != 1) return false;
    }
    // each pattern's path (Eq. 1) ends at the node that lists it; lengths fit the header
    uint32_t minl = UINT32_MAX, maxl = 0;
    for (uint32_t j = 0; j < N; j++) {
        const uint64_t len = a->pat_off[j + 1] - a->pat_off[j];
        if (len == 0 || len > pfac::kMaxPatternLen) return false;
        minl = std::min<uint32_t>(minl, (uint32_t)len);
        maxl = std::max<uint32_t>(maxl, (uint32_t)len);
        const uint8_t *p = a->pat_bytes.data() + a->pat_off[j];
        uint32_t q = 0;
        for (uint64_t i = 0; i < len; i++) {
            const uint32_t c = p[i];
            if (c >= a->alphabet) return false;
            const uint64_t *b = &a->bitmap[(size_t)q * W];
            if (!((b[c >> 6] >> (c & 63)) & 1)) return false;
            uint32_t r = 0;
            for (uint32_t w = 0; w < (c >> 6); w++) r += popc64(b[w]);
            r += popc64(b[c >> 6] & ((1ull << (c & 63)) - 1));
            q = a->first_child[q] + r;
        }
        if (q != node_of[j]) return false;
    }
    if (N == 0) minl = 0;
    if (minl != a->min_len || maxl != a->max_len) return false;
    // first node of every depth (the depths are non-decreasing in breadth-first order)
    a->depth_start.assign(1, 0);
    for (uint32_t q = 1; q < Q; q++) {
        if (depth[q] < depth[q - 1]) return false;
        while (a->depth_start.size() <= depth[q]) a->depth_start.push_back(q);
    }
    if (a->depth_start.size() != (size_t)maxl + 1) return false;
    a->depth_start.push_back(Q);
    while (a->depth_start.size() < (size_t)maxl + 3) a->depth_start.push_back(Q);
    return true;
}

}  // namespace

extern "C" int pfac_save(const pfac_automaton *a, uint8_t *buf, uint64_t cap, uint64_t *size) {
    if (!a || !size) return PFAC_EINVAL;
    const Sizes z = section_sizes(a->n_pats, a->n_nodes, a->nbw, a->pat_bytes.size());
    const uint64_t need = kHeader + z.total;
    *size = need;
    if (!buf || cap < need) return PFAC_ECAPACITY;
    memset(buf, 0, need);
    memcpy(buf, kMagic, 8);
    put<uint32_t>(buf, 8, kVersion);
    put<uint32_t>(buf, 12, kHeader);
    put<uint32_t>(buf, 16, a->alphabet);
    put<uint32_t>(buf, 20, a->n_pats);
    put<uint32_t>(buf, 24, a->n_nodes);
    put<uint32_t>(buf, 28, a->max_len);
    put<uint32_t>(buf, 32, a->min_len);
    put<uint32_t>(buf, 36, a->merge_levels);
    put<uint32_t>(buf, 40, (a->algo & 0xff) | ((a->span_log2 & 0xff) << 8) | ((a->req_depth & 0xff) << 16) |
                               ((a->req_k & 0xff) << 24));
    put<uint32_t>(buf, 44, (a->grid & 0xffffffu) | ((a->lane_bytes & 0xffu) << 24));
    put<uint64_t>(buf, 48, z.total);
    uint64_t at = kHeader;
    memcpy(buf + at, a->pat_off.data(), z.pat_off);
    at += z.pat_off;
    if (!a->pat_bytes.empty()) memcpy(buf + at, a->pat_bytes.data(), a->pat_bytes.size());
    at += z.pat_bytes;
    memcpy(buf + at, a->first_child.data(), (size_t)a->n_nodes * 4);
    at += z.first;
    memcpy(buf + at, a->bitmap.data(), z.bitmap);
    at += z.bitmap;
    memcpy(buf + at, a->out_first.data(), ((size_t)a->n_nodes + 1) * 4);
    at += z.out_first;
    if (a->n_pats) memcpy(buf + at, a->out_ids.data(), (size_t)a->n_pats * 4);
    uint64_t h = fnv1a(kFnvBasis, buf, 56);
    h = fnv1a(h, buf + kHeader, z.total);
    put<uint64_t>(buf, 56, h);
    return PFAC_OK;
}

extern "C" int pfac_load(const uint8_t *buf, uint64_t size, pfac_automaton **out) {
    if (!out) return PFAC_EINVAL;
    *out = nullptr;
    if (!buf) return PFAC_EINVAL;
    if (size < kHeader || memcmp(buf, kMagic, 8) != 0) return PFAC_EFORMAT;
    if (get<uint32_t>(buf, 8) != kVersion || get<uint32_t>(buf, 12) != kHeader) return PFAC_EFORMAT;
    const uint32_t alphabet = get<uint32_t>(buf, 16), n_pats = get<uint32_t>(buf, 20),
                   n_nodes = get<uint32_t>(buf, 24), maxl = get<uint32_t>(buf, 28), minl = get<uint32_t>(buf, 32),
                   levels = get<uint32_t>(buf, 36), tune = get<uint32_t>(buf, 40), grid = get<uint32_t>(buf, 44);
    const uint64_t payload = get<uint64_t>(buf, 48);
    if (alphabet < 1 || alphabet > 256 || levels > pfac::kMaxMergeLevels) return PFAC_EFORMAT;
    const uint32_t nbw = (alphabet + 63) / 64;
    if (n_nodes == 0 || n_nodes > pfac::kMaxNodes || maxl > pfac::kMaxPatternLen) return PFAC_EFORMAT;
    if (payload != size - kHeader) return PFAC_EFORMAT;
    // the pattern bytes' size comes from the last pattern offset: check the offsets'
    // section fits before reading it
    const uint64_t off_bytes = ((uint64_t)n_pats + 1) * 8;
    if (off_bytes > payload) return PFAC_EFORMAT;
    const uint64_t total_pat = get<uint64_t>(buf, kHeader + off_bytes - 8);
    if (total_pat > payload) return PFAC_EFORMAT;
    const Sizes z = section_sizes(n_pats, n_nodes, nbw, total_pat);
    if (z.total != payload) return PFAC_EFORMAT;
    uint64_t h = fnv1a(kFnvBasis, buf, 56);
    h = fnv1a(h, buf + kHeader, payload);
    if (h != get<uint64_t>(buf, 56)) return PFAC_EFORMAT;
    pfac_automaton *a = new (std::nothrow) pfac_automaton();
    if (!a) return PFAC_ENOMEM;
    try {
        a->alphabet = alphabet;
        a->n_pats = n_pats;
        a->n_nodes = n_nodes;
        a->max_len = maxl;
        a->min_len = minl;
        a->nbw = nbw;
        a->merge_levels = levels;
        uint64_t at = kHeader;
        a->pat_off.resize((size_t)n_pats + 1);
        memcpy(a->pat_off.data(), buf + at, off_bytes);
        at += z.pat_off;
        if (a->pat_off[0] != 0) throw 1;
        for (uint32_t j = 0; j < n_pats; j++)
            if (a->pat_off[j + 1] < a->pat_off[j]) throw 1;
        a->pat_bytes.assign(buf + at, buf + at + total_pat);
        at += z.pat_bytes;
        a->first_child.resize(n_nodes);
        memcpy(a->first_child.data(), buf + at, (size_t)n_nodes * 4);
        at += z.first;
        a->bitmap.resize((size_t)n_nodes * nbw);
        memcpy(a->bitmap.data(), buf + at, z.bitmap);
        at += z.bitmap;
        a->out_first.resize((size_t)n_nodes + 1);
        memcpy(a->out_first.data(), buf + at, ((size_t)n_nodes + 1) * 4);
        at += z.out_first;
        a->out_ids.resize(n_pats);
        if (n_pats) memcpy(a->out_ids.data(), buf + at, (size_t)n_pats * 4);
        a->pat_len.resize(n_pats);
        for (uint32_t j = 0; j < n_pats; j++) a->pat_len[j] = (uint32_t)(a->pat_off[j + 1] - a->pat_off[j]);
        if (!valid_trie(a)) throw 1;
        // tuning: algo, grid, span and the LDS image's root depth / key as saved, when
        // they are valid for these patterns
        a->algo = tune & 0xff;
        a->span_log2 = (tune >> 8) & 0xff;
        a->req_depth = (tune >> 16) & 0xff;
        a->req_k = tune >> 24;
        a->grid = grid & 0xffffffu;
        const uint32_t lb = grid >> 24;
        if (lb != 0 && lb != 16 && lb != 32) throw 1;
        a->lane_bytes = lb == 16 ? 16u : 32u;
        if (a->algo > PFAC_ALGO_TILED) throw 1;
        if (a->span_log2 && (a->span_log2 < pfac::kMinSpanLog2 || a->span_log2 > pfac::kMaxSpanLog2)) throw 1;
        if (n_pats) {
            const bool pack2 = alphabet <= 4;
            const uint32_t dmax = std::min(minl, pack2 ? 8u : 2u), kmax = std::min(maxl, pack2 ? 16u : 4u);
            const uint32_t d = a->req_depth ? a->req_depth : dmax;
            if (a->req_depth > dmax || (a->req_k && (a->req_k < d || a->req_k > kmax))) throw 1;
        } else if (a->req_depth || a->req_k) {
            throw 1;
        }
        pfac::finish_automaton(a);
    } catch (const std::bad_alloc &) {
        delete a;
        return PFAC_ENOMEM;
    } catch (const std::length_error &) {
        delete a;
        return PFAC_EFORMAT;
    } catch (int) {
        delete a;
        return PFAC_EFORMAT;
    }
    *out = a;
    return PFAC_OK;
}

extern "C" int pfac_key_to_packet(const uint64_t *h_keys, uint64_t n_keys, const uint64_t *h_offsets,
                                  uint32_t n_pkts, uint32_t *pkt, uint32_t *start, uint32_t *ids) {
    if (n_keys == 0) return PFAC_OK;
    if (!h_keys || !h_offsets || !pkt || !start || !ids) return PFAC_EINVAL;
    const uint64_t *lo = h_offsets, *hi = h_offsets + n_pkts + 1;
    for (uint64_t i = 0; i < n_keys; i++) {
        const uint64_t s = h_keys[i] >> 32;
        // last packet whose first byte is <= s and that is not empty past s
        const uint64_t *u = std::upper_bound(lo, hi, s);
        if (u == lo || u == hi) return PFAC_EINVAL;  // before the batch or past its end
        const uint32_t p = (uint32_t)(u - lo - 1);
        pkt[i] = p;
        start[i] = (uint32_t)(s - h_offsets[p]);
        ids[i] = (uint32_t)h_keys[i];
    }
    return PFAC_OK;
}
