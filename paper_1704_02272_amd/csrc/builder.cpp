// Host-side construction of the compressed trie (Section 3.1) and of the device images.
//
// Patterns are sorted bytewise (shorter first when one is a prefix of another, pattern
// id breaking ties) and the trie is built breadth-first, level by level. Because the
// patterns are sorted, the patterns under any trie node form one contiguous run of the
// sorted order; a node is kept as that run, and its children are the maximal sub-runs
// that agree on the next byte, taken in increasing byte order. Numbering nodes in the
// order they are created is then the breadth-first order of Section 3.1, and the first
// child of a node is simply the index its first sub-run receives (Eq. 1's offset).
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <stdexcept>

#include "pfac.h"
#include "pfac_impl.h"
#include "scan_internal.h"

namespace pfac {
namespace {

inline uint32_t popc64(uint64_t x) { return (uint32_t)__builtin_popcountll(x); }

struct Run {
    uint32_t lo, hi;  // range of the sorted pattern order
};

// Key of the first `d` symbols of p in the root image: lexicographic order, i.e. the
// first symbol in the most significant position, `bits` bits per symbol.
inline uint32_t root_key(const uint8_t *p, uint32_t d, uint32_t bits) {
    uint32_t k = 0;
    for (uint32_t i = 0; i < d; i++) k = (k << bits) | p[i];
    return k;
}

// Key of the first k symbols of p in the prefix filter. Byte symbols: little-endian
// bytes (symbol 0 in bits 0..7), which is how the kernels read four text bytes as one
// 32-bit word. Two-bit symbols: first symbol most significant.
inline uint32_t filter_key(const uint8_t *p, uint32_t k, bool pack2) {
    uint32_t key = 0;
    if (pack2) {
        for (uint32_t i = 0; i < k; i++) key = (key << 2) | p[i];
    } else {
        for (uint32_t i = 0; i < k; i++) key |= (uint32_t)p[i] << (8 * i);
    }
    return key;
}

void build_lds_image(pfac_automaton *a, const std::vector<const uint8_t *> &P, uint32_t reqD, uint32_t reqK) {
    DevTable &t = a->shape;
    t.pack2 = a->alphabet <= 4 ? 1 : 0;
    const uint32_t bits = t.pack2 ? 2 : 8;
    if (a->n_pats == 0) {
        t.root_depth = t.root_bits = t.root_base = 0;
        t.filter_k = t.filter_log2 = t.has_short = t.sampled = t.exact = 0;
        t.lds_words = t.root_word = t.rank_word = t.short_word = 0;
        a->lds_image.clear();
        return;
    }
    const uint32_t dmax = t.pack2 ? 8 : 2;
    const uint32_t kmax = t.pack2 ? 16 : 4;
    const uint32_t D = reqD ? reqD : std::min(a->min_len, dmax);
    t.root_depth = D;
    t.root_bits = D * bits;
    t.root_base = a->depth_start[D];
    const uint32_t root_nbits = 1u << t.root_bits;
    const uint32_t root_words = std::max<uint32_t>(1, root_nbits / 32);
    const uint32_t rank_words = (root_words + 1) / 2;  // one u16 per root word
    // Filter key length K: patterns of length >= K are tested by their K-gram in the
    // hashed filter, shorter ones by their D-gram in the short bitmap. K minimizes the
    // estimated pass rate on uniform text: the short D-grams' share of all D-grams, plus
    // the long K-grams' false-positive share of the filter bits (one bit per key), plus
    // their true share of all K-grams. Ties go to the longer key.
    const uint32_t kcap = std::min(kmax, a->max_len);
    // Estimated pass rate of a hashed filter with key length k (k == D: the root image
    // alone). Two-bit symbols skip k == D + 1 and D + 2, which are the exact form below.
    auto estimate = [&](uint32_t k) {
        std::vector<uint32_t> sk, lk;
        for (uint32_t j = 0; j < a->n_pats; j++) {
            if (a->pat_len[j] < k) sk.push_back(root_key(P[j], D, bits));
            else lk.push_back(filter_key(P[j], k, t.pack2));
        }
        std::sort(sk.begin(), sk.end());
        sk.erase(std::unique(sk.begin(), sk.end()), sk.end());
        std::sort(lk.begin(), lk.end());
        lk.erase(std::unique(lk.begin(), lk.end()), lk.end());
        const double space = std::pow((double)a->alphabet, (double)k);
        double est = (double)sk.size() / root_nbits + (double)lk.size() / space;
        if (k > D) est += (double)lk.size() / (double)(1u << kMaxFilterLog2) * (double)lk.size() / (double)(1u << kFilter2Log2);
        return est;
    };
    uint32_t K = D;
    double best = 1e30;
    for (uint32_t k = reqK ? reqK : D; k <= (reqK ? reqK : kcap); k++) {
        if (t.pack2 && (k == D + 1 || k == D + 2)) continue;  // the exact form's keys
        const double est = estimate(k);
        if (est <= best * 1.001) {
            best = est;
            K = k;
        }
    }
    // Two-bit symbols: the exact form (the trie's first D + E levels, E = 1 or 2, as a
    // direct bitmap over (D+E)-symbol keys: one cheap probe per start) when asked for (a
    // key of D + 1 or D + 2 symbols), and by default when its pass rate (the (D+E)-prefixes
    // plus every extension of a whole pattern shorter than D + E) is close to the best
    // hashed filter's. Keys of D + E symbols of each pattern; a pattern of D + e symbols
    // (e < E) stands for all its 4^(E-e) extensions.
    auto exact_keys = [&](uint32_t E) {
        std::vector<uint32_t> keys;
        for (uint32_t j = 0; j < a->n_pats; j++) {
            const uint32_t L = a->pat_len[j];
            if (L >= D + E) {
                keys.push_back(root_key(P[j], D + E, bits));
            } else {
                const uint32_t e = L - D, free = 2 * (E - e);
                const uint32_t base = root_key(P[j], L, bits) << free;
                for (uint32_t x = 0; x < (1u << free); x++) keys.push_back(base | x);
            }
        }
        std::sort(keys.begin(), keys.end());
        keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
        return keys;
    };
    uint32_t E = 0;
    if (t.pack2 && (reqK == D + 1 || reqK == D + 2)) E = reqK - D;
    if (t.pack2 && reqK == 0) {
        double e_best = 1e30;
        for (uint32_t e = 1; e <= 2; e++) {
            const double est = (double)exact_keys(e).size() / (double)(1ull << (2 * (D + e)));
            if (est < e_best * 0.999) {
                e_best = est;
                E = e;
            }
        }
        if (!(e_best <= std::max(1.25 * best, best + 0.002))) E = 0;
    }
    if (E) {
        const uint32_t K1 = D + E, kbits = 2 * K1;
        const uint32_t fwords = std::max<uint32_t>(4, (1u << kbits) / 32);  // whole 16-byte units
        t.filter_k = K1;
        t.filter_log2 = kbits;
        t.has_short = 0;
        t.sampled = 0;
        t.exact = 1;
        t.root_word = fwords;
        t.rank_word = fwords + root_words;
        t.short_word = t.rank_word + rank_words;
        t.lds_words = t.short_word;
        a->lds_image.assign(t.lds_words, 0);
        uint32_t *img = a->lds_image.data();
        uint32_t *root = img + t.root_word;
        for (uint32_t j = 0; j < a->n_pats; j++) {
            const uint32_t key = root_key(P[j], D, bits);
            root[key >> 5] |= 1u << (key & 31);
        }
        for (uint32_t k1 : exact_keys(E)) img[k1 >> 5] |= 1u << (k1 & 31);
        uint16_t *rank = reinterpret_cast<uint16_t *>(img + t.rank_word);
        uint32_t run = 0;
        for (uint32_t w = 0; w < root_words; w++) {
            rank[w] = (uint16_t)run;
            run += (uint32_t)__builtin_popcount(root[w]);
        }
        if (run != a->depth_start[D + 1] - a->depth_start[D]) throw std::bad_alloc();
        return;
    }
    t.exact = 0;
    uint32_t flog2 = 0;
    std::vector<uint32_t> fkeys;
    bool any_short = false;
    if (K > D) {
        for (uint32_t j = 0; j < a->n_pats; j++) {
            if (a->pat_len[j] >= K) fkeys.push_back(filter_key(P[j], K, t.pack2));
            else any_short = true;
        }
        std::sort(fkeys.begin(), fkeys.end());
        fkeys.erase(std::unique(fkeys.begin(), fkeys.end()), fkeys.end());
        flog2 = kMaxFilterLog2;  // its LDS is reserved in any case: take all of it
    }
    t.filter_k = K > D ? K : 0;
    t.filter_log2 = flog2;
    t.has_short = any_short ? 1 : 0;
    // four-byte keys and no shorter pattern: the sampled layout
    t.sampled = (!t.pack2 && t.filter_k == 4 && !any_short) ? 1u : 0u;
    // the image holds the filter words the kernel copies to LDS offset 0
    const uint32_t filter_words = !flog2 ? 0 : t.sampled ? kSampledWords : kGeneralWords;
    t.root_word = filter_words;
    t.rank_word = filter_words + root_words;
    t.short_word = t.rank_word + rank_words;
    t.lds_words = t.short_word + (any_short ? root_words : 0);
    a->lds_image.assign(t.lds_words, 0);
    uint32_t *img = a->lds_image.data();
    uint32_t *root = img + t.root_word;
    uint32_t *shrt = img + t.short_word;
    for (uint32_t j = 0; j < a->n_pats; j++) {
        const uint32_t key = root_key(P[j], D, bits);
        root[key >> 5] |= 1u << (key & 31);
        if (any_short && a->pat_len[j] < K) shrt[key >> 5] |= 1u << (key & 31);
    }
    uint16_t *rank = reinterpret_cast<uint16_t *>(img + t.rank_word);
    uint32_t run = 0;
    for (uint32_t w = 0; w < root_words; w++) {
        rank[w] = (uint16_t)run;
        run += (uint32_t)__builtin_popcount(root[w]);
    }
    // every depth-D node is a D-prefix of some pattern (D <= shortest length)
    if (run != a->depth_start[D + 1] - a->depth_start[D]) throw std::bad_alloc();
    if (t.sampled) {
        for (uint32_t key : fkeys) filter4s_insert(img, key, kLdsS1, kS1Words, kLdsS2, kS2Words);
        for (uint32_t j = 0; j < a->n_pats; j++) {
            const uint8_t *p = P[j];  // every pattern has four or more bytes here
            filter3_insert(img, (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16), kFilterMul3, kLdsS3, kS3Words);
            filter3_insert(img, (uint32_t)p[1] | ((uint32_t)p[2] << 8) | ((uint32_t)p[3] << 16), kFilterMul3, kLdsS3, kS3Words);
        }
    } else {
        for (uint32_t key : fkeys) filter_insert(img, key, kLdsF1, kFilterWordsMax, 0, kFilter2Words);
    }
}

}  // namespace

// Path tails (see DevTable::tails), bottom-up over the breadth-first order: node q
// qualifies when it has one child c and c is a leaf, or c is not terminal and qualifies.
// The path's symbols are those of a pattern ending at its end node, from q's depth on.
void build_tails(pfac_automaton *a) {
    const uint32_t Q = a->n_nodes;
    a->dev_tails.assign((size_t)Q * 4, 0);
    if (a->pat_bytes.size() >= (1ull << 32)) return;  // offsets are 32-bit: no tails
    auto term = [&](uint32_t q) { return a->out_first[q + 1] > a->out_first[q]; };
    auto nchild = [&](uint32_t q) {
        uint32_t c = 0;
        for (uint32_t w = 0; w < a->nbw; w++) c += popc64(a->bitmap[(size_t)q * a->nbw + w]);
        return c;
    };
    uint32_t d = (uint32_t)a->depth_start.size() - 1;
    for (uint32_t q = Q; q-- > 0;) {
        while (d > 0 && a->depth_start[d] > q) d--;  // depth of q
        if (nchild(q) != 1) continue;
        const uint32_t c = a->first_child[q];
        uint32_t len = 0, leaf = 0;
        if (a->first_child[c] == 0) {
            len = 1;
            leaf = c;
        } else if (!term(c) && a->dev_tails[(size_t)c * 4 + 1]) {
            len = 1 + a->dev_tails[(size_t)c * 4 + 1];
            leaf = a->dev_tails[(size_t)c * 4 + 2];
        } else {
            continue;
        }
        const uint32_t j = a->out_ids[a->out_first[leaf]];
        a->dev_tails[(size_t)q * 4 + 0] = (uint32_t)(a->pat_off[j] + d);
        a->dev_tails[(size_t)q * 4 + 1] = len;
        a->dev_tails[(size_t)q * 4 + 2] = leaf;
    }
}

}  // namespace pfac

// Device copies are freed by the runtime (release_device_copies).
pfac_automaton::~pfac_automaton() { pfac::release_device_copies(this); }

namespace pfac {

int rebuild_lds_image(pfac_automaton *a, uint32_t D, uint32_t K) {
    if (!a || a->n_pats == 0) return (D || K) ? PFAC_EINVAL : PFAC_OK;
    const bool pack2 = a->alphabet <= 4;
    const uint32_t dmax = std::min(a->min_len, pack2 ? 8u : 2u);
    const uint32_t kmax = std::min(a->max_len, pack2 ? 16u : 4u);
    if (D > dmax) return PFAC_EINVAL;
    const uint32_t d = D ? D : dmax;
    if (K && (K < d || K > kmax)) return PFAC_EINVAL;
    std::vector<const uint8_t *> P(a->n_pats);
    for (uint32_t j = 0; j < a->n_pats; j++) P[j] = a->pat_bytes.data() + a->pat_off[j];
    try {
        build_lds_image(a, P, D, K);
    } catch (const std::bad_alloc &) {
        return PFAC_ENOMEM;
    }
    return PFAC_OK;
}

// Everything the scans need that follows from the trie and the patterns: the count of
// terminal nodes, the node images of HBM, the path tails and the LDS image (with the
// root depth and filter key the tuning asks for). Shared by building and loading.
void finish_automaton(pfac_automaton *a) {
    a->n_term = 0;
    for (uint32_t q = 0; q < a->n_nodes; q++)
        if (a->out_first[q + 1] > a->out_first[q]) a->n_term++;
    build_tails(a);    // over the trie
    build_records(a);  // the walked table; tails move onto its records
    // The device table. The compressed table (Section 3.2) is its records as they are,
    // with a path tail per record. The plain table collapses every unary tail: a node
    // below the root image's deepest possible level whose subtree is one path ending at
    // its only terminal (a tail head) keeps its own word, with the tail flag set and the
    // index of its tail record in place of the first child; the nodes of the path below
    // it are not stored. Nodes down to that level are all kept, so they keep their
    // breadth-first indices (the root image depends on them).
    std::vector<uint32_t> dfirst, dord;  // device first child (or tail index), node of each device record
    std::vector<uint8_t> dtail;
    a->dev_out_first.clear();
    a->dev_out_ids.clear();
    a->dev_tail_head.clear();  // plain table only (below)
    if (a->merge_levels) {
        const uint32_t R = a->n_rec;
        dfirst = a->rec_first;
        dtail.assign(R, 0);
        dord.resize(R);
        for (uint32_t x = 0; x < R; x++) dord[x] = x;
        a->dev_out_first = a->rank_first;
        a->dev_out_ids = a->rank_ids;
    } else {
        const uint32_t Q = a->n_nodes;
        const uint32_t dkeep = a->n_pats ? std::min(a->min_len, a->alphabet <= 4 ? 8u : 2u) : 0u;
        std::vector<uint32_t> depth(Q, 0), parent(Q, 0);
        for (uint32_t d = 0; d + 1 < a->depth_start.size(); d++)
            for (uint32_t q = a->depth_start[d]; q < a->depth_start[d + 1] && q < Q; q++) depth[q] = d;
        auto deg = [&](uint32_t q) {
            uint32_t c = 0;
            for (uint32_t w = 0; w < a->nbw; w++) c += popc64(a->bitmap[(size_t)q * a->nbw + w]);
            return c;
        };
        for (uint32_t q = 0; q < Q; q++)
            for (uint32_t i = 0, k = deg(q); i < k; i++) parent[a->first_child[q] + i] = q;
        auto tailed = [&](uint32_t q) { return a->dev_tails[(size_t)q * 4 + 1] != 0 && depth[q] >= dkeep; };
        std::vector<uint8_t> head(Q, 0), below(Q, 0);  // below: inside a head's path
        std::vector<uint32_t> nid(Q, 0);
        std::vector<uint32_t> heads;
        for (uint32_t q = 0; q < Q; q++) {
            if (q > 0) below[q] = head[parent[q]] || below[parent[q]];
            if (below[q]) continue;
            head[q] = tailed(q) && !(q > 0 && tailed(parent[q]));
            nid[q] = (uint32_t)dord.size();
            dord.push_back(q);
            if (head[q]) heads.push_back(q);
        }
        const uint32_t R = (uint32_t)dord.size();
        dfirst.assign(R, 0);
        dtail.assign(R, 0);
        std::vector<uint32_t> tidx(Q, 0);
        for (uint32_t i = 0; i < heads.size(); i++) tidx[heads[i]] = i;
        a->dev_out_first.assign(R + 1, 0);
        for (uint32_t x = 0; x < R; x++) {
            const uint32_t q = dord[x];
            if (head[q]) {
                dtail[x] = 1;
                dfirst[x] = tidx[q];
            } else {
                dfirst[x] = deg(q) ? nid[a->first_child[q]] : 0u;
            }
            a->dev_out_ids.insert(a->dev_out_ids.end(), a->out_ids.begin() + a->out_first[q],
                                  a->out_ids.begin() + a->out_first[q + 1]);
            a->dev_out_first[x + 1] = (uint32_t)a->dev_out_ids.size();
        }
        // tail records {offset of the path's symbols in the pattern bytes, length, ids of
        // its end: first index in the device id list (the id itself when it is the only
        // one), count}
        std::vector<uint32_t> tails((size_t)heads.size() * 4, 0);
        for (uint32_t i = 0; i < heads.size(); i++) {
            const uint32_t *tq = &a->dev_tails[(size_t)heads[i] * 4];
            const uint32_t leaf = tq[2];
            tails[(size_t)i * 4 + 0] = tq[0];
            tails[(size_t)i * 4 + 1] = tq[1];
            tails[(size_t)i * 4 + 2] = (uint32_t)a->dev_out_ids.size();
            a->dev_out_ids.insert(a->dev_out_ids.end(), a->out_ids.begin() + a->out_first[leaf],
                                  a->out_ids.begin() + a->out_first[leaf + 1]);
            tails[(size_t)i * 4 + 3] = (uint32_t)a->dev_out_ids.size() - tails[(size_t)i * 4 + 2];
            if (tails[(size_t)i * 4 + 3] == 1) tails[(size_t)i * 4 + 2] = a->dev_out_ids.back();  // the id itself
        }
        a->dev_tails.swap(tails);
        // the first kHeadBytes bytes of every record's path, beside the records
        a->dev_tail_head.assign((size_t)heads.size() * kHeadBytes, 0);
        for (uint32_t i = 0; i < heads.size(); i++) {
            const uint32_t off = a->dev_tails[(size_t)i * 4 + 0], len = a->dev_tails[(size_t)i * 4 + 1];
            const uint32_t h = len < kHeadBytes ? len : kHeadBytes;
            if (h) memcpy(&a->dev_tail_head[(size_t)i * kHeadBytes], &a->pat_bytes[off], h);
        }
    }
    const uint32_t R = (uint32_t)dord.size();
    a->dev_records = R;
    auto rec_of = [&](uint32_t x) { return a->merge_levels ? x : dord[x]; };  // row of rec_* arrays
    a->dev_nodes.clear();
    a->dev_bm.clear();
    if (a->alphabet <= 32) {
        a->layout = LAYOUT_NARROW;
        a->nw = 0;
        a->dev_nodes.resize(R);
        // two-bit symbols, plain table: a terminal with one pattern id carries that id in
        // the bitmap word's spare bits (bit 4 set, id in bits 5..31), so a walk reads it
        // with the node instead of through the id lists
        const bool one_id = a->alphabet <= 4 && !a->merge_levels && a->n_pats <= kOneIdMax;
        for (uint32_t x = 0; x < R; x++) {
            const uint32_t r = rec_of(x);
            if (dfirst[x] > kNarrowIndexMask) throw std::length_error("node index");
            uint64_t w = a->rec_bitmap[(size_t)r * a->nbw] & 0xffffffffull;
            w |= (uint64_t)dfirst[x] << 32;
            if (dtail[x]) w |= kTailBit;
            if (a->rec_term[r]) {
                w |= kTermBit;
                if (one_id && a->dev_out_first[x + 1] - a->dev_out_first[x] == 1)
                    w |= kOneIdBit | ((uint64_t)a->dev_out_ids[a->dev_out_first[x]] << kOneIdShift);
            }
            a->dev_nodes[x] = w;
        }
    } else {
        a->layout = LAYOUT_WIDE;
        a->nw = a->nbw <= 1 ? 1 : a->nbw <= 2 ? 2 : 4;
        a->dev_nodes.resize(R);
        a->dev_bm.assign((size_t)R * a->nw, 0);
        for (uint32_t x = 0; x < R; x++) {
            const uint32_t r = rec_of(x);
            const uint64_t *b = &a->rec_bitmap[(size_t)r * a->nbw];
            uint64_t r1 = 0, r2 = 0, r3 = 0;
            for (uint32_t w = 0; w < a->nbw; w++) a->dev_bm[(size_t)x * a->nw + w] = b[w];
            if (a->nbw > 1) r1 = popc64(b[0]);
            if (a->nbw > 2) r2 = r1 + popc64(b[1]);
            if (a->nbw > 3) r3 = r2 + popc64(b[2]);
            uint64_t m = dfirst[x] | (r1 << 32) | (r2 << 40) | (r3 << 48);
            if (dtail[x]) m |= kTailBit;
            if (a->rec_term[r]) m |= kTermBit;
            a->dev_nodes[x] = m;
        }
    }
    DevTable &t = a->shape;
    t = DevTable{};
    t.alphabet = a->alphabet;
    t.layout = a->layout;
    t.nw_log2 = a->nw == 4 ? 2 : a->nw == 2 ? 1 : 0;
    t.n_nodes = R;
    t.merged = a->merge_levels ? 1u : 0u;
    t.shared_base = a->shared_base;
    t.min_len = a->min_len;
    t.max_len = a->max_len;
    std::vector<const uint8_t *> P(a->n_pats);
    for (uint32_t j = 0; j < a->n_pats; j++) P[j] = a->pat_bytes.data() + a->pat_off[j];
    build_lds_image(a, P, a->req_depth, a->req_k);
}

int build_automaton(const uint8_t *const *pats, const uint64_t *lens, uint32_t n_pats,
                    uint32_t alphabet, pfac_automaton **out) {
    return build_automaton_ex(pats, lens, n_pats, alphabet, 0, out);
}

int build_automaton_ex(const uint8_t *const *pats, const uint64_t *lens, uint32_t n_pats, uint32_t alphabet,
                       uint32_t merge_levels, pfac_automaton **out) {
    if (!out) return PFAC_EINVAL;
    *out = nullptr;
    if (alphabet < 1 || alphabet > 256 || merge_levels > kMaxMergeLevels) return PFAC_EINVAL;
    if (n_pats > 0 && (!pats || !lens)) return PFAC_EINVAL;
    uint64_t total = 0;
    uint32_t minl = UINT32_MAX, maxl = 0;
    for (uint32_t j = 0; j < n_pats; j++) {
        if (lens[j] == 0) return PFAC_EEMPTY_PATTERN;
        if (!pats[j]) return PFAC_EINVAL;
        if (lens[j] > kMaxPatternLen) return PFAC_ETOO_LARGE;
        for (uint64_t i = 0; i < lens[j]; i++)
            if (pats[j][i] >= alphabet) return PFAC_ESYMBOL;
        total += lens[j];
        minl = std::min<uint32_t>(minl, (uint32_t)lens[j]);
        maxl = std::max<uint32_t>(maxl, (uint32_t)lens[j]);
    }
    if (n_pats == 0) minl = 0;
    pfac_automaton *a = new (std::nothrow) pfac_automaton();
    if (!a) return PFAC_ENOMEM;
    try {
        a->alphabet = alphabet;
        a->n_pats = n_pats;
        a->merge_levels = merge_levels;
        a->min_len = minl;
        a->max_len = maxl;
        a->nbw = (alphabet + 63) / 64;
        std::vector<const uint8_t *> P(pats, pats + n_pats);
        std::vector<uint32_t> &L = a->pat_len;
        L.resize(n_pats);
        for (uint32_t j = 0; j < n_pats; j++) L[j] = (uint32_t)lens[j];
        // bytewise sort; a proper prefix sorts before its extensions; ties by id
        std::vector<uint32_t> ord(n_pats);
        for (uint32_t j = 0; j < n_pats; j++) ord[j] = j;
        std::sort(ord.begin(), ord.end(), [&](uint32_t x, uint32_t y) {
            uint32_t m = std::min(L[x], L[y]);
            int c = memcmp(P[x], P[y], m);
            if (c) return c < 0;
            if (L[x] != L[y]) return L[x] < L[y];
            return x < y;
        });
        // breadth-first construction, one level at a time
        std::vector<Run> cur{{0, n_pats}}, nxt;
        a->depth_start.push_back(0);
        a->out_first.push_back(0);
        uint32_t next_id = 1;  // index the next created node will get
        for (uint32_t d = 0; !cur.empty(); d++) {
            nxt.clear();
            for (const Run &r : cur) {
                uint32_t i = r.lo;
                // patterns of length d end at this node (ids ascending: ties sorted by id)
                while (i < r.hi && L[ord[i]] == d) a->out_ids.push_back(ord[i++]);
                a->out_first.push_back((uint32_t)a->out_ids.size());
                size_t base = a->bitmap.size();
                a->bitmap.resize(base + a->nbw, 0);
                a->first_child.push_back(i < r.hi ? next_id : 0);
                while (i < r.hi) {
                    uint8_t c = P[ord[i]][d];
                    uint32_t j = i + 1;
                    while (j < r.hi && P[ord[j]][d] == c) j++;
                    nxt.push_back({i, j});
                    a->bitmap[base + (c >> 6)] |= 1ull << (c & 63);
                    if (next_id >= kMaxNodes) {
                        delete a;
                        return PFAC_ETOO_LARGE;
                    }
                    next_id++;
                    i = j;
                }
            }
            a->depth_start.push_back(a->depth_start.back() + (uint32_t)cur.size());
            cur.swap(nxt);
        }
        a->n_nodes = (uint32_t)a->first_child.size();
        while (a->depth_start.size() < (size_t)maxl + 3) a->depth_start.push_back(a->n_nodes);
        a->pat_off.assign(n_pats + 1, 0);
        for (uint32_t j = 0; j < n_pats; j++) a->pat_off[j + 1] = a->pat_off[j] + lens[j];
        a->pat_bytes.resize(a->pat_off[n_pats]);
        for (uint32_t j = 0; j < n_pats; j++) memcpy(a->pat_bytes.data() + a->pat_off[j], P[j], lens[j]);
        (void)total;
        finish_automaton(a);
    } catch (const std::bad_alloc &) {
        delete a;
        return PFAC_ENOMEM;
    } catch (const std::length_error &) {  // a device index past its field
        delete a;
        return PFAC_ETOO_LARGE;
    }
    *out = a;
    return PFAC_OK;
}

}  // namespace pfac
