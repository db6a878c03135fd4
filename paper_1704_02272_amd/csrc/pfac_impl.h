// Internal definitions shared by the host builder, the HIP runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <vector>

namespace pfac {

// Node layouts in HBM.
//
// NARROW (alphabet <= 32): one 64-bit word per node:
//     bits  0..31  child bitmap (bit c = symbol c)
//     bits 32..61  first-child index (0 when the node has no child), or the tail index
//   (two-bit symbols, plain table: bit 4 flags a terminal with one id, held in bits 5..31)
//     bit  62      tail flag (plain table only)
//     bit  63      terminal: at least one pattern ends here
//   This is the paper's 8-byte node at |Sigma| = 32 (Section 3.1) with the terminal flag
//   taken from the top bit of the offset.
//
// WIDE (alphabet 33..256): bitmap words and per-node metadata in two arrays:
//     bm[q * NW + w]  bits 64w .. 64w+63 of the child bitmap, NW = 1, 2 or 4
//     meta[q]         bits  0..31 first-child index, or the tail index
//                     bits 32..55 three rank bytes: set bits in words < 1, < 2, < 3
//                     bit  62     tail flag (plain table only)
//                     bit  63     terminal
//   A lookup reads one bitmap word and the metadata word; Eq. 1's popcount then covers
//   one 64-bit word plus a stored rank byte instead of up to four words.
enum Layout : uint32_t { LAYOUT_NARROW = 0, LAYOUT_WIDE = 1 };

constexpr uint64_t kTermBit = 1ull << 63;
// Tail flag (plain table): the node heads a collapsed unary path; its first-child field
// holds the index of the path's tail record instead (see DevTable::tails).
constexpr uint64_t kTailBit = 1ull << 62;
constexpr uint32_t kNarrowIndexMask = 0x3fffffffu;  // NARROW: first child / tail index, bits 32..61
// Two-bit symbols, plain table: the bitmap field holds four bits; a terminal with a single
// pattern id keeps it in bits 5..31 of the word, flagged by bit 4.
constexpr uint64_t kOneIdBit = 1ull << 4;
constexpr uint32_t kOneIdShift = 5;
constexpr uint32_t kOneIdMax = 1u << 27;
constexpr uint32_t kHeadBytes = 16;  // path bytes kept beside each tail record (plain table)
constexpr uint32_t kMaxPatternLen = 1u << 24;
constexpr uint32_t kMaxNodes = 0x7fffffffu;
constexpr uint32_t kMaxMergeLevels = 255;  // levels >= the deepest height merge everything

// Per-workgroup LDS image (copied from HBM at kernel start), in 32-bit words:
//   [filter: 2^filter_log2 bits]         k-gram prefix filter (optional), at offset 0
//   [root bitmap: 2^root_bits bits]      D-gram -> present?   (D = root_depth)
//   [root rank: 2^(root_bits-5) u16]     set bits before each 32-bit word
//   [short bitmap: 2^root_bits bits]     D-grams of the patterns shorter than k (optional)
// A start passes the prefilter when its k-gram is in the filter or its D-gram is in the
// short bitmap; with no filter (k = D) it passes when its D-gram is in the root bitmap.
// The root image folds the top D trie levels into one direct-indexed bitmap whose rank
// (the popcount rule of Eq. 1 applied to a D-symbol root) is the breadth-first index of
// the depth-D node: node = depth_start[D] + rank(key), keys in lexicographic order.
struct DevTable {
    const uint64_t *nodes;      // NARROW: node words. WIDE: meta words.
    const uint64_t *bm;         // WIDE: bitmap words. NARROW: unused (null).
    const uint32_t *out_first;  // n_nodes + 1: ids of q at out_ids[out_first[q] .. [q+1])
    const uint32_t *out_ids;
    const uint32_t *lds_image;  // see above
    // Path tails. Compressed table: tails[4q .. 4q+3] = {byte offset in tail_bytes,
    // length, end record, 0} when everything below record q is one path whose only
    // terminal is its end (length > 0), else zeros; a walk at such a record compares the
    // text with the path's symbols at once instead of stepping record by record. Plain
    // table: one record per tail head (a node with the tail flag; index in its word):
    // {byte offset of the path's symbols, length, first index of the end's ids in
    // out_ids (the id itself when the count is 1), their count}; the path's nodes are
    // not stored.
    const uint32_t *tails;
    const uint8_t *tail_bytes;
    // Plain table: the first kHeadBytes bytes of each tail record's path (zero past its
    // length), kHeadBytes per record in record order, so a walk loads them together with
    // the record. Null for a compressed table.
    const uint4 *tail_head;
    uint32_t alphabet;
    uint32_t layout;            // Layout
    uint32_t nw_log2;           // WIDE: log2(NW)
    uint32_t n_nodes;
    uint32_t min_len, max_len;
    uint32_t pack2;             // 1: symbols coded in 2 bits (alphabet <= 4), else bytes
    uint32_t root_depth;        // D (0 = no root image: walks start at node 0)
    uint32_t root_bits;         // D * bits-per-symbol
    uint32_t root_base;         // index of the first depth-D node
    uint32_t filter_k;          // k (symbols per filter key); 0 = no hashed filter
    uint32_t has_short;         // 1: some pattern is shorter than k (short bitmap used)
    uint32_t filter_log2;       // log2(bits of the first-probe region); 0 = no filter
    uint32_t sampled;           // 1: sampled prefilter layout (every second start probed)
    uint32_t exact;             // 1: exact form: the filter is the (D+E)-symbol bitmap (two-bit
                                //    symbols, filter_k = D + E, E = 1 or 2)
    uint32_t lds_words;         // total image size in 32-bit words
    uint32_t root_word;         // word offset of the root bitmap
    uint32_t rank_word;         // word offset of the rank table
    uint32_t short_word;        // word offset of the short bitmap (= lds_words if none)
    // Compressed tables (Section 3.2): records from shared_base on lie in shared blocks;
    // rk[x] is the rank word of record x (see reduce.cpp), and out_first / out_ids then
    // hold the ids by rank of the spelled string instead of by node.
    const uint32_t *rk;
    uint32_t merged;            // 1: compressed table, ids found by rank
    uint32_t shared_base;       // first record of a shared block (= n_nodes when none)
};

constexpr uint32_t kFilterMul = 0x9E3779B1u;  // multiplicative hash (golden ratio)
constexpr uint32_t kFilterMul2 = 0x85EBCA6Bu; // second hash (MurmurHash3 finalizer constant)

// Prefilter over k-gram keys: a two-probe Bloom filter split into two regions, probe 2's
// region of 2^log2_b bits first, then probe 1's region of 2^log2_a bits. A key sets one bit
// in each. Probe 1: word from the high half of key * kFilterMul masked to the region
// (the masked value is the word's byte offset in the region), bit = key & 31. Probe 2: the
// same with kFilterMul2, bit = the top five bits of that high half. A key passes only if
// both bits are set; the scan takes probe 2 only for starts that pass probe 1. The
// builder and the kernels must agree bit for bit.
__host__ __device__ inline uint32_t filter_hi(uint32_t key, uint32_t mul) {
    return (uint32_t)(((uint64_t)key * mul) >> 32);
}
// Insert key into a two-probe filter whose first-probe part (wa words) starts at word
// oa of F and whose second-probe part (wb words) starts at word ob.
inline void filter_insert(uint32_t *F, uint32_t key, uint32_t oa, uint32_t wa, uint32_t ob, uint32_t wb) {
    F[oa + ((filter_hi(key, kFilterMul) >> 2) & (wa - 1u))] |= 1u << (key & 31);
    const uint32_t h2 = filter_hi(key, kFilterMul2);
    F[ob + ((h2 >> 2) & (wb - 1u))] |= 1u << (h2 >> 27);
}

// 3-gram key (three bytes, first one lowest) of the sampled prefilter: the word from the
// top bits of the low 32 bits of key * mul3 (both 24-bit), bit = key & 31.
inline void filter3_insert(uint32_t *F, uint32_t key, uint32_t mul3, uint32_t off, uint32_t words) {
    const uint32_t h = (uint32_t)((uint64_t)(key & 0xffffffu) * (mul3 & 0xffffffu));
    F[off + ((h >> 18) & (words - 1u))] |= 1u << (key & 31);
}

// Two-probe filter over 4-gram keys of the sampled prefilter, hashed with 24-bit products
// (full-rate multiplies on the GPU). Probe 1: word from bits 18.. of bytes 1..3 * kS1Mul,
// bit = the low five bits of byte 0. Probe 2: word from bits 18.. of bytes 0..2 * kS2Mul,
// bit = the low five bits of byte 1. The builder and the kernels must agree bit for bit.
constexpr uint32_t kS1Mul = 0x9E3779u, kS2Mul = 0x85EBCBu;
__host__ __device__ inline uint32_t s1_hash(uint32_t key) { return (key >> 8) * kS1Mul; }
__host__ __device__ inline uint32_t s2_hash(uint32_t key) { return (key & 0xffffffu) * kS2Mul; }
inline void filter4s_insert(uint32_t *F, uint32_t key, uint32_t o1, uint32_t w1, uint32_t o2, uint32_t w2) {
    F[o1 + ((s1_hash(key) >> 18) & (w1 - 1u))] |= 1u << (key & 31);
    F[o2 + ((s2_hash(key) >> 18) & (w2 - 1u))] |= 1u << ((key >> 8) & 31);
}

struct Workspace;  // per (device, stream) scratch, defined in the runtime

struct DeviceCopy {
    int device = -1;
    uint32_t cus = 256;  // compute units of the device
    void *nodes = nullptr, *bm = nullptr, *out_first = nullptr, *out_ids = nullptr,
         *lds_image = nullptr, *tails = nullptr, *tail_bytes = nullptr, *rk = nullptr, *tail_head = nullptr;
    DevTable view{};
    std::map<void *, Workspace *> workspaces;  // keyed by stream
    // LDS images replaced by a change of tuning. Queued scans and captured graphs may
    // still read them, so they are freed with the copy, not when replaced.
    std::vector<void *> retired;
};

}  // namespace pfac

struct pfac_automaton {
    uint32_t alphabet = 0, n_pats = 0, n_nodes = 0, n_term = 0;
    uint32_t min_len = 0, max_len = 0;
    uint32_t layout = 0, nw = 0;  // nw: 64-bit bitmap words per node (WIDE)
    uint32_t algo = 0, grid = 0;  // tuning: kernel choice, persistent grid (0 = auto)
    uint32_t span_log2 = 0;       // tuning: log2 of the count kernel's span length (0 = by text size)
    uint32_t lane_bytes = 32;     // tuning: positions per thread and wave step (16 or 32)
    uint32_t req_depth = 0, req_k = 0;  // tuning: requested root depth / filter key (0 = builder's)
    // The patterns as given (CSR), kept to rebuild the LDS image when tuning asks.
    std::vector<uint8_t> pat_bytes;
    std::vector<uint64_t> pat_off;
    // Paper layout (Section 3.1): first-child offset and the bitmap in 64-bit words.
    std::vector<uint32_t> first_child;
    std::vector<uint64_t> bitmap;      // n_nodes * nbw, nbw = ceil(alphabet / 64)
    uint32_t nbw = 0;
    std::vector<uint32_t> depth_start;  // first node of each depth, depth 0..max_len+1
    std::vector<uint32_t> out_first, out_ids;
    std::vector<uint32_t> pat_len;
    // The table the scans walk (reduce.cpp): the trie itself (merge_levels 0) or its
    // compressed form (Section 3.2, nodes of height < merge_levels merged).
    uint32_t merge_levels = 0;
    uint32_t reduced_nodes = 0;         // nodes after merging (the paper's measure)
    uint32_t n_rec = 0, shared_base = 0;
    std::vector<uint32_t> rec_first;    // first child record (0: none)
    std::vector<uint64_t> rec_bitmap;   // n_rec * nbw
    std::vector<uint8_t> rec_term;
    std::vector<uint32_t> rec_rank;     // rank words
    std::vector<uint32_t> rank_first, rank_ids;  // ids of each distinct pattern string, by rank
    // Device images.
    std::vector<uint64_t> dev_nodes, dev_bm;
    std::vector<uint32_t> lds_image;
    std::vector<uint32_t> dev_tails;  // see DevTable::tails
    std::vector<uint8_t> dev_tail_head;  // see DevTable::tail_head
    std::vector<uint32_t> dev_out_first, dev_out_ids;  // ids as the device table indexes them
    uint32_t dev_records = 0;         // records of the device table
    pfac::DevTable shape{};  // pointer fields null; filled per device copy
    std::vector<pfac::DeviceCopy *> copies;
    std::mutex mu;
    ~pfac_automaton();
};

namespace pfac {
int build_automaton(const uint8_t *const *pats, const uint64_t *lens, uint32_t n_pats,
                    uint32_t alphabet, pfac_automaton **out);
void release_device_copies(pfac_automaton *a);
// Rebuild the LDS image with root depth D and filter key length K (0 = the builder's
// choice for either). PFAC_EINVAL when D or K is outside what the pattern set allows.
int rebuild_lds_image(pfac_automaton *a, uint32_t D, uint32_t K);
// Derive the device images (node words, path tails, LDS image) from the trie arrays,
// the patterns and the requested root depth / filter key. Throws std::bad_alloc.
void finish_automaton(pfac_automaton *a);
// The record table (plain or compressed) and the ids by rank; remaps the path tails.
void build_records(pfac_automaton *a);
void build_tails(pfac_automaton *a);
// pfac_build with the table compressed (Section 3.2) below `merge_levels` (0: plain).
int build_automaton_ex(const uint8_t *const *pats, const uint64_t *lens, uint32_t n_pats, uint32_t alphabet,
                       uint32_t merge_levels, pfac_automaton **out);
}  // namespace pfac
