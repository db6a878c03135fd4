// The table the scans walk: the trie of Section 3.1 itself, or its compressed form of
// Section 3.2, as one array of records walked with Eq. 1.
//
// A record is what the paper stores per node: a child bitmap and the index of the first
// child (0 without children), plus the terminal flag. The children of a record are the
// consecutive records offset + popcount(bits below c) (Eq. 1). In the plain trie every
// record is one node and every node's children form its own block.
//
// Compression (Section 3.2). Nodes of the bottom levels are merged when everything below
// them is the same (their suffix languages agree), and the global final node of step 1
// is the leaves merged into one. With Eq. 1 a node's children must stay consecutive, so
// what a table can share is a block of children: the children of two nodes are stored
// once when they are the same sequence of merged nodes. Blocks made only of final nodes
// all point into one block of leaf records (the global final node, repeated for as many
// children as a node can have). Sharing is allowed for the block of a node whose height
// (longest path down to a leaf) is at most `levels`, i.e. whose children are all of
// height below `levels`: levels 1 shares only final nodes, 3 the last three levels of
// the paper. Blocks of nodes above the LDS root image's depth are never shared, so the
// top levels keep the breadth-first numbering the root image relies on.
//
// Pattern identity (the paper's node has none). A walk from start s that reaches a
// terminal record has spelled one pattern string w; its ids are found by the rank of w
// among the distinct pattern strings in bytewise order (shorter first). Every record
// holds a rank word: a record of the unshared top part (index < shared_base) holds the
// rank of its own prefix; a record in a shared block holds the number of strings spelled
// below its lower siblings in the block. A walk remembers the last unshared record u and
// adds, for every step into a shared record y from record q, term(q) + rank[y]; the rank
// of the string spelled at a shared terminal is rank[u] plus that sum (at an unshared
// terminal, its own rank word). This counts exactly the pattern strings that sort before
// w, whichever parent the walk came through. Ids of rank r: rank_ids[rank_first[r] ..
// rank_first[r+1]).
#include <string.h>

#include <algorithm>
#include <string>
#include <unordered_map>

#include "pfac.h"
#include "pfac_impl.h"

namespace pfac {

void build_records(pfac_automaton *a) {
    const uint32_t Q = a->n_nodes, W = a->nbw;
    std::vector<uint32_t> deg(Q), height(Q, 0), depth(Q, 0), parent(Q, 0);
    std::vector<uint8_t> term(Q);
    for (uint32_t d = 0; d + 1 < a->depth_start.size(); d++)
        for (uint32_t q = a->depth_start[d]; q < a->depth_start[d + 1] && q < Q; q++) depth[q] = d;
    for (uint32_t q = 0; q < Q; q++) {
        uint32_t k = 0;
        for (uint32_t w = 0; w < W; w++) k += (uint32_t)__builtin_popcountll(a->bitmap[(size_t)q * W + w]);
        deg[q] = k;
        term[q] = a->out_first[q + 1] > a->out_first[q];
        for (uint32_t i = 0; i < k; i++) parent[a->first_child[q] + i] = q;
    }
    // strings spelled below each node, and heights (children have larger indices)
    std::vector<uint64_t> lsize(Q);
    for (uint32_t q = Q; q-- > 0;) {
        uint64_t s = term[q];
        uint32_t h = 0;
        for (uint32_t i = 0; i < deg[q]; i++) {
            const uint32_t c = a->first_child[q] + i;
            s += lsize[c];
            h = std::max(h, height[c] + 1);
        }
        lsize[q] = s;
        height[q] = h;
    }
    // rank of every prefix among the distinct pattern strings (top-down)
    std::vector<uint64_t> acc(Q, 0);
    for (uint32_t q = 0; q < Q; q++) {
        uint64_t run = acc[q] + term[q];
        for (uint32_t i = 0; i < deg[q]; i++) {
            const uint32_t c = a->first_child[q] + i;
            acc[c] = run;
            run += lsize[c];
        }
    }
    const uint64_t n_str = Q ? lsize[0] : 0;
    a->rank_first.assign(n_str + 1, 0);
    a->rank_ids.assign(a->n_pats, 0);
    for (uint32_t q = 0; q < Q; q++)
        if (term[q]) a->rank_first[acc[q] + 1] = a->out_first[q + 1] - a->out_first[q];
    for (uint64_t r = 0; r < n_str; r++) a->rank_first[r + 1] += a->rank_first[r];
    for (uint32_t q = 0; q < Q; q++)
        if (term[q])
            std::copy(a->out_ids.begin() + a->out_first[q], a->out_ids.begin() + a->out_first[q + 1],
                      a->rank_ids.begin() + a->rank_first[acc[q]]);

    const uint32_t L = a->merge_levels;
    if (L == 0) {
        a->n_rec = Q;
        a->shared_base = Q;
        a->reduced_nodes = Q;
        a->rec_first = a->first_child;
        a->rec_bitmap = a->bitmap;
        a->rec_term = term;
        a->rec_rank.resize(Q);
        for (uint32_t q = 0; q < Q; q++) a->rec_rank[q] = (uint32_t)acc[q];
        return;
    }

    // classes of equal suffix language among nodes of height < L, bottom-up: a node's
    // class is fixed by its bitmap, its terminal flag and its children's classes
    constexpr uint32_t kNone = 0xffffffffu;
    std::vector<uint32_t> cls(Q, kNone), rep;
    {
        std::unordered_map<std::string, uint32_t> intern;
        std::string key;
        for (uint32_t q = Q; q-- > 0;) {
            if (height[q] >= L) continue;
            key.assign(reinterpret_cast<const char *>(&a->bitmap[(size_t)q * W]), W * 8);
            key.push_back((char)term[q]);
            for (uint32_t i = 0; i < deg[q]; i++)
                key.append(reinterpret_cast<const char *>(&cls[a->first_child[q] + i]), 4);
            auto it = intern.emplace(key, (uint32_t)intern.size());
            if (it.second) rep.push_back(q);
            cls[q] = it.first->second;
        }
    }
    uint32_t kept = 0;
    for (uint32_t q = 0; q < Q; q++) kept += height[q] >= L;
    a->reduced_nodes = kept + (uint32_t)rep.size();

    // which blocks are shared: children all merged (height of q <= L), below the root image
    const uint32_t D0 = a->n_pats ? std::min(a->min_len, a->alphabet <= 4 ? 8u : 2u) : 0u;
    auto shared_blk = [&](uint32_t q) { return deg[q] > 0 && height[q] <= L && depth[q] >= D0; };
    auto all_leaves = [&](uint32_t q) {
        for (uint32_t i = 0; i < deg[q]; i++)
            if (deg[a->first_child[q] + i]) return false;
        return true;
    };

    // unshared top part: breadth-first order among nodes whose ancestors' blocks are unshared
    std::vector<uint32_t> rec(Q, kNone);
    std::vector<uint32_t> top;  // node of each top record
    for (uint32_t q = 0; q < Q; q++) {
        if (q == 0 || (rec[parent[q]] != kNone && !shared_blk(parent[q]))) {
            rec[q] = (uint32_t)top.size();
            top.push_back(q);
        }
    }
    const uint32_t S = (uint32_t)top.size();
    // shared blocks, allocated breadth-first from the references of the top part; the
    // block of final nodes once, as long as the widest such block
    uint32_t final_len = 0;
    for (uint32_t q = 0; q < Q; q++)
        if (shared_blk(q) && all_leaves(q)) final_len = std::max(final_len, deg[q]);
    std::unordered_map<std::string, uint32_t> blocks;  // children classes -> first record
    std::vector<uint32_t> blk_node;                     // node (representative) of each shared record
    uint32_t final_base = kNone;
    auto block_of = [&](uint32_t q) -> uint32_t {      // q: a node whose block is shared
        if (all_leaves(q)) {
            if (final_base == kNone) {
                final_base = S + (uint32_t)blk_node.size();
                const uint32_t leaf = a->first_child[q];
                for (uint32_t i = 0; i < final_len; i++) blk_node.push_back(leaf);
            }
            return final_base;
        }
        std::string key(reinterpret_cast<const char *>(&cls[a->first_child[q]]), (size_t)deg[q] * 4);
        auto it = blocks.emplace(key, S + (uint32_t)blk_node.size());
        if (it.second)
            for (uint32_t i = 0; i < deg[q]; i++) blk_node.push_back(rep[cls[a->first_child[q] + i]]);
        return it.first->second;
    };
    a->rec_first.assign(S, 0);
    for (uint32_t x = 0; x < S; x++) {
        const uint32_t q = top[x];
        if (!deg[q]) continue;
        a->rec_first[x] = shared_blk(q) ? block_of(q) : rec[a->first_child[q]];
    }
    // records of shared blocks: their own blocks are shared (they lie below the root
    // image and have height < L); blk_node grows while this loop runs
    for (size_t i = 0; i < blk_node.size(); i++) {
        const uint32_t q = blk_node[i];
        a->rec_first.push_back(deg[q] ? block_of(q) : 0u);
    }
    const uint32_t R = (uint32_t)a->rec_first.size();
    a->n_rec = R;
    a->shared_base = S;
    a->rec_bitmap.assign((size_t)R * W, 0);
    a->rec_term.assign(R, 0);
    a->rec_rank.assign(R, 0);
    for (uint32_t x = 0; x < R; x++) {
        const uint32_t q = x < S ? top[x] : blk_node[x - S];
        std::copy(&a->bitmap[(size_t)q * W], &a->bitmap[(size_t)q * W] + W, &a->rec_bitmap[(size_t)x * W]);
        a->rec_term[x] = term[q];
        if (x < S) a->rec_rank[x] = (uint32_t)acc[q];
    }
    // rank words of shared records: strings below the lower siblings in the block
    auto fill_block = [&](uint32_t base, uint32_t len) {
        uint64_t run = 0;
        for (uint32_t i = 0; i < len; i++) {
            a->rec_rank[base + i] = (uint32_t)run;
            run += lsize[blk_node[base + i - S]];
        }
    };
    if (final_base != kNone) fill_block(final_base, final_len);
    for (const auto &kv : blocks) fill_block(kv.second, (uint32_t)(kv.first.size() / 4));
    // record of every trie node (Eq. 1 over the records), and the path tails of the trie
    // moved onto the records
    for (uint32_t q = 0; q < Q; q++) {
        const uint32_t x = rec[q];
        if (x == kNone) continue;
        for (uint32_t i = 0; i < deg[q]; i++) {
            const uint32_t c = a->first_child[q] + i;
            if (rec[c] == kNone) rec[c] = a->rec_first[x] + i;
        }
    }
    std::vector<uint32_t> tails((size_t)R * 4, 0);
    for (uint32_t q = 0; q < Q; q++) {
        const uint32_t *t = &a->dev_tails[(size_t)q * 4];
        if (!t[1]) continue;
        uint32_t *o = &tails[(size_t)rec[q] * 4];
        if (o[1]) continue;  // the same path already came from another node of the class
        o[0] = t[0];
        o[1] = t[1];
        o[2] = rec[t[2]];
    }
    a->dev_tails.swap(tails);
}

}  // namespace pfac
