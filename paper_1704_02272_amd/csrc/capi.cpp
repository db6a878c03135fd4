// C ABI entry points that need no device: status strings, building, introspection.
#include <algorithm>
#include <new>
#include <vector>

#include "pfac.h"
#include "kernels.h"
#include "pfac_impl.h"

using namespace pfac;

extern "C" const char *pfac_strerror(int status) {
    switch (status) {
        case PFAC_OK: return "ok";
        case PFAC_EINVAL: return "invalid argument";
        case PFAC_EEMPTY_PATTERN: return "empty pattern";
        case PFAC_ESYMBOL: return "pattern symbol outside the alphabet";
        case PFAC_ETOO_LARGE: return "size exceeds the 32-bit limits of the table or key";
        case PFAC_ENOMEM: return "out of memory";
        case PFAC_EHIP: return "HIP runtime error";
        case PFAC_ECAPACITY: return "output capacity too small";
        case PFAC_ENODEVICE: return "no usable gfx950 device";
        case PFAC_EFORMAT: return "malformed serialized automaton";
        case PFAC_ETIMEOUT: return "device-side wait timed out";
        case PFAC_EINTERNAL: return "internal consistency check failed";
        case PFAC_EBUSY: return "server queue is full";
        default: return "unknown status";
    }
}

extern "C" int pfac_version(void) { return 1 * 10000 + 1 * 100 + 0; }

extern "C" int pfac_build(const uint8_t *const *pats, const uint64_t *lens, uint32_t n_pats,
                          uint32_t alphabet, pfac_automaton **out) {
    return build_automaton(pats, lens, n_pats, alphabet, out);
}

extern "C" int pfac_build_csr(const uint8_t *bytes, const uint64_t *offsets, uint32_t n_pats,
                              uint32_t alphabet, pfac_automaton **out) {
    if (!out) return PFAC_EINVAL;
    *out = nullptr;
    if (n_pats > 0 && (!bytes || !offsets)) return PFAC_EINVAL;
    std::vector<const uint8_t *> p;
    std::vector<uint64_t> l;
    try {
        p.resize(n_pats);
        l.resize(n_pats);
    } catch (const std::bad_alloc &) {
        return PFAC_ENOMEM;
    }
    for (uint32_t i = 0; i < n_pats; i++) {
        if (offsets[i + 1] < offsets[i]) return PFAC_EINVAL;
        p[i] = bytes + offsets[i];
        l[i] = offsets[i + 1] - offsets[i];
    }
    return build_automaton(p.data(), l.data(), n_pats, alphabet, out);
}

extern "C" int pfac_build_ex(const uint8_t *bytes, const uint64_t *offsets, uint32_t n_pats, uint32_t alphabet,
                             const pfac_build_options *opt, pfac_automaton **out) {
    if (!out) return PFAC_EINVAL;
    *out = nullptr;
    if (n_pats > 0 && (!bytes || !offsets)) return PFAC_EINVAL;
    const uint32_t levels = opt ? opt->merge_levels : 0;
    std::vector<const uint8_t *> p;
    std::vector<uint64_t> l;
    try {
        p.resize(n_pats);
        l.resize(n_pats);
    } catch (const std::bad_alloc &) {
        return PFAC_ENOMEM;
    }
    for (uint32_t i = 0; i < n_pats; i++) {
        if (offsets[i + 1] < offsets[i]) return PFAC_EINVAL;
        p[i] = bytes + offsets[i];
        l[i] = offsets[i + 1] - offsets[i];
    }
    return build_automaton_ex(p.data(), l.data(), n_pats, alphabet, levels, out);
}

extern "C" void pfac_destroy(pfac_automaton *a) { delete a; }

// Every byte a device copy of the automaton holds in HBM (as the runtime uploads it).
static uint64_t device_bytes(const pfac_automaton *a) {
    uint64_t b = a->dev_nodes.size() * 8 + a->dev_bm.size() * 8 + a->dev_tails.size() * 4 +
                 a->dev_tail_head.size() + a->pat_bytes.size() + a->lds_image.size() * 4 +
                 a->dev_out_first.size() * 4 + a->dev_out_ids.size() * 4;
    if (a->merge_levels) b += a->rec_rank.size() * 4;
    return b;
}

extern "C" int pfac_table_info(const pfac_automaton *a, pfac_table_info_t *o) {
    if (!a || !o) return PFAC_EINVAL;
    o->alphabet = a->alphabet;
    o->n_patterns = a->n_pats;
    o->n_nodes = a->n_nodes;
    o->n_terminal_nodes = a->n_term;
    o->min_len = a->min_len;
    o->max_len = a->max_len;
    o->depth = a->max_len;
    o->node_layout = a->layout;
    const uint64_t node_bytes = 4 + (a->alphabet + 7) / 8;
    o->paper_table_bytes = (uint64_t)a->n_nodes * node_bytes;
    o->device_table_bytes = device_bytes(a);
    o->root_depth = a->shape.root_depth;
    o->filter_k = a->shape.filter_k;
    o->filter_log2_bits = a->shape.filter_log2;
    o->lds_image_bytes = a->shape.lds_words * 4;
    o->merge_levels = a->merge_levels;
    o->reduced_nodes = a->reduced_nodes;
    o->table_records = a->n_rec;
    o->shared_base = a->shared_base;
    o->reduced_paper_bytes = (uint64_t)a->reduced_nodes * node_bytes;
    o->node_array_bytes = a->dev_nodes.size() * 8 + a->dev_bm.size() * 8;
    o->stream_scratch = pfac::workspace_count(const_cast<pfac_automaton *>(a));
    o->device_records = a->dev_records;
    o->device_tails = a->merge_levels ? 0u : (uint32_t)(a->dev_tails.size() / 4);
    return PFAC_OK;
}

extern "C" int pfac_export_paper_table(const pfac_automaton *a, uint32_t *offsets,
                                       uint64_t offsets_cap, uint32_t *bitmaps,
                                       uint64_t bitmaps_cap) {
    if (!a || !offsets || !bitmaps) return PFAC_EINVAL;
    const uint32_t words = (a->alphabet + 31) / 32;
    if (offsets_cap < a->n_nodes || bitmaps_cap < (uint64_t)a->n_nodes * words) return PFAC_EINVAL;
    for (uint32_t q = 0; q < a->n_nodes; q++) {
        offsets[q] = a->first_child[q];
        const uint64_t *b = &a->bitmap[(size_t)q * a->nbw];
        for (uint32_t w = 0; w < words; w++)
            bitmaps[(size_t)q * words + w] = (uint32_t)(b[w / 2] >> (32 * (w & 1)));
    }
    return PFAC_OK;
}

extern "C" int pfac_export_outputs(const pfac_automaton *a, uint32_t *first, uint64_t first_cap,
                                   uint32_t *ids, uint64_t ids_cap) {
    if (!a || !first || (!ids && a->n_pats > 0)) return PFAC_EINVAL;
    if (first_cap < (uint64_t)a->n_nodes + 1 || ids_cap < a->out_ids.size()) return PFAC_EINVAL;
    std::copy(a->out_first.begin(), a->out_first.end(), first);
    std::copy(a->out_ids.begin(), a->out_ids.end(), ids);
    return PFAC_OK;
}

extern "C" int pfac_export_records(const pfac_automaton *a, uint32_t *first, uint32_t *bitmaps, uint8_t *term,
                                   uint32_t *rank, uint64_t cap) {
    if (!a || !first || !bitmaps || !term || !rank) return PFAC_EINVAL;
    if (cap < a->n_rec) return PFAC_EINVAL;
    const uint32_t words = (a->alphabet + 31) / 32;
    for (uint32_t x = 0; x < a->n_rec; x++) {
        first[x] = a->rec_first[x];
        term[x] = a->rec_term[x];
        rank[x] = a->rec_rank[x];
        const uint64_t *b = &a->rec_bitmap[(size_t)x * a->nbw];
        for (uint32_t w = 0; w < words; w++) bitmaps[(size_t)x * words + w] = (uint32_t)(b[w / 2] >> (32 * (w & 1)));
    }
    return PFAC_OK;
}

extern "C" int pfac_export_rank_ids(const pfac_automaton *a, uint32_t *first, uint64_t first_cap, uint32_t *ids,
                                    uint64_t ids_cap) {
    if (!a || !first || (!ids && a->n_pats > 0)) return PFAC_EINVAL;
    if (first_cap < a->rank_first.size() || ids_cap < a->rank_ids.size()) return PFAC_EINVAL;
    std::copy(a->rank_first.begin(), a->rank_first.end(), first);
    std::copy(a->rank_ids.begin(), a->rank_ids.end(), ids);
    return PFAC_OK;
}
