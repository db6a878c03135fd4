// Scan of a text in host memory: pinned staging, chunks with a halo, copy/compute overlap.
//
// The text is cut into chunks [a, b); each chunk is sent with the next maxlen - 1 bytes
// (the overlap rule of Section 2.2: a match starting before b may end after it) and only
// matches starting before b are kept. Two slots, each with its own stream, pinned
// staging buffer, device text buffer and key buffer, alternate: while one slot's chunk is
// copied and scanned, the host fills the other slot and collects the one before. Keys
// come back as chunk-local (start << 32) | id and are expanded on the host to 64-bit
// starts by adding the chunk base (texts may exceed 2^32 bytes).
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "pfac.h"
#include "kernels.h"
#include "pfac_impl.h"

namespace {

struct Slot {
    hipStream_t s = nullptr;
    uint8_t *h_stage = nullptr;   // pinned staging (pageable input only)
    uint8_t *d_text = nullptr;
    uint64_t *d_keys = nullptr, cap = 0;
    uint64_t *d_count = nullptr;
    uint64_t *h_count = nullptr;  // pinned
    uint64_t *h_keys = nullptr, h_cap = 0;  // pinned
    // chunk in flight
    bool busy = false;
    uint64_t base = 0, own = 0, len = 0;
};

struct Pipeline {
    pfac_automaton *a;
    const uint8_t *h_text;
    uint64_t n;
    bool pinned_input;
    Slot slot[2];
    std::vector<pfac_match> out;

    ~Pipeline() {
        for (Slot &s : slot) {
            if (s.s) (void)hipStreamSynchronize(s.s);
            if (s.s) pfac::release_stream(a, s.s);  // scratch keyed by this stream
            hipHostFree(s.h_stage);
            hipFree(s.d_text);
            hipFree(s.d_keys);
            hipFree(s.d_count);
            hipHostFree(s.h_count);
            hipHostFree(s.h_keys);
            if (s.s) (void)hipStreamDestroy(s.s);
        }
    }
};

int grow_keys(Slot &s, uint64_t need) {
    if (need <= s.cap && need <= s.h_cap) return PFAC_OK;
    const uint64_t want = std::max<uint64_t>(need + need / 4, 4096);
    if (need > s.cap) {
        hipFree(s.d_keys);
        s.d_keys = nullptr;
        s.cap = 0;
        if (hipMalloc(&s.d_keys, want * 8) != hipSuccess) return PFAC_ENOMEM;
        s.cap = want;
    }
    if (need > s.h_cap) {
        hipHostFree(s.h_keys);
        s.h_keys = nullptr;
        s.h_cap = 0;
        if (hipHostMalloc(&s.h_keys, want * 8, hipHostMallocDefault) != hipSuccess) return PFAC_ENOMEM;
        s.h_cap = want;
    }
    return PFAC_OK;
}

// Wait for the slot's chunk and append its matches (starts inside the chunk only).
int collect(Pipeline &p, Slot &s) {
    if (!s.busy) return PFAC_OK;
    s.busy = false;
    if (hipStreamSynchronize(s.s) != hipSuccess) return PFAC_EHIP;
    uint64_t cnt = *s.h_count;
    if (cnt == ~0ull) return PFAC_ETIMEOUT;
    if (cnt > s.cap) {
        // more matches than the slot held: grow and scan the chunk again
        int rc = grow_keys(s, cnt);
        if (rc) return rc;
        rc = pfac_scan_async(p.a, s.d_text, s.len, s.d_keys, s.cap, s.d_count, s.s);
        if (rc) return rc;
        if (hipMemcpyAsync(s.h_count, s.d_count, 8, hipMemcpyDeviceToHost, s.s) != hipSuccess) return PFAC_EHIP;
        if (hipStreamSynchronize(s.s) != hipSuccess) return PFAC_EHIP;
        cnt = *s.h_count;
        if (cnt > s.cap) return PFAC_EINTERNAL;
    }
    if (cnt == 0) return PFAC_OK;
    int rc = grow_keys(s, cnt);
    if (rc) return rc;
    if (hipMemcpyAsync(s.h_keys, s.d_keys, cnt * 8, hipMemcpyDeviceToHost, s.s) != hipSuccess) return PFAC_EHIP;
    if (hipStreamSynchronize(s.s) != hipSuccess) return PFAC_EHIP;
    // keys are sorted: the ones that start in the halo form the tail
    const uint64_t lim = s.own << 32;
    const uint64_t keep = (uint64_t)(std::lower_bound(s.h_keys, s.h_keys + cnt, lim) - s.h_keys);
    const size_t at = p.out.size();
    p.out.resize(at + keep);
    for (uint64_t i = 0; i < keep; i++) {
        const uint64_t k = s.h_keys[i];
        p.out[at + i].start = s.base + (k >> 32);
        p.out[at + i].pattern_id = (uint32_t)k;
        p.out[at + i].reserved = 0;
    }
    return PFAC_OK;
}

}  // namespace

extern "C" int pfac_scan_host(pfac_automaton *a, const uint8_t *h_text, uint64_t n, uint64_t chunk_bytes,
                              pfac_matches *out) {
    if (!out) return PFAC_EINVAL;
    out->matches = nullptr;
    out->count = 0;
    if (!a || (n > 0 && !h_text)) return PFAC_EINVAL;
    if (chunk_bytes == 0) chunk_bytes = 64ull << 20;
    const uint64_t halo = a->max_len > 0 ? a->max_len - 1 : 0;
    if (chunk_bytes + halo >= (1ull << 32)) return PFAC_ETOO_LARGE;
    if (n == 0 || a->n_pats == 0) return PFAC_OK;
    Pipeline *pp = new (std::nothrow) Pipeline{a, h_text, n, false, {}, {}};
    if (!pp) return PFAC_ENOMEM;
    Pipeline &p = *pp;
    int rc = PFAC_OK;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, h_text) == hipSuccess && attr.type == hipMemoryTypeHost)
        p.pinned_input = true;
    (void)hipGetLastError();  // a pageable pointer leaves an error behind
    const uint64_t buf = std::min<uint64_t>(chunk_bytes, n) + halo;
    for (Slot &s : p.slot) {
        if (rc) break;
        if (hipStreamCreateWithFlags(&s.s, hipStreamNonBlocking) != hipSuccess) rc = PFAC_EHIP;
        if (!rc && !p.pinned_input && hipHostMalloc(&s.h_stage, buf, hipHostMallocDefault) != hipSuccess)
            rc = PFAC_ENOMEM;
        if (!rc && hipMalloc(&s.d_text, buf) != hipSuccess) rc = PFAC_ENOMEM;
        if (!rc && hipMalloc(&s.d_count, 8) != hipSuccess) rc = PFAC_ENOMEM;
        if (!rc && hipHostMalloc(&s.h_count, 8, hipHostMallocDefault) != hipSuccess) rc = PFAC_ENOMEM;
        if (!rc) rc = grow_keys(s, 1 + buf / 1024);
    }
    try {
        uint64_t i = 0;
        for (uint64_t a0 = 0; !rc && a0 < n; a0 += chunk_bytes, i++) {
            Slot &s = p.slot[i & 1];
            rc = collect(p, s);  // the chunk this slot held two steps ago
            if (rc) break;
            s.base = a0;
            s.own = std::min(chunk_bytes, n - a0);
            s.len = std::min(n, a0 + s.own + halo) - a0;
            const uint8_t *src = h_text + a0;
            if (!p.pinned_input) {
                memcpy(s.h_stage, src, s.len);
                src = s.h_stage;
            }
            if (hipMemcpyAsync(s.d_text, src, s.len, hipMemcpyHostToDevice, s.s) != hipSuccess) {
                rc = PFAC_EHIP;
                break;
            }
            rc = pfac_scan_async(a, s.d_text, s.len, s.d_keys, s.cap, s.d_count, s.s);
            if (rc) break;
            if (hipMemcpyAsync(s.h_count, s.d_count, 8, hipMemcpyDeviceToHost, s.s) != hipSuccess) {
                rc = PFAC_EHIP;
                break;
            }
            s.busy = true;
            // collect the previous chunk while this one runs (keeps the output in order)
            rc = collect(p, p.slot[(i + 1) & 1]);
        }
        if (!rc) rc = collect(p, p.slot[0]);
        if (!rc) rc = collect(p, p.slot[1]);
    } catch (const std::bad_alloc &) {
        rc = PFAC_ENOMEM;
    }
    if (!rc && !p.out.empty()) {
        out->matches = (pfac_match *)malloc(p.out.size() * sizeof(pfac_match));
        if (!out->matches) rc = PFAC_ENOMEM;
        else {
            memcpy(out->matches, p.out.data(), p.out.size() * sizeof(pfac_match));
            out->count = p.out.size();
        }
    }
    delete pp;
    return rc;
}

extern "C" void pfac_matches_free(pfac_matches *m) {
    if (!m) return;
    free(m->matches);
    m->matches = nullptr;
    m->count = 0;
}
