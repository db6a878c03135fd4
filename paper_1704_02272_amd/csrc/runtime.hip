// Device side of the library: table upload, per-stream scratch, scan launches.
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "pfac.h"
#include "kernels.h"
#include "pfac_impl.h"
#include "scan_internal.h"

namespace pfac {

struct Workspace {
    int device = -1;
    uint64_t cap_blocks = 0;  // plain scan: per-block counts and offsets
    uint64_t *block_counts = nullptr, *block_offsets = nullptr;
    uint64_t cap_spans = 0;   // tiled scan: per-span results
    uint64_t cap_recs = 0;    // tiled scan: match records (all spans)
    SpanOut so{};
    uint64_t cap_tiles = 0;   // tiled scan: look-back words (one per placement block)
    TileState ts{};
    uint64_t launches = 0;    // tiled launches since the look-back words were last cleared
    uint64_t *d_count = nullptr;  // count for the blocking scan
    uint64_t *h_count = nullptr;  // pinned host mirror
};

namespace {

__global__ void set_u64_kernel(uint64_t *dst, uint64_t v) { *dst = v; }

// Order-sensitive digest of the first min(*count, cap) keys: the wrapping sum over i of
// SplitMix64's output mix applied to key_i ^ (i * golden ratio). The autotuner compares it
// with the first scan's, so a candidate tuning must reproduce the keys, not only their
// count. *out must be zero before the launch.
__global__ void keys_digest_kernel(const uint64_t *__restrict__ keys, const uint64_t *__restrict__ count, uint64_t cap,
                                   unsigned long long *out) {
    uint64_t n = *count;
    if (n > cap) n = cap;
    uint64_t acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t z = keys[i] ^ (i * 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        acc += z ^ (z >> 31);
    }
    for (int o = 32; o; o >>= 1) acc += __shfl_xor((unsigned long long)acc, o);
    if ((threadIdx.x & 63) == 0) atomicAdd(out, (unsigned long long)acc);
}

int check_device(int device) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return PFAC_ENODEVICE;
    if (device < 0 || device >= n) return PFAC_ENODEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return PFAC_EHIP;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return PFAC_ENODEVICE;
    return PFAC_OK;
}

template <typename T>
int upload_vec(const std::vector<T> &v, void **dst) {
    size_t bytes = v.size() * sizeof(T);
    if (bytes == 0) bytes = sizeof(T);  // keep a valid pointer for empty arrays
    if (hipMalloc(dst, bytes) != hipSuccess) return PFAC_ENOMEM;
    if (!v.empty() && hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return PFAC_EHIP;
    return PFAC_OK;
}

void free_tiles(Workspace *w) {
    hipFree(w->ts.word);
    hipFree(w->ts.ctrl);
    w->ts = TileState{};
    w->cap_tiles = 0;
    hipFree(w->so.cnt);
    hipFree(w->so.nh);
    hipFree(w->so.ovf);
    hipFree(w->so.rec);
    w->so = SpanOut{};
    w->cap_spans = 0;
    w->cap_recs = 0;
}

__global__ void clear_tiles_kernel(uint64_t *word, uint64_t n, uint32_t *ctrl) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        word[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl[0] = 0;
        ctrl[1] = 0;
        ctrl[2] = 1;
        ctrl[3] = 0;
    }
}

void free_workspace(Workspace *w) {
    if (!w) return;
    free_tiles(w);
    hipFree(w->block_counts);
    hipFree(w->block_offsets);
    hipFree(w->d_count);
    hipHostFree(w->h_count);
    delete w;
}

void free_copy(DeviceCopy *c) {
    if (!c) return;
    int prev = 0;
    hipGetDevice(&prev);
    hipSetDevice(c->device);
    for (auto &kv : c->workspaces) free_workspace(kv.second);
    hipFree(c->nodes);
    hipFree(c->bm);
    hipFree(c->out_first);
    hipFree(c->out_ids);
    hipFree(c->lds_image);
    hipFree(c->tails);
    hipFree(c->tail_bytes);
    hipFree(c->tail_head);
    hipFree(c->rk);
    for (void *p : c->retired) hipFree(p);
    hipSetDevice(prev);
    delete c;
}

}  // namespace

int launch_set_u64(uint64_t *dst, uint64_t value, hipStream_t s) {
    set_u64_kernel<<<1, 1, 0, s>>>(dst, value);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

void release_stream(pfac_automaton *a, void *stream) {
    if (!a) return;
    std::lock_guard<std::mutex> g(a->mu);
    int prev = 0;
    (void)hipGetDevice(&prev);
    for (DeviceCopy *c : a->copies) {
        auto it = c->workspaces.find(stream);
        if (it == c->workspaces.end()) continue;
        (void)hipSetDevice(c->device);
        if (stream) (void)hipStreamSynchronize((hipStream_t)stream);
        free_workspace(it->second);
        c->workspaces.erase(it);
    }
    (void)hipSetDevice(prev);
}

size_t workspace_count(pfac_automaton *a) {
    if (!a) return 0;
    std::lock_guard<std::mutex> g(a->mu);
    size_t k = 0;
    for (DeviceCopy *c : a->copies) k += c->workspaces.size();
    return k;
}

void release_device_copies(pfac_automaton *a) {
    for (DeviceCopy *c : a->copies) free_copy(c);
    a->copies.clear();
}

// Scratch of pfac_scan_noalloc: one array per device, kept until the process ends. Host
// code never uses the array's name as an address (that is a host-side stand-in); it uses
// the device address hipGetSymbolAddress returns, fetched once per device.
// Layout for up to kNoAllocSpans spans with 2^kNoAllocRecLog2 records each:
//   [records: spans << rec_log2 u64][cnt: spans u64][nh: spans u32][ovf: spans u32]
//   [look-back words: spans / kBlockSpans u64][ctrl: 4 u32]
constexpr uint32_t kNoAllocSpans = 4096;
constexpr uint32_t kNoAllocRecLog2 = 8;
constexpr uint64_t kNoAllocRecBytes = ((uint64_t)kNoAllocSpans << kNoAllocRecLog2) * 8;
constexpr uint64_t kNoAllocBytes = kNoAllocRecBytes + (uint64_t)kNoAllocSpans * 16 +
                                   (uint64_t)(kNoAllocSpans / kBlockSpans) * 8 + 16;
static_assert(kNoAllocSpans <= kDirectMaxSpans, "placement without look-back: no state carried between calls");
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kNoAllocMaxDevices];  // device address of `scratch` per device, once fetched

// Device address of the scratch array on device `dev` (current), fetched on first use.
static int scratch_address(int dev, uint8_t **out) {
    if (dev < 0 || dev >= kNoAllocMaxDevices) return PFAC_ENODEVICE;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PFAC_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = (uint8_t *)g_scratch_ptr[dev];
    return PFAC_OK;
}

// Device copy for the current device, uploading it on first use. Caller holds a->mu.
static int get_copy(pfac_automaton *a, DeviceCopy **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PFAC_ENODEVICE;
    for (DeviceCopy *c : a->copies)
        if (c->device == dev) {
            *out = c;
            return PFAC_OK;
        }
    int rc = check_device(dev);
    if (rc) return rc;
    DeviceCopy *c = new (std::nothrow) DeviceCopy();
    if (!c) return PFAC_ENOMEM;
    c->device = dev;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        c->cus = (uint32_t)cus;
    rc = upload_vec(a->dev_nodes, &c->nodes);
    if (!rc && a->layout == LAYOUT_WIDE) rc = upload_vec(a->dev_bm, &c->bm);
    // ids by device record and tail (plain table), or by rank of the spelled string plus
    // the rank words (compressed table)
    if (!rc) rc = upload_vec(a->dev_out_first, &c->out_first);
    if (!rc) rc = upload_vec(a->dev_out_ids, &c->out_ids);
    if (!rc && a->merge_levels) rc = upload_vec(a->rec_rank, &c->rk);
    if (!rc) rc = upload_vec(a->lds_image, &c->lds_image);
    if (!rc) rc = upload_vec(a->dev_tails, &c->tails);
    if (!rc) rc = upload_vec(a->pat_bytes, &c->tail_bytes);
    if (!rc) rc = upload_vec(a->dev_tail_head, &c->tail_head);
    if (rc) {
        free_copy(c);
        return rc;
    }
    c->view = a->shape;
    c->view.nodes = (const uint64_t *)c->nodes;
    c->view.bm = (const uint64_t *)c->bm;
    c->view.out_first = (const uint32_t *)c->out_first;
    c->view.out_ids = (const uint32_t *)c->out_ids;
    c->view.lds_image = (const uint32_t *)c->lds_image;
    c->view.tails = (const uint32_t *)c->tails;
    c->view.tail_bytes = (const uint8_t *)c->tail_bytes;
    c->view.tail_head = (const uint4 *)c->tail_head;
    c->view.rk = (const uint32_t *)c->rk;
    // set-up of pfac_scan_noalloc on this device (its scratch array's device address);
    // a failure here is reported by that call, which tries again
    uint8_t *sp = nullptr;
    (void)scratch_address(dev, &sp);
    a->copies.push_back(c);
    *out = c;
    return PFAC_OK;
}

static int ensure_tiles(Workspace *w, uint64_t n, uint32_t span_log2, void *stream);

static int get_workspace(DeviceCopy *c, void *stream, uint64_t n, uint32_t algo, uint32_t span_log2,
                         Workspace **out) {
    Workspace *&w = c->workspaces[stream];
    if (!w) {
        w = new (std::nothrow) Workspace();
        if (!w) return PFAC_ENOMEM;
        w->device = c->device;
        if (hipMalloc(&w->d_count, sizeof(uint64_t)) != hipSuccess) return PFAC_ENOMEM;
        if (hipHostMalloc(&w->h_count, sizeof(uint64_t), hipHostMallocDefault) != hipSuccess)
            return PFAC_ENOMEM;
    }
    if (algo == PFAC_ALGO_TILED) {
        const int rc = ensure_tiles(w, n, span_log2, stream);
        if (rc) return rc;
        *out = w;
        return PFAC_OK;
    }
    uint64_t nb = plain_blocks(n);
    if (nb > w->cap_blocks) {
        // the stream may still use the old buffers
        if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return PFAC_EHIP;
        hipFree(w->block_counts);
        hipFree(w->block_offsets);
        w->block_counts = w->block_offsets = nullptr;
        w->cap_blocks = 0;
        uint64_t want = nb < 1024 ? 1024 : nb + nb / 4;
        if (hipMalloc(&w->block_counts, want * 8) != hipSuccess) return PFAC_ENOMEM;
        if (hipMalloc(&w->block_offsets, want * 8) != hipSuccess) return PFAC_ENOMEM;
        w->cap_blocks = want;
    }
    *out = w;
    return PFAC_OK;
}

}  // namespace pfac

using namespace pfac;


extern "C" int pfac_upload(pfac_automaton *a, int device) {
    if (!a) return PFAC_EINVAL;
    int rc = check_device(device);
    if (rc) return rc;
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return PFAC_EHIP;
    if (hipSetDevice(device) != hipSuccess) return PFAC_EHIP;
    DeviceCopy *c = nullptr;
    {
        std::lock_guard<std::mutex> g(a->mu);
        rc = get_copy(a, &c);
    }
    hipSetDevice(prev);
    return rc;
}

namespace pfac {

// Tiled-path scratch for n bytes in workspace w (grown on demand; the stream is drained
// before old buffers are freed). Clears the look-back words before the epoch could wrap.
static int ensure_tiles(Workspace *w, uint64_t n, uint32_t span_log2, void *stream) {
    const uint64_t ns = (n + (1ull << span_log2) - 1) >> span_log2;
    const uint64_t nrec = ns << rec_cap_log2(span_log2);
    if (ns > w->cap_spans || nrec > w->cap_recs || !w->ts.ctrl) {
        if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return PFAC_EHIP;
        const uint64_t old_spans = w->cap_spans, old_recs = w->cap_recs;
        free_tiles(w);
        uint64_t spans = ns < 1024 ? 1024 : ns + ns / 4;
        if (spans < old_spans) spans = old_spans;
        uint64_t recs = spans << rec_cap_log2(span_log2);
        if (recs < old_recs) recs = old_recs;
        const uint64_t blocks = (spans + kBlockSpans - 1) / kBlockSpans;
        if (hipMalloc(&w->so.cnt, spans * 8) != hipSuccess) return PFAC_ENOMEM;
        if (hipMalloc(&w->so.nh, spans * 4) != hipSuccess) return PFAC_ENOMEM;
        if (hipMalloc(&w->so.ovf, spans * 4) != hipSuccess) return PFAC_ENOMEM;
        if (hipMalloc(&w->so.rec, recs * 8) != hipSuccess) return PFAC_ENOMEM;
        if (hipMalloc(&w->ts.word, blocks * 8) != hipSuccess) return PFAC_ENOMEM;
        if (hipMalloc(&w->ts.ctrl, 16) != hipSuccess) return PFAC_ENOMEM;
        w->cap_spans = spans;
        w->cap_recs = recs;
        w->cap_tiles = blocks;
        w->launches = kEpochPeriod;  // forces a clear before the first launch
    }
    if (w->launches >= kEpochPeriod) {
        // words 0 never match an epoch (epochs start at 1); clearing before the device
        // epoch can wrap keeps stale words from ever matching
        clear_tiles_kernel<<<256, 256, 0, (hipStream_t)stream>>>(w->ts.word, w->cap_tiles, w->ts.ctrl);
        if (hipGetLastError() != hipSuccess) return PFAC_EHIP;
        w->launches = 0;
    }
    return PFAC_OK;
}

}  // namespace pfac

namespace pfac {
int reserve_stream(pfac_automaton *a, void *stream, uint64_t n) {
    if (!a || n >= (1ull << 32)) return PFAC_EINVAL;
    std::lock_guard<std::mutex> g(a->mu);
    DeviceCopy *c = nullptr;
    int rc = get_copy(a, &c);
    if (rc) return rc;
    const uint32_t span_log2 = a->span_log2 ? a->span_log2 : auto_span_log2(n, (uint64_t)c->cus * kWaves);
    Workspace *w = nullptr;
    return get_workspace(c, stream, n, PFAC_ALGO_TILED, span_log2, &w);
}
}  // namespace pfac

// Enqueue one scan of a text (offsets == null) or a packet batch.
static int scan_enqueue(pfac_automaton *a, const uint8_t *d_text, uint64_t n, const uint64_t *d_offsets,
                        uint32_t n_pkts, uint64_t *d_keys, uint64_t cap, uint64_t *d_count, void *stream,
                        Workspace **ws_out) {
    if (!a) return PFAC_EINVAL;
    if (n > 0 && !d_text) return PFAC_EINVAL;
    if (cap > 0 && !d_keys) return PFAC_EINVAL;
    if (n >= (1ull << 32)) return PFAC_ETOO_LARGE;
    hipStream_t s = (hipStream_t)stream;
    std::lock_guard<std::mutex> g(a->mu);
    DeviceCopy *c = nullptr;
    int rc = get_copy(a, &c);
    if (rc) return rc;
    const bool batch = d_offsets != nullptr;
    const uint32_t algo = (a->algo == PFAC_ALGO_PLAIN && !batch) ? PFAC_ALGO_PLAIN : PFAC_ALGO_TILED;
    Workspace *w = nullptr;
    const uint32_t span_log2 = a->span_log2 ? a->span_log2 : auto_span_log2(n, (uint64_t)c->cus * kWaves);
    rc = get_workspace(c, stream, n, algo, span_log2, &w);
    if (rc) return rc;
    if (ws_out) *ws_out = w;
    uint64_t *cnt = d_count ? d_count : w->d_count;
    if (n == 0 || a->n_pats == 0 || (batch && n_pkts == 0)) return launch_set_u64(cnt, 0, s) ? PFAC_EHIP : PFAC_OK;
    if (algo == PFAC_ALGO_PLAIN) {
        if (launch_plain(c->view, d_text, n, d_keys, cap, cnt, w->block_counts, w->block_offsets, s))
            return PFAC_EHIP;
        return PFAC_OK;
    }
    const uint64_t ns = (n + (1ull << span_log2) - 1) >> span_log2;
    const uint32_t grid = a->grid ? (uint32_t)std::min<uint64_t>(a->grid, (ns + kWaves - 1) / kWaves) : 0u;
    if (launch_tiled(c->view, d_text, n, d_offsets, n_pkts, d_keys, cap, cnt, w->so, w->ts, nullptr, grid,
                     span_log2, a->lane_bytes, s))
        return PFAC_EHIP;
    w->launches++;
    return PFAC_OK;
}

static int finish_count(Workspace *w, uint64_t cap, uint64_t *h_count, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(w->h_count, w->d_count, sizeof(uint64_t), hipMemcpyDeviceToHost, s) != hipSuccess)
        return PFAC_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return PFAC_EHIP;
    *h_count = *w->h_count;
    if (*h_count == kCountTimeout) return PFAC_ETIMEOUT;
    if (*h_count == kCountOverflow) return PFAC_ETOO_LARGE;
    return *h_count > cap ? PFAC_ECAPACITY : PFAC_OK;
}

extern "C" int pfac_scan_async(pfac_automaton *a, const uint8_t *d_text, uint64_t n,
                               uint64_t *d_keys, uint64_t cap, uint64_t *d_count, void *stream) {
    if (!d_count) return PFAC_EINVAL;
    return scan_enqueue(a, d_text, n, nullptr, 0, d_keys, cap, d_count, stream, nullptr);
}

extern "C" int pfac_scan(pfac_automaton *a, const uint8_t *d_text, uint64_t n, uint64_t *d_keys,
                         uint64_t cap, uint64_t *h_count, void *stream) {
    if (!h_count) return PFAC_EINVAL;
    Workspace *w = nullptr;
    int rc = scan_enqueue(a, d_text, n, nullptr, 0, d_keys, cap, nullptr, stream, &w);
    if (rc) return rc;
    return finish_count(w, cap, h_count, stream);
}

extern "C" int pfac_scan_batch_async(pfac_automaton *a, const uint8_t *d_bytes, const uint64_t *d_offsets,
                                     uint32_t n_pkts, uint64_t n_bytes, uint64_t *d_keys, uint64_t cap,
                                     uint64_t *d_count, void *stream) {
    if (!d_count || (!d_offsets && n_pkts > 0)) return PFAC_EINVAL;
    if (n_pkts == 0) return scan_enqueue(a, d_bytes, 0, nullptr, 0, d_keys, cap, d_count, stream, nullptr);
    return scan_enqueue(a, d_bytes, n_bytes, d_offsets, n_pkts, d_keys, cap, d_count, stream, nullptr);
}

extern "C" int pfac_scan_batch(pfac_automaton *a, const uint8_t *d_bytes, const uint64_t *d_offsets,
                               uint32_t n_pkts, uint64_t n_bytes, uint64_t *d_keys, uint64_t cap,
                               uint64_t *h_count, void *stream) {
    if (!h_count || (!d_offsets && n_pkts > 0)) return PFAC_EINVAL;
    Workspace *w = nullptr;
    int rc = n_pkts == 0 ? scan_enqueue(a, d_bytes, 0, nullptr, 0, d_keys, cap, nullptr, stream, &w)
                         : scan_enqueue(a, d_bytes, n_bytes, d_offsets, n_pkts, d_keys, cap, nullptr, stream, &w);
    if (rc) return rc;
    return finish_count(w, cap, h_count, stream);
}

// ------------------------------------------------------------------ scans that allocate nothing
extern "C" int pfac_scan_noalloc(pfac_automaton *a, const uint8_t *d_text, uint64_t n, uint64_t *d_keys,
                                 uint64_t cap, uint64_t *d_count, void *stream) {
    if (!a || !d_count || (n > 0 && !d_text) || (cap > 0 && !d_keys)) return PFAC_EINVAL;
    if (n >= (1ull << 32)) return PFAC_ETOO_LARGE;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PFAC_ENODEVICE;
    std::lock_guard<std::mutex> g(a->mu);
    DeviceCopy *c = nullptr;
    for (DeviceCopy *x : a->copies)
        if (x->device == dev) c = x;
    if (!c) return PFAC_EINVAL;  // not on this device yet: pfac_upload allocates, this call does not
    uint8_t *base = nullptr;
    int rc = scratch_address(dev, &base);
    if (rc) return rc;
    if (n == 0 || a->n_pats == 0) return launch_set_u64(d_count, 0, s) ? PFAC_EHIP : PFAC_OK;
    // the span length chosen by text size, lengthened until the spans fit the scratch
    // (results do not depend on it); a tuned length is kept as it is
    uint32_t span_log2 = a->span_log2 ? a->span_log2 : auto_span_log2(n, (uint64_t)c->cus * kWaves);
    auto spans = [&](uint32_t sl) { return (n + (1ull << sl) - 1) >> sl; };
    if (!a->span_log2)
        while (spans(span_log2) > kNoAllocSpans && span_log2 < kMaxSpanLog2) span_log2++;
    const uint64_t ns = spans(span_log2);
    if (ns > kNoAllocSpans) return PFAC_ETOO_LARGE;  // more spans than the scratch holds
    SpanOut so{};
    so.rec = (uint64_t *)base;
    so.cnt = (uint64_t *)(base + kNoAllocRecBytes);
    so.nh = (uint32_t *)(base + kNoAllocRecBytes + (uint64_t)kNoAllocSpans * 8);
    so.ovf = (uint32_t *)(base + kNoAllocRecBytes + (uint64_t)kNoAllocSpans * 12);
    so.rec_log2 = kNoAllocRecLog2;  // fewer records than a workspace keeps: a span past them is walked again
    TileState ts{};
    ts.word = (uint64_t *)(base + kNoAllocRecBytes + (uint64_t)kNoAllocSpans * 16);
    ts.ctrl = (uint32_t *)(base + kNoAllocRecBytes + (uint64_t)kNoAllocSpans * 16 +
                           (uint64_t)(kNoAllocSpans / kBlockSpans) * 8);
    const uint32_t grid = a->grid ? (uint32_t)std::min<uint64_t>(a->grid, (ns + kWaves - 1) / kWaves) : 0u;
    // every span's count, record count and overflow are written by the count kernel
    // before the placement reads them, and placement of this many spans uses no
    // look-back state: nothing in the array needs clearing between calls
    if (launch_tiled(c->view, d_text, n, nullptr, 0, d_keys, cap, d_count, so, ts, nullptr, grid, span_log2,
                     a->lane_bytes, s))
        return PFAC_EHIP;
    return PFAC_OK;
}

// ------------------------------------------------------------------ prefix depths
extern "C" int pfac_prefix_histogram(pfac_automaton *a, const uint8_t *d_text, uint64_t n, uint32_t cap,
                                     uint64_t *d_hist, void *stream) {
    if (!a || !d_hist || (n > 0 && !d_text) || cap == 0 || cap > 63) return PFAC_EINVAL;
    std::lock_guard<std::mutex> g(a->mu);
    DeviceCopy *c = nullptr;
    int rc = get_copy(a, &c);
    if (rc) return rc;
    return launch_prefix_hist(c->view, d_text, n, cap, d_hist, c->cus, (hipStream_t)stream) ? PFAC_EHIP : PFAC_OK;
}

// ------------------------------------------------------------------ captured graphs
struct pfac_graph {
    pfac_automaton *a = nullptr;
    int device = -1;
    Workspace ws;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static void graph_free(pfac_graph *g) {
    if (!g) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    if (g->device >= 0) (void)hipSetDevice(g->device);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    free_tiles(&g->ws);
    (void)hipSetDevice(prev);
    delete g;
}

extern "C" int pfac_graph_create(pfac_automaton *a, const uint8_t *d_bytes, const uint64_t *d_offsets,
                                 uint64_t max_bytes, uint32_t max_pkts, uint64_t *d_keys, uint64_t cap,
                                 uint64_t *d_count, const uint64_t *d_sizes, void *stream, pfac_graph **out) {
    if (!out) return PFAC_EINVAL;
    *out = nullptr;
    if (!a || !stream || !d_bytes || !d_count || !d_sizes || max_bytes == 0 || (cap > 0 && !d_keys))
        return PFAC_EINVAL;
    if (d_offsets && max_pkts == 0) return PFAC_EINVAL;
    if (max_bytes >= (1ull << 32)) return PFAC_ETOO_LARGE;
    if (a->n_pats == 0) return PFAC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    pfac_graph *g = new (std::nothrow) pfac_graph();
    if (!g) return PFAC_ENOMEM;
    g->a = a;
    DevTable view{};
    uint32_t span_log2 = kSpanLog2, grid = 0, lane_bytes = 32;
    {
        std::lock_guard<std::mutex> lk(a->mu);
        grid = a->grid;
        lane_bytes = a->lane_bytes;
        DeviceCopy *c = nullptr;
        int rc = get_copy(a, &c);
        if (rc) {
            delete g;
            return rc;
        }
        g->device = c->device;
        view = c->view;
        span_log2 = a->span_log2 ? a->span_log2 : auto_span_log2(max_bytes, (uint64_t)c->cus * kWaves);
    }
    // everything that allocates happens before the capture
    int rc = ensure_tiles(&g->ws, max_bytes, span_log2, stream);
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = PFAC_EHIP;
    if (!rc && hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = PFAC_EHIP;
    if (!rc) {
        const int lr = launch_tiled(view, d_bytes, max_bytes, d_offsets, d_offsets ? max_pkts : 0, d_keys, cap,
                                    d_count, g->ws.so, g->ws.ts, d_sizes, grid, span_log2, lane_bytes, s);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(s, &graph);
        g->graph = graph;
        if (lr || ec != hipSuccess || !graph) rc = PFAC_EHIP;
    }
    if (!rc && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) rc = PFAC_EHIP;
    if (rc) {
        graph_free(g);
        return rc;
    }
    *out = g;
    return PFAC_OK;
}

extern "C" int pfac_graph_launch(pfac_graph *g, void *stream) {
    if (!g || !g->exec) return PFAC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (g->ws.launches >= kEpochPeriod) {
        clear_tiles_kernel<<<256, 256, 0, s>>>(g->ws.ts.word, g->ws.cap_tiles, g->ws.ts.ctrl);
        if (hipGetLastError() != hipSuccess) return PFAC_EHIP;
        g->ws.launches = 0;
    }
    if (hipGraphLaunch(g->exec, s) != hipSuccess) return PFAC_EHIP;
    g->ws.launches++;
    return PFAC_OK;
}

extern "C" void pfac_graph_destroy(pfac_graph *g) { graph_free(g); }

// Give every device copy the new LDS image after the host image changed. The old image
// is retired, not freed: queued scans and captured graphs keep reading it.
static int reupload_lds_images(pfac_automaton *a) {
    if (a->copies.empty()) return PFAC_OK;  // nothing on any device yet
    int prev = 0;
    if (hipGetDevice(&prev) != hipSuccess) return PFAC_EHIP;
    int rc = PFAC_OK;
    for (DeviceCopy *c : a->copies) {
        if (hipSetDevice(c->device) != hipSuccess) {
            rc = PFAC_EHIP;
            break;
        }
        void *img = nullptr;
        rc = upload_vec(a->lds_image, &img);
        if (rc) {
            hipFree(img);
            break;
        }
        c->retired.push_back(c->lds_image);
        c->lds_image = img;
        DevTable v = a->shape;
        v.nodes = c->view.nodes;
        v.bm = c->view.bm;
        v.out_first = c->view.out_first;
        v.out_ids = c->view.out_ids;
        v.tails = c->view.tails;
        v.tail_bytes = c->view.tail_bytes;
        v.tail_head = c->view.tail_head;
        v.rk = c->view.rk;
        v.lds_image = (const uint32_t *)c->lds_image;
        c->view = v;
    }
    (void)hipSetDevice(prev);
    return rc;
}

static int set_tuning_locked(pfac_automaton *a, const pfac_tuning *t) {
    if (t->algo > PFAC_ALGO_TILED) return PFAC_EINVAL;
    if (t->algo == PFAC_ALGO_PLAIN && a->merge_levels) return PFAC_EINVAL;  // the baseline walks the plain trie
    const uint32_t span = t->span_log2;  // 0: chosen per scan from the text size
    if (span && (span < kMinSpanLog2 || span > kMaxSpanLog2)) return PFAC_EINVAL;
    if (t->lane_bytes != 0 && t->lane_bytes != 16 && t->lane_bytes != 32) return PFAC_EINVAL;
    if (t->grid > 0xffffffu) return PFAC_EINVAL;
    if (t->root_depth != a->req_depth || t->filter_k != a->req_k) {
        int rc = rebuild_lds_image(a, t->root_depth, t->filter_k);
        if (rc) {
            // keep the previous image in force
            (void)rebuild_lds_image(a, a->req_depth, a->req_k);
            return rc;
        }
        a->req_depth = t->root_depth;
        a->req_k = t->filter_k;
        rc = reupload_lds_images(a);
        if (rc) return rc;
    }
    a->algo = t->algo;
    a->grid = t->grid;
    a->span_log2 = span;
    a->lane_bytes = t->lane_bytes == 16 ? 16u : 32u;
    return PFAC_OK;
}

extern "C" int pfac_set_tuning(pfac_automaton *a, const pfac_tuning *t) {
    if (!a || !t) return PFAC_EINVAL;
    std::lock_guard<std::mutex> g(a->mu);
    return set_tuning_locked(a, t);
}

extern "C" int pfac_get_tuning(const pfac_automaton *a, pfac_tuning *t) {
    if (!a || !t) return PFAC_EINVAL;
    memset(t, 0, sizeof(*t));
    t->algo = a->algo == PFAC_ALGO_PLAIN ? PFAC_ALGO_PLAIN : PFAC_ALGO_TILED;
    t->grid = a->grid;
    t->span_log2 = a->span_log2;
    t->root_depth = a->shape.root_depth;
    t->filter_k = a->shape.filter_k ? a->shape.filter_k : a->shape.root_depth;
    // the sampled prefilter form takes 32 bytes a lane whatever was asked for
    t->lane_bytes = a->shape.sampled ? 32u : a->lane_bytes;
    return PFAC_OK;
}

// ------------------------------------------------------------------ autotuner
namespace {

struct TuneRun {
    pfac_automaton *a;
    const uint8_t *d_bytes;
    uint64_t n;
    const uint64_t *d_offsets;
    uint32_t n_pkts;
    uint32_t reps;
    hipStream_t s;
    uint64_t *d_keys = nullptr, cap = 0, *d_count = nullptr, *d_digest = nullptr;
    uint64_t want = ~0ull;         // the match count every candidate must reproduce
    uint64_t want_digest = 0;      // and the digest of its keys
    hipEvent_t e0 = nullptr, e1 = nullptr;
};

int tune_enqueue(TuneRun &r) {
    if (r.d_offsets)
        return scan_enqueue(r.a, r.d_bytes, r.n, r.d_offsets, r.n_pkts, r.d_keys, r.cap, r.d_count, r.s, nullptr);
    return scan_enqueue(r.a, r.d_bytes, r.n, nullptr, 0, r.d_keys, r.cap, r.d_count, r.s, nullptr);
}

// Digest of the keys of the last scan enqueued (see keys_digest_kernel), on the host.
int tune_digest(TuneRun &r, uint64_t *out) {
    if (launch_set_u64(r.d_digest, 0, r.s)) return PFAC_EHIP;
    keys_digest_kernel<<<64, 256, 0, r.s>>>(r.d_keys, r.d_count, r.cap, (unsigned long long *)r.d_digest);
    if (hipGetLastError() != hipSuccess) return PFAC_EHIP;
    if (hipMemcpyAsync(out, r.d_digest, 8, hipMemcpyDeviceToHost, r.s) != hipSuccess) return PFAC_EHIP;
    return hipStreamSynchronize(r.s) == hipSuccess ? PFAC_OK : PFAC_EHIP;
}

// Mean milliseconds per scan under the automaton's current tuning (one warm-up scan, then
// `reps` timed). Checks that the count and the keys' digest are the ones every other
// candidate produced.
int tune_measure(TuneRun &r, float *ms) {
    int rc = tune_enqueue(r);
    if (rc) return rc;
    if (hipEventRecord(r.e0, r.s) != hipSuccess) return PFAC_EHIP;
    for (uint32_t i = 0; i < r.reps; i++)
        if ((rc = tune_enqueue(r))) return rc;
    if (hipEventRecord(r.e1, r.s) != hipSuccess || hipEventSynchronize(r.e1) != hipSuccess) return PFAC_EHIP;
    float t = 0;
    if (hipEventElapsedTime(&t, r.e0, r.e1) != hipSuccess) return PFAC_EHIP;
    uint64_t cnt = 0;
    if (hipMemcpy(&cnt, r.d_count, 8, hipMemcpyDeviceToHost) != hipSuccess) return PFAC_EHIP;
    if (cnt == kCountTimeout) return PFAC_ETIMEOUT;
    if (cnt != r.want) return PFAC_EINTERNAL;
    uint64_t dg = 0;
    if ((rc = tune_digest(r, &dg))) return rc;
    if (dg != r.want_digest) return PFAC_EINTERNAL;
    *ms = t / (float)r.reps;
    return PFAC_OK;
}

int tune_try(TuneRun &r, const pfac_tuning &cand, float *ms) {
    {
        std::lock_guard<std::mutex> g(r.a->mu);
        int rc = set_tuning_locked(r.a, &cand);
        if (rc) return rc;
    }
    return tune_measure(r, ms);
}

}  // namespace

extern "C" int pfac_tune(pfac_automaton *a, const uint8_t *d_bytes, uint64_t n_bytes, const uint64_t *d_offsets,
                         uint32_t n_pkts, uint32_t reps, void *stream, pfac_tuning *out, float *out_ms) {
    if (!a || !out || (n_bytes > 0 && !d_bytes) || (d_offsets == nullptr && n_pkts > 0)) return PFAC_EINVAL;
    if (n_bytes >= (1ull << 32)) return PFAC_ETOO_LARGE;
    if (a->n_pats == 0 || n_bytes == 0) {
        int rc = pfac_get_tuning(a, out);
        if (out_ms) *out_ms = 0.f;
        return rc;
    }
    TuneRun r{a, d_bytes, n_bytes, d_offsets, n_pkts, reps ? reps : 5, (hipStream_t)stream};
    int rc = PFAC_OK;
    pfac_tuning start{};
    (void)pfac_get_tuning(a, &start);
    start.root_depth = a->req_depth;  // as requested, so restoring keeps the builder's choice
    start.filter_k = a->req_k;
    // the match count under the current tuning sizes the key buffer and is the answer
    // every candidate has to reproduce
    if (hipMalloc(&r.d_count, 8) != hipSuccess) return PFAC_ENOMEM;
    if (hipMalloc(&r.d_digest, 8) != hipSuccess) {
        hipFree(r.d_count);
        return PFAC_ENOMEM;
    }
    if (hipEventCreate(&r.e0) != hipSuccess || hipEventCreate(&r.e1) != hipSuccess) rc = PFAC_EHIP;
    if (!rc) rc = tune_enqueue(r);
    if (!rc && hipMemcpyAsync(&r.want, r.d_count, 8, hipMemcpyDeviceToHost, r.s) != hipSuccess) rc = PFAC_EHIP;
    if (!rc && hipStreamSynchronize(r.s) != hipSuccess) rc = PFAC_EHIP;
    if (!rc && (r.want == kCountTimeout || r.want == kCountOverflow)) rc = PFAC_ETIMEOUT;
    if (!rc) {
        r.cap = r.want;
        if (r.cap && hipMalloc(&r.d_keys, r.cap * 8) != hipSuccess) rc = PFAC_ENOMEM;
    }
    // the keys under the starting tuning, whose digest every candidate must reproduce
    if (!rc) rc = tune_enqueue(r);
    if (!rc) rc = tune_digest(r, &r.want_digest);
    pfac_tuning best = start;
    best.algo = PFAC_ALGO_TILED;
    best.root_depth = a->req_depth;
    best.filter_k = a->req_k;
    float best_ms = 0.f;
    if (!rc) rc = tune_try(r, best, &best_ms);
    // coordinate descent: span length, then root depth, then filter key, then positions
    // per thread, then grid
    const bool pack2 = a->alphabet <= 4;
    const uint32_t dmax = std::min(a->min_len, pack2 ? 8u : 2u);
    const uint32_t kmax = std::min(a->max_len, pack2 ? 16u : 4u);
    auto consider = [&](pfac_tuning cand) {
        if (rc) return;
        float ms = 0.f;
        const int e = tune_try(r, cand, &ms);
        if (e == PFAC_EINVAL) return;  // not a valid point for this pattern set
        if (e) {
            rc = e;
            return;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = cand;
        }
    };
    for (uint32_t sl = 11; sl <= kMaxSpanLog2; sl++) {
        if (sl == best.span_log2) continue;
        pfac_tuning c = best;
        c.span_log2 = sl;
        consider(c);
    }
    for (uint32_t d = 1; d <= dmax; d++) {
        pfac_tuning c = best;
        c.root_depth = d;
        c.filter_k = 0;  // the builder's key length for that depth
        consider(c);
    }
    {
        const uint32_t d0 = best.root_depth ? best.root_depth : dmax;
        for (uint32_t k = d0; k <= kmax; k++) {
            pfac_tuning c = best;
            c.filter_k = k;
            consider(c);
        }
    }
    {
        pfac_tuning c = best;
        c.lane_bytes = best.lane_bytes == 16 ? 32u : 16u;
        consider(c);
    }
    {
        int dev = 0, cus = 256;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        for (uint32_t g : {(uint32_t)cus / 2, (uint32_t)cus * 2}) {
            pfac_tuning c = best;
            c.grid = g;
            consider(c);
        }
    }
    // leave the automaton at the best point (or where it started, on error)
    {
        std::lock_guard<std::mutex> g(a->mu);
        const int e = set_tuning_locked(a, rc ? &start : &best);
        if (!rc) rc = e;
    }
    if (r.e0) hipEventDestroy(r.e0);
    if (r.e1) hipEventDestroy(r.e1);
    hipFree(r.d_keys);
    hipFree(r.d_count);
    hipFree(r.d_digest);
    if (!rc) {
        (void)pfac_get_tuning(a, out);
        if (out_ms) *out_ms = best_ms;
    }
    return rc;
}
