// Serving loop: continuous batching of packet requests onto a resident automaton.
//
// Requests (a few packets each, copied at submit) wait in a FIFO. The server has S
// slots, each with its own host thread; a slot holds the device memory for one batch
// (bytes, offsets, keys, count, scratch), pinned staging, a stream and a captured scan
// graph that reads its batch sizes from device memory (or scratch for eager launches).
// Whenever a slot is free and requests wait, its thread packs as many waiting requests
// as fit into one batch and launches it at once, so requests that arrive while other
// batches are on the GPU join the next free slot and batches of different slots overlap
// on the device; staging and finishing of different slots also overlap on the host. The
// number of slots is what the device-memory budget admits. A finished batch's keys are
// split back into requests (keys are global byte offsets in the batch, so each
// request's keys form one run) and reported with their arrival, launch and completion
// times.
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "pfac.h"
#include "pfac_impl.h"
#include "kernels.h"
#include "scan_internal.h"

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    uint64_t ticket = 0;
    std::vector<uint8_t> bytes;
    std::vector<uint64_t> offs;  // n_pkts + 1, from 0
    uint32_t n_pkts = 0;
    uint64_t arrival_ns = 0;
};

struct Slot {
    hipStream_t s = nullptr;
    hipEvent_t done = nullptr;
    pfac_graph *g = nullptr;
    uint8_t *d_bytes = nullptr, *h_bytes = nullptr;
    uint64_t *d_offs = nullptr, *h_offs = nullptr;
    uint64_t *d_sizes = nullptr, *h_sizes = nullptr;
    uint64_t *d_keys = nullptr, *h_keys = nullptr, cap = 0;
    uint64_t *d_count = nullptr, *h_count = nullptr;
    bool busy = false;
    std::vector<Request *> reqs;
    std::vector<uint64_t> byte0;  // first batch byte of each request, plus the end
    uint64_t launch_ns = 0;
};

struct LatSample {
    uint64_t ns;
    uint32_t pkts;
};

}  // namespace

struct pfac_server {
    pfac_automaton *a = nullptr;
    int device = 0;
    pfac_server_config cfg{};
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> pending;
    uint64_t pending_bytes = 0;
    std::deque<pfac_result> results;
    std::vector<std::thread> workers;  // one per slot
    bool stop = false;
    int fatal = PFAC_OK;  // a device error stops the server; later calls report it
    std::atomic<uint64_t> next_ticket{1};
    // statistics (under mu)
    std::vector<LatSample> lat;
    uint64_t st_requests = 0, st_packets = 0, st_bytes = 0, st_matches = 0, st_batches = 0, st_rejected = 0;
    uint64_t st_first_arrival = 0, st_last_done = 0, st_busy_slot_ns = 0;
};

namespace {

void free_slot(pfac_automaton *a, Slot &s) {
    if (s.s) pfac::release_stream(a, s.s);  // overflow rescans keep scratch keyed by the stream
    if (s.g) pfac_graph_destroy(s.g);
    if (s.done) (void)hipEventDestroy(s.done);
    hipFree(s.d_bytes);
    hipFree(s.d_offs);
    hipFree(s.d_sizes);
    hipFree(s.d_keys);
    hipFree(s.d_count);
    hipHostFree(s.h_bytes);
    hipHostFree(s.h_offs);
    hipHostFree(s.h_sizes);
    hipHostFree(s.h_keys);
    hipHostFree(s.h_count);
    if (s.s) (void)hipStreamDestroy(s.s);
    s = Slot{};
}

int alloc_slot(pfac_server *sv, Slot &s) {
    const pfac_server_config &c = sv->cfg;
    if (hipStreamCreateWithFlags(&s.s, hipStreamNonBlocking) != hipSuccess) return PFAC_EHIP;
    if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) return PFAC_EHIP;
    if (hipMalloc(&s.d_bytes, c.max_batch_bytes) != hipSuccess) return PFAC_ENOMEM;
    if (hipMalloc(&s.d_offs, ((uint64_t)c.max_batch_packets + 1) * 8) != hipSuccess) return PFAC_ENOMEM;
    if (hipMalloc(&s.d_sizes, 16) != hipSuccess) return PFAC_ENOMEM;
    if (hipMalloc(&s.d_keys, c.key_capacity * 8) != hipSuccess) return PFAC_ENOMEM;
    if (hipMalloc(&s.d_count, 8) != hipSuccess) return PFAC_ENOMEM;
    if (hipHostMalloc(&s.h_bytes, c.max_batch_bytes, hipHostMallocDefault) != hipSuccess) return PFAC_ENOMEM;
    if (hipHostMalloc(&s.h_offs, ((uint64_t)c.max_batch_packets + 1) * 8, hipHostMallocDefault) != hipSuccess)
        return PFAC_ENOMEM;
    if (hipHostMalloc(&s.h_sizes, 16, hipHostMallocDefault) != hipSuccess) return PFAC_ENOMEM;
    if (hipHostMalloc(&s.h_keys, c.key_capacity * 8, hipHostMallocDefault) != hipSuccess) return PFAC_ENOMEM;
    if (hipHostMalloc(&s.h_count, 8, hipHostMallocDefault) != hipSuccess) return PFAC_ENOMEM;
    s.cap = c.key_capacity;
    if (c.flags & PFAC_SERVER_EAGER)  // scratch for a full batch now, so launches never allocate
        return pfac::reserve_stream(sv->a, s.s, c.max_batch_bytes);
    return pfac_graph_create(sv->a, s.d_bytes, s.d_offs, c.max_batch_bytes, c.max_batch_packets, s.d_keys, s.cap,
                             s.d_count, s.d_sizes, s.s, &s.g);
}

// Device bytes one slot holds: batch buffers, keys, and the scan's per-span scratch.
uint64_t slot_device_bytes(const pfac_server_config &c, uint32_t span_log2) {
    // the scan's scratch is sized as the runtime sizes it: at least 1,024 spans, else
    // the spans of a full batch plus a quarter
    const uint64_t ns = (c.max_batch_bytes + (1ull << span_log2) - 1) >> span_log2;
    const uint64_t spans = ns < 1024 ? 1024 : ns + ns / 4;
    const uint64_t scratch = spans * (8 + 4 + 4 + (8ull << pfac::rec_cap_log2(span_log2))) +
                             spans / pfac::kBlockSpans * 8 + 16 + 1024 * 16;
    return c.max_batch_bytes + ((uint64_t)c.max_batch_packets + 1) * 8 + 16 + c.key_capacity * 8 + 8 + scratch;
}

// Take waiting requests (FIFO) for the slot, as many as fit one batch. Caller holds mu.
void take_requests(pfac_server *sv, Slot &s) {
    const pfac_server_config &c = sv->cfg;
    s.reqs.clear();
    uint64_t nb = 0;
    uint32_t np = 0;
    while (!sv->pending.empty()) {
        Request *r = sv->pending.front();
        if (!s.reqs.empty() && (nb + r->bytes.size() > c.max_batch_bytes || np + r->n_pkts > c.max_batch_packets))
            break;
        sv->pending.pop_front();
        sv->pending_bytes -= r->bytes.size();
        s.reqs.push_back(r);
        nb += r->bytes.size();
        np += r->n_pkts;
    }
}

// Stage the slot's requests as one CSR batch and launch its scan (a replay of the slot's
// graph, or an eager launch pair). Called without mu.
int launch_slot(pfac_server *sv, Slot &s) {
    s.byte0.clear();
    uint64_t nb = 0;
    uint32_t np = 0;
    for (Request *r : s.reqs) {
        s.byte0.push_back(nb);
        if (!r->bytes.empty()) memcpy(s.h_bytes + nb, r->bytes.data(), r->bytes.size());
        for (uint32_t i = 0; i < r->n_pkts; i++) s.h_offs[np + i] = nb + r->offs[i];
        nb += r->bytes.size();
        np += r->n_pkts;
    }
    s.byte0.push_back(nb);
    s.h_offs[np] = nb;
    s.h_sizes[0] = nb;
    s.h_sizes[1] = np;
    s.launch_ns = now_ns();
    if (nb && hipMemcpyAsync(s.d_bytes, s.h_bytes, nb, hipMemcpyHostToDevice, s.s) != hipSuccess) return PFAC_EHIP;
    if (hipMemcpyAsync(s.d_offs, s.h_offs, ((uint64_t)np + 1) * 8, hipMemcpyHostToDevice, s.s) != hipSuccess)
        return PFAC_EHIP;
    int rc;
    if (s.g) {
        if (hipMemcpyAsync(s.d_sizes, s.h_sizes, 16, hipMemcpyHostToDevice, s.s) != hipSuccess) return PFAC_EHIP;
        rc = pfac_graph_launch(s.g, s.s);
    } else {
        rc = pfac_scan_batch_async(sv->a, s.d_bytes, s.d_offs, np, nb, s.d_keys, s.cap, s.d_count, s.s);
    }
    if (rc) return rc;
    if (hipMemcpyAsync(s.h_count, s.d_count, 8, hipMemcpyDeviceToHost, s.s) != hipSuccess) return PFAC_EHIP;
    if (hipEventRecord(s.done, s.s) != hipSuccess) return PFAC_EHIP;
    return PFAC_OK;
}

// Keys of a finished slot, split into per-request results. Called without mu.
int finish_slot(pfac_server *sv, Slot &s, std::vector<pfac_result> &out) {
    uint64_t cnt = *s.h_count;
    if (cnt == ~0ull) return PFAC_ETIMEOUT;
    const uint64_t *keys = s.h_keys;
    std::vector<uint64_t> big;
    if (cnt > s.cap) {
        // more matches than the slot holds: scan the batch again into a buffer that fits
        uint64_t *d = nullptr;
        if (hipMalloc(&d, cnt * 8) != hipSuccess) return PFAC_ENOMEM;
        uint64_t c2 = 0;
        int rc = pfac_scan_batch(sv->a, s.d_bytes, s.d_offs, (uint32_t)s.h_sizes[1], s.h_sizes[0], d, cnt, &c2, s.s);
        if (!rc && c2 != cnt) rc = PFAC_EINTERNAL;
        if (!rc) {
            big.resize(cnt);
            if (hipMemcpy(big.data(), d, cnt * 8, hipMemcpyDeviceToHost) != hipSuccess) rc = PFAC_EHIP;
        }
        hipFree(d);
        if (rc) return rc;
        keys = big.data();
    } else if (cnt) {
        if (hipMemcpyAsync(s.h_keys, s.d_keys, cnt * 8, hipMemcpyDeviceToHost, s.s) != hipSuccess) return PFAC_EHIP;
        if (hipStreamSynchronize(s.s) != hipSuccess) return PFAC_EHIP;
    }
    const uint64_t t_done = now_ns();
    uint64_t k = 0;
    for (size_t i = 0; i < s.reqs.size(); i++) {
        Request *r = s.reqs[i];
        const uint64_t lo = s.byte0[i], hi = s.byte0[i + 1];
        const uint64_t k0 = k;
        while (k < cnt && (keys[k] >> 32) < hi) k++;
        pfac_result res{};
        res.ticket = r->ticket;
        res.status = PFAC_OK;
        res.n_pkts = r->n_pkts;
        res.n_bytes = r->bytes.size();
        res.n_matches = k - k0;
        res.arrival_ns = r->arrival_ns;
        res.launch_ns = s.launch_ns;
        res.done_ns = t_done;
        if (res.n_matches) {
            res.keys = (uint64_t *)malloc(res.n_matches * 8);
            if (!res.keys) return PFAC_ENOMEM;
            for (uint64_t x = 0; x < res.n_matches; x++) res.keys[x] = keys[k0 + x] - (lo << 32);
        }
        out.push_back(res);
    }
    return PFAC_OK;
}

// Results of a finished batch (or the failure of a batch) to the result queue and the
// statistics. Caller holds mu.
void publish(pfac_server *sv, Slot &s, int rc, std::vector<pfac_result> &fresh) {
    if (rc && !sv->fatal) sv->fatal = rc;
    for (size_t i = 0; i < s.reqs.size(); i++) {
        Request *r = s.reqs[i];
        if (rc) {
            pfac_result e{};
            e.ticket = r->ticket;
            e.status = rc;
            e.n_pkts = r->n_pkts;
            e.n_bytes = r->bytes.size();
            e.arrival_ns = r->arrival_ns;
            e.launch_ns = s.launch_ns;
            e.done_ns = now_ns();
            sv->results.push_back(e);
        }
        delete r;
    }
    for (pfac_result &res : fresh) {
        if (rc) {
            free(res.keys);
            continue;
        }
        sv->lat.push_back({res.done_ns > res.arrival_ns ? res.done_ns - res.arrival_ns : 0, res.n_pkts});
        sv->st_requests++;
        sv->st_packets += res.n_pkts;
        sv->st_bytes += res.n_bytes;
        sv->st_matches += res.n_matches;
        if (!sv->st_first_arrival || res.arrival_ns < sv->st_first_arrival) sv->st_first_arrival = res.arrival_ns;
        sv->st_last_done = std::max(sv->st_last_done, res.done_ns);
        sv->results.push_back(res);
    }
    if (s.launch_ns) sv->st_busy_slot_ns += now_ns() - s.launch_ns;
    s.reqs.clear();
    if (sv->fatal) {
        // fail whatever still waits
        while (!sv->pending.empty()) {
            Request *r = sv->pending.front();
            sv->pending.pop_front();
            pfac_result e{};
            e.ticket = r->ticket;
            e.status = sv->fatal;
            e.n_pkts = r->n_pkts;
            e.n_bytes = r->bytes.size();
            e.arrival_ns = r->arrival_ns;
            e.done_ns = now_ns();
            sv->results.push_back(e);
            delete r;
        }
        sv->pending_bytes = 0;
        sv->cv_work.notify_all();
    }
    sv->cv_done.notify_all();
}

// One host thread per slot: whenever the slot is free and requests wait, it takes every
// waiting request that fits one batch (continuous batching), stages and launches it,
// waits for its completion event and publishes the results. Staging, launching and
// finishing of different slots run in parallel, so no slot waits for another one's
// host work.
void slot_main(pfac_server *sv, size_t idx) {
    (void)hipSetDevice(sv->device);
    Slot &s = sv->slots[idx];
    std::vector<pfac_result> fresh;
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        sv->cv_work.wait(lk, [&] { return sv->stop || sv->fatal || !sv->pending.empty(); });
        if (sv->fatal || sv->pending.empty()) {
            if (sv->stop || sv->fatal) break;
            continue;
        }
        take_requests(sv, s);
        s.busy = true;
        sv->st_batches++;
        lk.unlock();
        fresh.clear();
        s.launch_ns = 0;
        int rc = launch_slot(sv, s);
        if (!rc && hipEventSynchronize(s.done) != hipSuccess) rc = PFAC_EHIP;
        if (!rc) rc = finish_slot(sv, s, fresh);
        lk.lock();
        s.busy = false;
        publish(sv, s, rc, fresh);
    }
}

}  // namespace

extern "C" int pfac_server_create(pfac_automaton *a, const pfac_server_config *cfg, pfac_server **out) {
    if (!out) return PFAC_EINVAL;
    *out = nullptr;
    if (!a || a->n_pats == 0) return PFAC_EINVAL;
    pfac_server_config c = cfg ? *cfg : pfac_server_config{};
    if (!c.slots) c.slots = 4;
    if (!c.max_batch_bytes) c.max_batch_bytes = 8ull << 20;
    if (!c.max_batch_packets) c.max_batch_packets = 16384;
    if (!c.key_capacity) c.key_capacity = 1u << 16;
    if (!c.max_pending_bytes) c.max_pending_bytes = 1ull << 30;
    if (c.max_batch_bytes >= (1ull << 32) || c.slots > 64) return PFAC_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PFAC_ENODEVICE;
    int rc = pfac_upload(a, dev);
    if (rc) return rc;
    // admission by device memory: as many slots as the budget holds
    const uint32_t span_log2 = a->span_log2 ? a->span_log2 : pfac::auto_span_log2(c.max_batch_bytes, 256ull * pfac::kWaves);
    const uint64_t per_slot = slot_device_bytes(c, span_log2);
    uint64_t budget = c.device_memory_budget;
    if (!budget) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return PFAC_EHIP;
        budget = free_b / 4;
    }
    const uint64_t fit = budget / per_slot;
    if (fit == 0) return PFAC_ENOMEM;
    c.slots = (uint32_t)std::min<uint64_t>(c.slots, fit);
    pfac_server *sv = new (std::nothrow) pfac_server();
    if (!sv) return PFAC_ENOMEM;
    sv->a = a;
    sv->device = dev;
    sv->cfg = c;
    sv->slots.resize(c.slots);
    for (Slot &s : sv->slots)
        if (!rc) rc = alloc_slot(sv, s);
    if (!rc) {
        try {
            for (size_t i = 0; i < sv->slots.size(); i++) sv->workers.emplace_back(slot_main, sv, i);
        } catch (...) {
            rc = PFAC_ENOMEM;
        }
    }
    if (rc) {
        {
            std::lock_guard<std::mutex> g(sv->mu);
            sv->stop = true;
        }
        sv->cv_work.notify_all();
        for (std::thread &t : sv->workers)
            if (t.joinable()) t.join();
        for (Slot &s : sv->slots) free_slot(sv->a, s);
        delete sv;
        return rc;
    }
    *out = sv;
    return PFAC_OK;
}

extern "C" int pfac_server_config_get(const pfac_server *sv, pfac_server_config *out) {
    if (!sv || !out) return PFAC_EINVAL;
    *out = sv->cfg;
    return PFAC_OK;
}

extern "C" int pfac_server_submit(pfac_server *sv, const uint8_t *h_bytes, const uint64_t *h_offsets,
                                  uint32_t n_pkts, uint64_t arrival_ns, uint64_t *ticket) {
    if (!sv || !ticket || !h_offsets) return PFAC_EINVAL;
    const uint64_t nb = h_offsets[n_pkts];
    if (h_offsets[0] != 0 || (nb > 0 && !h_bytes)) return PFAC_EINVAL;
    for (uint32_t i = 0; i < n_pkts; i++)
        if (h_offsets[i + 1] < h_offsets[i]) return PFAC_EINVAL;
    if (nb > sv->cfg.max_batch_bytes || n_pkts > sv->cfg.max_batch_packets) return PFAC_ETOO_LARGE;
    Request *r = new (std::nothrow) Request();
    if (!r) return PFAC_ENOMEM;
    try {
        r->bytes.assign(h_bytes, h_bytes + nb);
        r->offs.assign(h_offsets, h_offsets + n_pkts + 1);
    } catch (const std::bad_alloc &) {
        delete r;
        return PFAC_ENOMEM;
    }
    r->n_pkts = n_pkts;
    r->arrival_ns = arrival_ns ? arrival_ns : now_ns();
    {
        std::lock_guard<std::mutex> g(sv->mu);
        if (sv->fatal || sv->stop) {
            const int rc = sv->fatal ? sv->fatal : PFAC_EINVAL;
            delete r;
            return rc;
        }
        if (sv->pending_bytes + nb > sv->cfg.max_pending_bytes) {
            sv->st_rejected++;
            delete r;
            return PFAC_EBUSY;
        }
        r->ticket = sv->next_ticket++;
        sv->pending.push_back(r);
        sv->pending_bytes += nb;
        *ticket = r->ticket;
    }
    sv->cv_work.notify_one();
    return PFAC_OK;
}

extern "C" int pfac_server_poll(pfac_server *sv, pfac_result *res, uint32_t max_results, uint32_t *n_out,
                                uint32_t timeout_us) {
    if (!sv || !n_out || (max_results > 0 && !res)) return PFAC_EINVAL;
    *n_out = 0;
    std::unique_lock<std::mutex> lk(sv->mu);
    if (sv->results.empty() && timeout_us)
        sv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return !sv->results.empty(); });
    uint32_t n = 0;
    while (n < max_results && !sv->results.empty()) {
        res[n++] = sv->results.front();
        sv->results.pop_front();
    }
    *n_out = n;
    return PFAC_OK;
}

extern "C" void pfac_result_free(pfac_result *r) {
    if (!r) return;
    free(r->keys);
    r->keys = nullptr;
    r->n_matches = 0;
}

extern "C" int pfac_server_stats(pfac_server *sv, pfac_server_stats_t *st, int reset) {
    if (!sv || !st) return PFAC_EINVAL;
    memset(st, 0, sizeof(*st));
    std::lock_guard<std::mutex> g(sv->mu);
    st->requests = sv->st_requests;
    st->packets = sv->st_packets;
    st->bytes = sv->st_bytes;
    st->matches = sv->st_matches;
    st->batches = sv->st_batches;
    st->rejected = sv->st_rejected;
    st->pending_requests = sv->pending.size();
    st->slots = (uint32_t)sv->slots.size();
    if (sv->st_last_done > sv->st_first_arrival)
        st->bytes_per_s = (double)sv->st_bytes * 1e9 / (double)(sv->st_last_done - sv->st_first_arrival);
    if (sv->st_batches) st->mean_batch_bytes = (double)sv->st_bytes / (double)sv->st_batches;
    if (!sv->lat.empty()) {
        // per-packet latency: each request's latency counts once per packet
        std::vector<LatSample> v = sv->lat;
        std::sort(v.begin(), v.end(), [](const LatSample &x, const LatSample &y) { return x.ns < y.ns; });
        uint64_t total = 0;
        for (const LatSample &x : v) total += x.pkts;
        auto pct = [&](double p) -> uint64_t {
            const double want = p * (double)total;
            uint64_t run = 0;
            for (const LatSample &x : v) {
                run += x.pkts;
                if ((double)run >= want && x.pkts) return x.ns;
            }
            return v.back().ns;
        };
        if (total) {
            st->p50_ns = pct(0.50);
            st->p99_ns = pct(0.99);
            st->max_ns = v.back().ns;
        }
    }
    if (reset) {
        sv->lat.clear();
        sv->st_requests = sv->st_packets = sv->st_bytes = sv->st_matches = sv->st_batches = sv->st_rejected = 0;
        sv->st_first_arrival = sv->st_last_done = sv->st_busy_slot_ns = 0;
    }
    return PFAC_OK;
}

extern "C" void pfac_server_destroy(pfac_server *sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    for (std::thread &t : sv->workers)
        if (t.joinable()) t.join();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(sv->device);
    for (Slot &s : sv->slots) {
        if (s.s) (void)hipStreamSynchronize(s.s);
        free_slot(sv->a, s);
    }
    (void)hipSetDevice(prev);
    for (pfac_result &r : sv->results) free(r.keys);
    delete sv;
}
