// Shapes and scratch of the tiled scan kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pfac_impl.h"

namespace pfac {

// Build-time shape of the count kernel (the defaults are the measured best on MI355X):
// threads per workgroup, log2 of the prefilter's bits, survivor queue entries per wave.
#ifndef PFAC_SCAN_THREADS
#define PFAC_SCAN_THREADS 1024
#endif
#ifndef PFAC_FILTER_LOG2
#define PFAC_FILTER_LOG2 19
#endif
#ifndef PFAC_FILTER2_LOG2
#define PFAC_FILTER2_LOG2 18
#endif
#ifndef PFAC_QCAP
#define PFAC_QCAP 512
#endif
#ifndef PFAC_PREFETCH
#define PFAC_PREFETCH 2
#endif
#ifndef PFAC_SCAN_MIN_WG
#define PFAC_SCAN_MIN_WG 1
#endif

constexpr uint32_t kThreads = PFAC_SCAN_THREADS;  // workgroup: waves sharing one LDS image
constexpr uint32_t kWaves = kThreads / 64;
constexpr uint32_t kSpanLog2 = 14;   // default bytes per work unit (a wave's span): 16 KiB
constexpr uint32_t kMinSpanLog2 = 11; // a span holds at least one wave step
constexpr uint32_t kMaxSpanLog2 = 16; // span-local starts are 16-bit
constexpr uint32_t kPrefetch = PFAC_PREFETCH;  // wave steps of 2 KiB whose loads are in flight (>= 2)
static_assert(PFAC_PREFETCH >= 2, "the next step's first word comes from the prefetch");

// Positions per thread: the bytes (starts) a lane takes per wave step, 32 (two 16-byte
// loads; the default) or 16 (one load). A tuning choice for every prefilter form but the
// sampled one, whose candidate checks read a lane's 32 bytes. The bytes a wave keeps in
// flight are the same either way (kPrefetch x 2 KiB).
constexpr uint32_t kLaneBytes = 32;
template <uint32_t LB>
struct Lanes {
    static_assert(LB == 16 || LB == 32, "a lane's starts fit one 32-bit mask");
    static constexpr uint32_t step = 64 * LB;                    // bytes a wave streams per step
    static constexpr uint32_t prefetch = kPrefetch * (32 / LB);  // steps whose loads are in flight
};
constexpr uint32_t kHCapMinLog2 = 8; // match records kept per span: span / 64, at least 256
constexpr uint32_t kBlockSpans = 64; // spans per placement block (one per lane of a wave)
constexpr uint32_t kRecMulti = 0x8000;  // record flag: several terminals (see SpanOut)
constexpr uint32_t kFastRecs = 8;    // a span with at most this many records is written by one lane
constexpr uint32_t kDirectMaxSpans = 16384;  // placement without look-back up to this many spans
constexpr uint32_t kRecRounds = 4;   // 64-record rounds whose loads a placement wave issues together
#ifndef PFAC_PLACE_THREADS
#define PFAC_PLACE_THREADS 1024
#endif
constexpr uint32_t kPlaceThreads = PFAC_PLACE_THREADS;  // placement workgroup (its waves share a block's spans)
constexpr uint32_t kPlaceWaves = kPlaceThreads / 64;
#ifndef PFAC_PLACE_SUM_LOADS
#define PFAC_PLACE_SUM_LOADS (4096 / PFAC_PLACE_THREADS)
#endif
constexpr uint32_t kSumLoads = PFAC_PLACE_SUM_LOADS;  // loads in flight per thread in a block's span-count sum

// LDS of the scan kernel (32-bit words), one of two layouts per kernel instance (a
// probe's masked hash plus its part's compile-time offset is its byte address; every
// filter part starts below 64 KiB, so that offset folds into the LDS instruction):
//   general   [second-probe part: 2^18 bits][first-probe part: 2^19 bits][short bitmap]
//             [root bitmap][rank table][survivor queues, 512 entries a wave]
//             two-probe Bloom filter over k-gram keys, every start probed; the short
//             bitmap holds the D-grams of patterns shorter than k
//   sampled   [second-probe part: 2^16 bits][first-probe part: 2^17 bits][3-gram part: 2^19 bits]
//             [root bitmap][rank table][step staging, 576 words a wave]
//             [survivor queues, 512 entries a wave]
//   exact     [(D+E)-symbol bitmap: up to 2^20 bits][root bitmap][rank table]
//             [survivor queues, 512 entries a wave]
//             two-bit symbols: every start probed once in an exact bitmap of the trie's
//             first D+E levels, E = 1 or 2 (no hash, no false positive beyond the
//             truncation)
//             patterns of four or more bytes and k = 4: only every second start is
//             probed, with the 3-gram there against the 3-grams at offsets 0 and 1 of
//             every pattern; the two starts it stands for are then checked against the
//             two-probe Bloom filter over 4-grams, by the lane that holds their bytes.
// The builder's image holds the filter words (copied to offset 0), then the root bitmap,
// the rank table and the short bitmap (copied to their places).
constexpr uint32_t kMaxFilterLog2 = PFAC_FILTER_LOG2;    // general first-probe part: 2^19 bits
constexpr uint32_t kFilter2Log2 = PFAC_FILTER2_LOG2;     // general second-probe part: 2^18 bits
constexpr uint32_t kFilterWordsMax = 1u << (kMaxFilterLog2 - 5);
constexpr uint32_t kFilter2Words = 1u << (kFilter2Log2 - 5);
constexpr uint32_t kLdsF1 = kFilter2Words;                // word offset of the first-probe part
constexpr uint32_t kAmask1 = (kFilterWordsMax - 1u) << 2; // byte-offset masks of the parts
constexpr uint32_t kAmask2 = (kFilter2Words - 1u) << 2;
constexpr uint32_t kGeneralWords = kFilter2Words + kFilterWordsMax;  // general filter words
#ifndef PFAC_S3_LOG2
#define PFAC_S3_LOG2 14
#endif
constexpr uint32_t kS3Words = 1u << PFAC_S3_LOG2;         // sampled: 3-gram part (64 KiB)
constexpr uint32_t kS2Words = 1u << 11;                   // sampled: second-probe part (8 KiB)
constexpr uint32_t kS1Words = 1u << 12;                   // sampled: first-probe part (16 KiB)
constexpr uint32_t kLdsS2 = 0, kLdsS1 = kS2Words, kLdsS3 = kS2Words + kS1Words;
static_assert(kLdsS3 * 4 < 65536, "the 3-gram part's offset fits the LDS instruction");
constexpr uint32_t kSampledWords = kLdsS3 + kS3Words;     // sampled filter words
static_assert(kSampledWords % 4 == 0 && kGeneralWords % 4 == 0, "filters copy in 16-byte units");
constexpr uint32_t kFilterMul3 = 0x9E3779u;  // 24-bit multiplier of the 3-gram hash
constexpr uint32_t kRootWordsMax = 1u << 11;    // 8 KiB: root keys up to 16 bits
constexpr uint32_t kRankWordsMax = 1u << 10;    // 4 KiB: one u16 per root word

// LDS layouts (see above), one per prefilter form.
enum LdsForm : int { kFormGeneral = 0, kFormSampled = 1, kFormExact = 2 };
template <int FORM>
struct Lds;
template <>
struct Lds<kFormGeneral> {
    static constexpr uint32_t shrt = kGeneralWords;
    static constexpr uint32_t root = shrt + kRootWordsMax;
    static constexpr uint32_t rank = root + kRootWordsMax;
    static constexpr uint32_t qcap = PFAC_QCAP;
    static constexpr uint32_t queues = rank + kRankWordsMax;
    static constexpr uint32_t words = queues + kWaves * qcap / 2;
};
// The sampled layout also stages each lane's bytes of the current step (its 32 bytes and
// the 4 after them: 9 words at a stride of 9 words per lane, so the 32 lanes of a bank
// group read distinct banks) for the candidate checks.
constexpr uint32_t kStageLaneWords = 9;
constexpr uint32_t kStageWords = 64 * kStageLaneWords;
template <>
struct Lds<kFormSampled> {
    static constexpr uint32_t root = kSampledWords;
    static constexpr uint32_t rank = root + kRootWordsMax;
    static constexpr uint32_t shrt = 0;  // none: no pattern is shorter than k
    static constexpr uint32_t qcap = PFAC_QCAP;
    static constexpr uint32_t stage = rank + kRankWordsMax;
    static constexpr uint32_t queues = stage + kWaves * kStageWords;
    static constexpr uint32_t words = queues + kWaves * qcap / 2;
};
// Exact form (two-bit symbols): the trie truncated E = 1 or 2 levels below the root image,
// as a direct bitmap over (D+E)-symbol keys: a key's bit is set when some pattern begins
// with it, or when a prefix of it is a whole pattern (every extension of a pattern shorter
// than D + E is set). 4^(D+E) bits, at most 2^20 (128 KiB, D = 8, E = 2).
constexpr uint32_t kExactWordsMax = 1u << 15;
template <>
struct Lds<kFormExact> {
    static constexpr uint32_t root = kExactWordsMax;
    static constexpr uint32_t rank = root + kRootWordsMax;
    static constexpr uint32_t shrt = 0;  // none
    static constexpr uint32_t qcap = PFAC_QCAP;
    static constexpr uint32_t queues = rank + kRankWordsMax;
    static constexpr uint32_t words = queues + kWaves * qcap / 2;
};
static_assert(Lds<kFormGeneral>::qcap >= 128 && Lds<kFormGeneral>::qcap % 8 == 0, "a queue holds two walk batches");
static_assert(Lds<kFormGeneral>::words * 4 <= 160 * 1024 && Lds<kFormSampled>::words * 4 <= 160 * 1024 &&
                  Lds<kFormExact>::words * 4 <= 160 * 1024,
              "LDS of one CU");

// Per-span results of the count kernel (device memory, owned by a workspace).
//   cnt[s]   matches in span s          nh[s]   records stored for span s
//   ovf[s]   span-local start of the first matching start without a record, or ~0
//   rec[(s << rec_log2) + i]   record i of a matching start, bits 0..15 = span-local start,
//                        bits 16..31 = F, bits 32..63 = H:
//                        F in 1 .. kRecMulti-1: one terminal with F ids; H = the id itself
//                          when F == 1, else the index of the ids in out_ids;
//                        F = kRecMulti | d: several terminals, the first one node H at depth
//                          d: the placement walks again from there;
//                        F = 0: walk again from the root (ids or depths past the fields)
struct SpanOut {
    uint64_t *cnt;
    uint32_t *nh;
    uint32_t *ovf;
    uint64_t *rec;
    uint32_t rec_log2;  // log2 of the records per span (0: rec_cap_log2 of the span, set per launch)
};

// Span length chosen when the tuning leaves it open: the longest power of two (4 to
// 64 KiB) that still gives every resident wave (`waves`) a span of an n-byte text.
inline uint32_t auto_span_log2(uint64_t n, uint64_t waves) {
    uint32_t s = kMaxSpanLog2;
    while (s > 12 && (n >> s) < waves) s--;
    return s;
}

// log2 of the record capacity of a span of 2^span_log2 bytes.
__host__ __device__ inline uint32_t rec_cap_log2(uint32_t span_log2) {
    return span_log2 - 6 > kHCapMinLog2 ? span_log2 - 6 : kHCapMinLog2;
}

// Decoupled look-back state of the placement kernel (device memory, in a workspace).
//   word[b]   one 64-bit word per block: epoch (bits 44..63) | flag (42..43) | value (0..41)
//             flag 1: value = matches in block b; flag 2: value = matches in blocks 0..b.
//             Flag and value share one word, so publishing and reading need only relaxed
//             device-scope atomics: no fence, no L2 write-back or invalidate per tile.
//   ctrl[0]   block ticket   ctrl[1] workgroups done   ctrl[2] epoch (1 .. 2^20 - 1)
//   ctrl[3]   error bits (1: a bounded wait expired, 2: count past 2^42)
// The last workgroup of a launch writes the count, resets the ticket and the done count
// and advances the epoch, so a later launch (or a replayed graph) needs no host-side
// reset; words of an older epoch never match. The host clears the words before the epoch
// could wrap (kEpochPeriod launches).
constexpr uint32_t kEpochBits = 20;
constexpr uint64_t kEpochPeriod = (1u << kEpochBits) - 2;
constexpr uint64_t kValueMask = (1ull << 42) - 1;
struct TileState {
    uint64_t *word;
    uint32_t *ctrl;
};

// End of the packet holding global position s of a packet batch (offsets: n_packets + 1
// ascending byte offsets), by binary search. A position at or past offsets[n_packets]
// (offsets that end before the batch's bytes do) gets offsets[n_packets]: every read
// stays inside the array, and a walk from there stops at once.
__host__ __device__ inline uint64_t packet_end(const uint64_t *__restrict__ offsets, uint32_t n_packets, uint64_t s) {
    uint32_t lo = 0, hi = n_packets;  // first i with offsets[i+1] > s
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (offsets[mid + 1] > s) hi = mid;
        else lo = mid + 1;
    }
    return offsets[lo < n_packets ? lo + 1 : n_packets];
}

// Count value that reports a device-side error (the host maps it to a status).
constexpr uint64_t kCountTimeout = ~0ull;
constexpr uint64_t kCountOverflow = ~0ull - 1;

// Count kernel then placement kernel on stream s. offsets: packet offsets (n_packets + 1)
// or null for one text. sizes: null, or device {n, n_packets} read at run time and
// bounded by the n / n_packets given here (graph replays). grid: workgroups of the
// count kernel (0 = as many as are resident at once). span_log2: log2 of the span length,
// kMinSpanLog2..kMaxSpanLog2 (else -1, nothing launched); the scratch in `so` must hold
// ceil(n / 2^span_log2) spans. lane_bytes: positions per thread and step, 16 or 32 (any
// other value: 32; the sampled form always takes 32).
int launch_tiled(const DevTable &t, const uint8_t *text, uint64_t n, const uint64_t *offsets, uint32_t n_packets,
                 uint64_t *keys, uint64_t cap, uint64_t *d_count, const SpanOut &so, const TileState &ts,
                 const uint64_t *sizes, uint32_t grid, uint32_t span_log2, uint32_t lane_bytes, hipStream_t s);
// The same for a compressed table (t.merged; launch_tiled dispatches to it).
int launch_tiled_merged(const DevTable &t, const uint8_t *text, uint64_t n, const uint64_t *offsets,
                        uint32_t n_packets, uint64_t *keys, uint64_t cap, uint64_t *d_count, const SpanOut &so,
                        const TileState &ts, const uint64_t *sizes, uint32_t grid, uint32_t span_log2,
                        uint32_t lane_bytes, hipStream_t s);

}  // namespace pfac
