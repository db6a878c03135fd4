/*
 * pfac.h -- C ABI of a failure-less Aho-Corasick matcher for AMD Instinct MI355X (gfx950).
 *
 * The method is the parallel failure-less Aho-Corasick of Section 2.3 (every text
 * position starts its own walk of a goto-only trie and stops at the first missing
 * transition) over the compressed storage model of Section 3.1 (a breadth-first node
 * array, each node a first-child offset plus a child bitmap, children found by the
 * popcount rule of Eq. 1).
 *
 * Result definition. For patterns p_0..p_{N-1} (non-empty byte strings over the symbols
 * 0..alphabet-1) and a text T of n bytes, the result is every pair (s, j) with
 * s + |p_j| <= n and T[s .. s+|p_j|) == p_j (the problem of Section 2.2). Each pair is
 * returned as the 64-bit key (s << 32) | j; keys are written in increasing order, so
 * they are sorted by start, then by pattern id. Duplicate patterns are all reported;
 * a pattern that is a prefix of another is reported wherever it occurs. A text byte
 * >= alphabet has no transition and so takes part in no match.
 *
 * Conventions.
 *  - Every function returns an int status: PFAC_OK (0) or a negative PFAC_E* code.
 *    No function throws or aborts across this boundary.
 *  - "d_" arguments are device pointers (HBM of the current HIP device, e.g. a torch
 *    tensor's data_ptr()); "h_" arguments are host pointers. The library never frees
 *    memory it did not allocate.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream). Device work
 *    is enqueued on it in order.
 *  - An automaton is immutable after pfac_build. Scans on different streams or threads
 *    may share it; destroying it while work that uses it is still queued is undefined
 *    (synchronize first).
 */
#ifndef PFAC_H
#define PFAC_H

#include <stddef.h>
#include <stdint.h>

#define PFAC_API __attribute__((visibility("default")))

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status codes */
#define PFAC_OK 0
#define PFAC_EINVAL (-1)         /* null pointer, size or option out of range          */
#define PFAC_EEMPTY_PATTERN (-2) /* a pattern of length 0 (it would match everywhere)   */
#define PFAC_ESYMBOL (-3)        /* a pattern byte >= alphabet                          */
#define PFAC_ETOO_LARGE (-4)     /* node or id count past 32-bit offsets, or n >= 2^32  */
#define PFAC_ENOMEM (-5)         /* host or device allocation failed                    */
#define PFAC_EHIP (-6)           /* a HIP runtime call failed                           */
#define PFAC_ECAPACITY (-7)      /* more matches than the output holds (see scans)      */
#define PFAC_ENODEVICE (-8)      /* no usable gfx950 device                             */
#define PFAC_EFORMAT (-9)        /* serialized automaton is malformed or truncated      */
#define PFAC_ETIMEOUT (-10)      /* a device-side bounded wait expired (internal error) */
#define PFAC_EINTERNAL (-11)     /* an internal consistency check failed               */
#define PFAC_EBUSY (-12)         /* a server's waiting queue is full; submit again later */

/* Human-readable name of a status code (static storage, never NULL). */
PFAC_API const char *pfac_strerror(int status);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
PFAC_API int pfac_version(void);

typedef struct pfac_automaton pfac_automaton;

/* ------------------------------------------------------------------- building
 * pfac_build -- build the compressed table (Section 3.1): patterns are sorted
 * bytewise, inserted breadth-first, and every node is stored as a first-child offset
 * plus a child bitmap; the child on symbol c is offset + popcount(bits below c) (Eq. 1).
 *
 *   pats[i], lens[i]  pattern i (pattern id = i); the bytes are copied, the caller may
 *                     free them on return. n_pats may be 0 (every scan then returns no
 *                     match).
 *   alphabet          1..256; symbols are the raw byte values 0..alphabet-1.
 *   out               receives the automaton; free with pfac_destroy.
 *
 * Errors: PFAC_EINVAL (out NULL, pats/lens NULL with n_pats > 0, alphabet outside
 * 1..256), PFAC_EEMPTY_PATTERN, PFAC_ESYMBOL, PFAC_ETOO_LARGE (more than 2^31 - 1
 * nodes or a pattern longer than 2^24 bytes), PFAC_ENOMEM. On error *out is NULL.
 * Host only: needs no GPU. */
PFAC_API int pfac_build(const uint8_t *const *pats, const uint64_t *lens, uint32_t n_pats,
               uint32_t alphabet, pfac_automaton **out);

/* Same as pfac_build with the patterns packed back to back: pattern i is
 * bytes[offsets[i] .. offsets[i+1]), offsets has n_pats + 1 entries. */
PFAC_API int pfac_build_csr(const uint8_t *bytes, const uint64_t *offsets, uint32_t n_pats,
                   uint32_t alphabet, pfac_automaton **out);

/* pfac_build_ex -- pfac_build_csr with options. merge_levels selects the table the
 * scans walk:
 *   0        the trie of Section 3.1 (what pfac_build makes);
 *   L >= 1   the compressed trie of Section 3.2: nodes whose height (longest path down to
 *            a leaf) is below L are merged when everything below them is the same (the
 *            same suffixes complete a pattern). L = 1 merges only the final nodes into one
 *            global final node (step 1, Eq. 2); L = 3 merges the last three levels (step
 *            2); L = 255 merges everything mergeable. Under Eq. 1 a node's children stay
 *            consecutive, so the table stores shared blocks of children once; the
 *            breadth-first top levels that the LDS root image folds are never shared.
 * Matches are the same for every L (pattern ids are recovered from the rank of the
 * spelled string among the distinct patterns, see pfac_export_records). opt may be NULL
 * (all options 0). Errors as pfac_build, plus PFAC_EINVAL for merge_levels > 255. */
typedef struct {
    uint32_t merge_levels;
    uint32_t reserved[7];
} pfac_build_options;

PFAC_API int pfac_build_ex(const uint8_t *bytes, const uint64_t *offsets, uint32_t n_pats, uint32_t alphabet,
                           const pfac_build_options *opt, pfac_automaton **out);

/* Free the automaton and its device copies. NULL is a no-op. */
PFAC_API void pfac_destroy(pfac_automaton *a);

/* Sizes and shape of a built automaton. */
typedef struct {
    uint32_t alphabet;
    uint32_t n_patterns;
    uint32_t n_nodes;            /* 1 + number of distinct non-empty pattern prefixes  */
    uint32_t n_terminal_nodes;   /* nodes where at least one pattern ends               */
    uint32_t min_len, max_len;   /* pattern lengths (0 when n_patterns == 0)            */
    uint32_t depth;              /* trie depth (= max_len)                              */
    uint32_t node_layout;        /* 0: 8-byte node (alphabet <= 32), 1: wide node      */
    uint64_t paper_table_bytes;  /* n_nodes * (4 + ceil(alphabet / 8)), Section 3.1    */
    uint64_t device_table_bytes; /* everything a device copy holds in HBM: node arrays,
                                    pattern ids (and rank words), path tails with the
                                    first 16 bytes of each path, pattern bytes, LDS
                                    image source                                        */
    uint32_t root_depth;         /* levels folded into the LDS-resident root image     */
    uint32_t filter_k;           /* symbols in the LDS prefix filter key (0 = none)    */
    uint32_t filter_log2_bits;   /* log2 of the filter's bit count (0 = none)          */
    uint32_t lds_image_bytes;    /* root image + filter, copied to LDS per workgroup   */
    uint32_t merge_levels;       /* as built (pfac_build_ex)                           */
    uint32_t reduced_nodes;      /* nodes after the compression of Section 3.2
                                    (= n_nodes when merge_levels is 0)                  */
    uint32_t table_records;      /* records of the walked table (= n_nodes uncompressed) */
    uint32_t shared_base;        /* first record of a shared block                     */
    uint64_t reduced_paper_bytes;/* reduced_nodes * (4 + ceil(alphabet / 8))            */
    uint64_t node_array_bytes;   /* the walked table's node words in HBM               */
    uint64_t stream_scratch;     /* per-stream scratch areas held on all devices (one
                                    per stream a scan ran on; freed with the automaton,
                                    or when the library's own streams are destroyed)    */
    uint32_t device_records;     /* node words of the device table: the plain table
                                    stores a unary path below the root image's levels as
                                    one tail record, not as nodes                       */
    uint32_t device_tails;       /* tail records of the plain table (0 when compressed) */
} pfac_table_info_t;

PFAC_API int pfac_table_info(const pfac_automaton *a, pfac_table_info_t *out);

/* Copy the table in the paper's own layout (Section 3.1): for node q,
 * offsets[q] = index of its first child (0 for a node without children) and
 * bitmaps[q * words + w] = bits 32w .. 32w+31 of its child bitmap (bit c = symbol c),
 * with words = ceil(alphabet / 32). Capacities are in elements; PFAC_EINVAL if either
 * is too small for n_nodes. */
PFAC_API int pfac_export_paper_table(const pfac_automaton *a, uint32_t *offsets, uint64_t offsets_cap,
                            uint32_t *bitmaps, uint64_t bitmaps_cap);

/* Pattern ids ending at each node as CSR: ids of node q are ids[first[q] .. first[q+1]),
 * ascending. first has n_nodes + 1 entries, ids n_patterns. */
PFAC_API int pfac_export_outputs(const pfac_automaton *a, uint32_t *first, uint64_t first_cap,
                        uint32_t *ids, uint64_t ids_cap);

/* The table the scans walk, one record per entry: first[x] = first child record (0 for
 * none), bitmaps[x * words + w] as in pfac_export_paper_table, term[x] = 1 when a pattern
 * ends there, rank[x] = its rank word. Without compression the records are the trie's
 * nodes and rank[x] is the number of distinct pattern strings that sort (bytewise,
 * shorter first) before the node's prefix. With compression, records from
 * info.shared_base on lie in shared blocks and rank[x] there counts the strings spelled
 * below the lower siblings in x's block; a walk remembers its last record u below
 * shared_base and adds term(q) + rank[y] for every step from q into a shared record y,
 * so that a terminal reached has rank rank[u] + that sum (its own rank word when below
 * shared_base). cap: entries of every array (>= table_records). */
PFAC_API int pfac_export_records(const pfac_automaton *a, uint32_t *first, uint32_t *bitmaps, uint8_t *term,
                                 uint32_t *rank, uint64_t cap);

/* Pattern ids of each distinct pattern string by rank: ids[first[r] .. first[r+1]),
 * ascending; first has (distinct strings + 1) entries, at most n_patterns + 1. */
PFAC_API int pfac_export_rank_ids(const pfac_automaton *a, uint32_t *first, uint64_t first_cap, uint32_t *ids,
                                  uint64_t ids_cap);

/* ------------------------------------------------------------------- saving
 * pfac_save -- serialize the automaton into buf (host memory, cap bytes): the table of
 * Section 3.1 (first-child offset and child bitmap of every node, breadth-first), the
 * pattern ids ending at each node, the patterns and the tuning in force, behind a
 * versioned header (magic, version, alphabet, node and pattern counts, longest and
 * shortest pattern, payload size, 64-bit FNV-1a checksum). *size always receives the
 * bytes needed; with buf NULL or cap too small nothing is written and the call returns
 * PFAC_ECAPACITY. Device copies are not saved. Errors: PFAC_EINVAL (a or size NULL),
 * PFAC_ECAPACITY. Host only.
 *
 * pfac_load -- rebuild an automaton from size bytes written by pfac_save. The blob is
 * checked (header, sizes, checksum) and so is the table itself: it must be the
 * breadth-first trie of the stored patterns (offsets of Section 3.1, every leaf ending a
 * pattern, each pattern's Eq. 1 path ending at the node that lists it), so a loaded
 * automaton equals the one pfac_build makes from the same patterns and scans only inside
 * its arrays. The buffer may be freed on return. Errors: PFAC_EINVAL (out or buf NULL),
 * PFAC_EFORMAT (truncated, corrupted or inconsistent blob; *out NULL), PFAC_ENOMEM.
 * Host only. */
PFAC_API int pfac_save(const pfac_automaton *a, uint8_t *buf, uint64_t cap, uint64_t *size);
PFAC_API int pfac_load(const uint8_t *buf, uint64_t size, pfac_automaton **out);

/* pfac_key_to_packet -- split n_keys batch keys (host memory, as written by the batch
 * scans: global byte offset << 32 | pattern id) into the packet holding each start,
 * the start within that packet and the pattern id, for packets given by h_offsets
 * (n_pkts + 1 entries, non-decreasing, as passed to pfac_scan_batch; a match lies inside
 * one packet, Section 2.2 applied per packet). Keys need not be sorted. Each output array
 * holds n_keys entries (host memory). Errors: PFAC_EINVAL (NULL arrays with n_keys > 0,
 * or a start outside [h_offsets[0], h_offsets[n_pkts])). Host only. */
PFAC_API int pfac_key_to_packet(const uint64_t *h_keys, uint64_t n_keys, const uint64_t *h_offsets,
                                uint32_t n_pkts, uint32_t *pkt, uint32_t *start, uint32_t *ids);

/* ------------------------------------------------------------------- device
 * Copy the table to device `device` (HIP ordinal). Done implicitly by the first scan
 * on a device; the copy stays resident until pfac_destroy. Errors: PFAC_ENODEVICE (no
 * such device, or not gfx950), PFAC_ENOMEM, PFAC_EHIP. */
PFAC_API int pfac_upload(pfac_automaton *a, int device);

/* ------------------------------------------------------------------- scanning
 * pfac_scan_async -- scan n bytes at d_text (device memory) and write the keys of all
 * matches, sorted, to d_keys (device memory); write the number of matches to *d_count
 * (device memory, one uint64). Only enqueues work on `stream`; results are valid once
 * the stream has completed. When the count exceeds cap, at most cap keys are written,
 * their content is unspecified, and *d_count still holds the full count: reallocate and
 * scan again. n must be < 2^32 (PFAC_ETOO_LARGE otherwise). The first call on a stream
 * allocates that stream's scratch (counters, tile states); later calls reuse it, and a
 * call whose text needs more scratch first waits for the stream, then grows it.
 * Concurrent calls on the same stream from different host threads are not supported.
 * Errors: PFAC_EINVAL (automaton or d_count NULL, d_text NULL with n > 0, d_keys NULL
 * with cap > 0), PFAC_ETOO_LARGE, PFAC_ENODEVICE, PFAC_ENOMEM, PFAC_EHIP. */
PFAC_API int pfac_scan_async(pfac_automaton *a, const uint8_t *d_text, uint64_t n,
                             uint64_t *d_keys, uint64_t cap, uint64_t *d_count, void *stream);

/* pfac_scan_noalloc -- pfac_scan_async for callers that cannot allocate memory (code
 * under stream capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and the same keys and count, but the call allocates nothing. Its scratch (per
 * span counts and match records) is one fixed array of about 8.1 MiB per device, held
 * from the library's first use of that device until the process ends. Limits and rules:
 *   - the automaton must already be on the current device (pfac_upload, or any earlier
 *     scan there): PFAC_EINVAL otherwise, since the upload allocates;
 *   - the text may take at most 4,096 spans: 256 MiB when the span length is left to
 *     the library (it is then lengthened as needed, up to 64 KiB), 4,096 times a tuned
 *     span length otherwise; PFAC_ETOO_LARGE beyond;
 *   - every call on one device shares that device's array: calls that overlap in time on
 *     one device (on different streams, or from different threads or automata) race
 *     and give wrong results; order them on one stream or wait in between;
 *   - a span keeps at most 256 match records (pfac_scan_async keeps up to span / 64);
 *     a span with more matching starts is walked again during placement, still exact.
 * d_keys, cap, d_count and stream as pfac_scan_async. Errors: PFAC_EINVAL (as
 * pfac_scan_async, or no device copy), PFAC_ETOO_LARGE, PFAC_ENODEVICE, PFAC_EHIP. */
PFAC_API int pfac_scan_noalloc(pfac_automaton *a, const uint8_t *d_text, uint64_t n, uint64_t *d_keys,
                               uint64_t cap, uint64_t *d_count, void *stream);

/* pfac_scan -- pfac_scan_async, then wait for `stream` and return the count in *h_count
 * (host memory). Returns PFAC_ECAPACITY when the count exceeds cap (*h_count = the
 * capacity needed; d_keys content unspecified). */
PFAC_API int pfac_scan(pfac_automaton *a, const uint8_t *d_text, uint64_t n, uint64_t *d_keys,
                       uint64_t cap, uint64_t *h_count, void *stream);

/* ------------------------------------------------------------------- host texts
 * pfac_scan_host -- scan n bytes of host memory (texts of any length, also past 2^32).
 * The text goes to the device in chunks of chunk_bytes (0 = 64 MiB), each sent with the
 * next (longest pattern - 1) bytes so that matches crossing a chunk end are found (the
 * overlap rule of Section 2.2), and each chunk keeps only matches that start inside it.
 * Two chunks are in flight at once on two library-owned streams: the copy of one
 * overlaps the scan of the other. A text in pinned memory (hipHostMalloc) is copied
 * straight from the caller's buffer; pageable text is staged through pinned buffers.
 * Runs on the current device and returns when done.
 *   out   receives a library-allocated array of matches sorted by (start, pattern_id),
 *         starts as 64-bit text offsets; free it with pfac_matches_free. On error
 *         out->matches is NULL and out->count 0.
 * Errors: PFAC_EINVAL (NULL out or automaton, NULL text with n > 0), PFAC_ETOO_LARGE
 * (chunk_bytes + longest pattern >= 2^32), PFAC_ENODEVICE, PFAC_ENOMEM, PFAC_EHIP. */
typedef struct {
    uint64_t start;
    uint32_t pattern_id;
    uint32_t reserved; /* 0 */
} pfac_match;

typedef struct {
    pfac_match *matches;
    uint64_t count;
} pfac_matches;

PFAC_API int pfac_scan_host(pfac_automaton *a, const uint8_t *h_text, uint64_t n, uint64_t chunk_bytes,
                            pfac_matches *out);

/* Free the array of a pfac_matches (and zero it). NULL is a no-op. */
PFAC_API void pfac_matches_free(pfac_matches *m);

/* pfac_prefix_histogram -- prefix depths of a text (device memory, n bytes): for every
 * start s, the number of symbols a failure-less walk from s consumes before a transition
 * is missing (Section 2.3), i.e. the length of the longest pattern prefix spelled at s,
 * capped at cap. Writes hist[d] = number of starts of depth d for d < cap and hist[cap] =
 * starts of depth cap or more (device memory, cap + 1 uint64 entries, zeroed by the
 * call). A trie truncated after k levels (Section 2.4) passes exactly the starts of depth
 * >= k; Section 4.2 studies how large k must be for an alphabet before those are only the
 * real matches. Stream-ordered like pfac_scan_async. Errors: PFAC_EINVAL (NULL
 * arguments, cap outside 1..63), PFAC_ENODEVICE, PFAC_ENOMEM, PFAC_EHIP. */
PFAC_API int pfac_prefix_histogram(pfac_automaton *a, const uint8_t *d_text, uint64_t n, uint32_t cap,
                                   uint64_t *d_hist, void *stream);

/* ------------------------------------------------------------------- packet batches
 * pfac_scan_batch_async -- scan a batch of packets held back to back in device memory
 * (CSR): packet i is d_bytes[d_offsets[i] .. d_offsets[i+1]), with d_offsets[0] = 0,
 * non-decreasing, d_offsets[n_pkts] = n_bytes (device memory, n_pkts + 1 entries; empty
 * packets are allowed). Each packet is its own text in the sense of Section 2.2: a walk
 * stops at its packet's end, so no match crosses a packet boundary. Keys use the global
 * byte offset as the start, so key order is (packet, start in packet, pattern id); map a
 * start back to its packet by an upper bound over the offsets. Offsets that break the
 * rules above give unspecified matches but no access outside d_bytes[0 .. n_bytes).
 * All packets go through one pair of persistent launches (count, then placement), not
 * one launch per packet. Count, capacity, scratch and errors as pfac_scan_async; the
 * automaton's PFAC_ALGO_PLAIN choice does not apply to batches. n_pkts == 0 gives 0. */
PFAC_API int pfac_scan_batch_async(pfac_automaton *a, const uint8_t *d_bytes, const uint64_t *d_offsets,
                                   uint32_t n_pkts, uint64_t n_bytes, uint64_t *d_keys, uint64_t cap,
                                   uint64_t *d_count, void *stream);

/* pfac_scan_batch -- pfac_scan_batch_async, then wait and return the count in *h_count,
 * with PFAC_ECAPACITY as in pfac_scan. */
PFAC_API int pfac_scan_batch(pfac_automaton *a, const uint8_t *d_bytes, const uint64_t *d_offsets,
                             uint32_t n_pkts, uint64_t n_bytes, uint64_t *d_keys, uint64_t cap,
                             uint64_t *h_count, void *stream);

/* ------------------------------------------------------------------- captured graphs
 * pfac_graph_create -- record one scan (a text when d_offsets is NULL, else a packet
 * batch) into a HIP graph that is replayed with pfac_graph_launch. The buffers are fixed
 * at creation; the sizes of each replay are read at run time from d_sizes (device memory,
 * two uint64: bytes, packets), bounded by max_bytes / max_pkts, so one graph serves
 * every batch up to those bounds: the caller writes new bytes, offsets and sizes into
 * the same buffers (stream-ordered) and launches again. d_offsets, when given, holds
 * max_pkts + 1 entries. The graph owns its scratch (allocated here, before capture),
 * uses no memset nodes, and resets its own device counters at the end of every replay.
 * `stream` is used for the capture and must not be the NULL stream. Keys, count and
 * capacity as pfac_scan_async. Errors: PFAC_EINVAL (NULL pointers, max_bytes == 0,
 * max_pkts == 0 with offsets, automaton without patterns), PFAC_ETOO_LARGE
 * (max_bytes >= 2^32), PFAC_ENODEVICE, PFAC_ENOMEM, PFAC_EHIP (capture failed). On
 * error *out is NULL. Free with pfac_graph_destroy after the last replay completed. */
typedef struct pfac_graph pfac_graph;

PFAC_API int pfac_graph_create(pfac_automaton *a, const uint8_t *d_bytes, const uint64_t *d_offsets,
                               uint64_t max_bytes, uint32_t max_pkts, uint64_t *d_keys, uint64_t cap,
                               uint64_t *d_count, const uint64_t *d_sizes, void *stream, pfac_graph **out);

/* Replay the graph on `stream` (any stream of the graph's device). Replays of one graph
 * share its scratch, so they must not run concurrently (keep them on one stream).
 * Errors: PFAC_EINVAL, PFAC_EHIP. */
PFAC_API int pfac_graph_launch(pfac_graph *g, void *stream);

/* Free the graph and its scratch. NULL is a no-op. */
PFAC_API void pfac_graph_destroy(pfac_graph *g);

/* ------------------------------------------------------------------- serving loop
 * A server keeps the automaton resident on the current device and scans packet requests
 * as they arrive (continuous batching). Requests wait in a FIFO; the server owns `slots`
 * batch slots, each with its own host thread, device buffers, stream and captured scan
 * graph (or, with PFAC_SERVER_EAGER, its own scan scratch sized for a full batch).
 * Whenever a slot is free, its thread packs every waiting request that fits
 * (max_batch_bytes / max_batch_packets) into one batch and launches it at once, so
 * requests that arrive while other batches run on the GPU are admitted as slots free up,
 * and the batches of different slots overlap on the device. Each packet is scanned as
 * its own text (as in pfac_scan_batch), so a request's result does not depend on what
 * it was batched with.
 *
 * Admission by device memory: at creation the server computes the device memory one
 * slot needs (batch buffers, key buffer, scan scratch) and keeps only as many slots as
 * device_memory_budget holds (0 = a quarter of the device's free memory); fewer than
 * one slot is PFAC_ENOMEM. Waiting requests are bounded by max_pending_bytes: a submit
 * beyond it returns PFAC_EBUSY. Fields left 0 take the defaults shown. */
typedef struct {
    uint32_t slots;               /* batches in flight at once (4)                       */
    uint32_t max_batch_packets;   /* packets per batch, and per request (16,384)         */
    uint64_t max_batch_bytes;     /* bytes per batch, and per request (8 MiB; < 2^32)    */
    uint64_t key_capacity;        /* keys a slot returns without a rescan (65,536)       */
    uint64_t max_pending_bytes;   /* bytes allowed to wait for a slot (1 GiB)            */
    uint64_t device_memory_budget;/* device bytes all slots may hold (0 = free / 4)      */
    uint32_t flags;               /* PFAC_SERVER_EAGER: each batch is enqueued as its own
                                     launch pair (pfac_scan_batch_async) instead of a
                                     replay of the slot's captured graph; same results  */
    uint32_t reserved[3];
} pfac_server_config;

#define PFAC_SERVER_EAGER 1u

/* One finished request. keys: (offset of the match start within the request's bytes
 * << 32) | pattern_id, sorted; map a start to its packet with the request's offsets.
 * Times are CLOCK_MONOTONIC nanoseconds: arrival (as submitted), launch of its batch,
 * completion seen by the server. status != PFAC_OK means the request was not scanned
 * (keys NULL). Free keys with pfac_result_free. */
typedef struct {
    uint64_t ticket;
    int32_t status;
    uint32_t n_pkts;
    uint64_t n_bytes;
    uint64_t n_matches;
    uint64_t *keys;
    uint64_t arrival_ns, launch_ns, done_ns;
} pfac_result;

typedef struct {
    uint64_t requests, packets, bytes, matches; /* completed since the last reset          */
    uint64_t batches, rejected, pending_requests;
    uint32_t slots, reserved0;
    double bytes_per_s;       /* completed bytes / (last completion - first arrival)        */
    double mean_batch_bytes;
    uint64_t p50_ns, p99_ns, max_ns; /* per-packet latency: completion - arrival, each
                                        request counted once per packet                 */
} pfac_server_stats_t;

typedef struct pfac_server pfac_server;

/* Create a server for automaton a (which must have patterns and outlive the server) on
 * the current device; cfg may be NULL. Errors: PFAC_EINVAL, PFAC_ENODEVICE, PFAC_ENOMEM
 * (budget below one slot, or allocation), PFAC_EHIP. */
PFAC_API int pfac_server_create(pfac_automaton *a, const pfac_server_config *cfg, pfac_server **out);

/* The configuration in force (defaults filled in, slots as admitted). */
PFAC_API int pfac_server_config_get(const pfac_server *s, pfac_server_config *out);

/* Submit one request: n_pkts packets, packet i = h_bytes[h_offsets[i] .. h_offsets[i+1])
 * (host memory, copied before return; h_offsets[0] = 0, non-decreasing). arrival_ns: its
 * arrival time on CLOCK_MONOTONIC (0 = now). *ticket identifies its result. Thread safe.
 * Errors: PFAC_EINVAL, PFAC_ETOO_LARGE (over a batch's limits), PFAC_EBUSY (queue full),
 * PFAC_ENOMEM, or the error that stopped the server. */
PFAC_API int pfac_server_submit(pfac_server *s, const uint8_t *h_bytes, const uint64_t *h_offsets,
                                uint32_t n_pkts, uint64_t arrival_ns, uint64_t *ticket);

/* Move up to max_results finished requests (completion order) into res; waits up to
 * timeout_us microseconds when none is ready. *n_out = number returned. */
PFAC_API int pfac_server_poll(pfac_server *s, pfac_result *res, uint32_t max_results, uint32_t *n_out,
                              uint32_t timeout_us);

/* Free a result's keys. */
PFAC_API void pfac_result_free(pfac_result *r);

/* Counters and latency percentiles; reset != 0 clears them after reading. */
PFAC_API int pfac_server_stats(pfac_server *s, pfac_server_stats_t *st, int reset);

/* Finish every submitted request, stop the worker and free the server. Results not yet
 * polled are freed. NULL is a no-op. */
PFAC_API void pfac_server_destroy(pfac_server *s);

/* ------------------------------------------------------------------- tuning
 * Launch choices of an automaton's scans. None of them changes any result (positions
 * per thread are a free parameter of the method, Section 2.3).
 *   algo        PFAC_ALGO_AUTO (= TILED), PFAC_ALGO_PLAIN (one lane per start, trie walked
 *               from the root in HBM, count pass + emit pass: the design of Section 2.3
 *               as printed, kept as a baseline; single texts only), PFAC_ALGO_TILED
 *               (persistent count kernel with the LDS prefilter and root image, then the
 *               placement kernel).
 *   grid        workgroups of the count kernel (0 = as many as are resident at once;
 *               at most 2^24 - 1).
 *   span_log2   log2 of the bytes one wave scans as a unit (its chunk): 11..16; 0 = per
 *               scan, the longest span (4..64 KiB) that still gives every resident wave
 *               one. Smaller spans spread small texts over more waves; a span keeps up to
 *               max(256, span / 64) match records in per-stream scratch.
 *   root_depth  trie levels folded into the LDS root image (1..min(shortest pattern, 2),
 *               or ..8 for alphabets <= 4); 0 = the builder's choice.
 *   filter_k    symbols per LDS prefilter key (root_depth..min(longest pattern, 4), or ..16
 *               for alphabets <= 4); 0 = the builder's choice for the root depth.
 *   lane_bytes  positions per thread: the consecutive start positions (text bytes) each
 *               lane of a wave takes per step, 16 (one 16-byte load) or 32 (two; 0 = 32).
 *               The sampled prefilter form (bytes, no pattern shorter than 4) always takes
 *               32, and pfac_get_tuning then reports 32. Results do not depend on it.
 * pfac_set_tuning with a new root_depth or filter_k rebuilds the LDS image and uploads it
 * to every device holding a copy; scans already queued and graphs already captured keep
 * the image and tuning they were launched or recorded with (old images are freed by
 * pfac_destroy). Calls that change the tuning must not race with scans of the same
 * automaton from other host threads. pfac_get_tuning reports the values in force
 * (root_depth and filter_k as built, never 0). Errors: PFAC_EINVAL (a field out of
 * range; the previous tuning stays), PFAC_ENOMEM, PFAC_EHIP. */
#define PFAC_ALGO_AUTO 0u
#define PFAC_ALGO_PLAIN 1u
#define PFAC_ALGO_TILED 2u
typedef struct {
    uint32_t algo;
    uint32_t grid;
    uint32_t span_log2;
    uint32_t root_depth;
    uint32_t filter_k;
    uint32_t lane_bytes;
    uint32_t reserved[2];
} pfac_tuning;

PFAC_API int pfac_set_tuning(pfac_automaton *a, const pfac_tuning *t);
PFAC_API int pfac_get_tuning(const pfac_automaton *a, pfac_tuning *t);

/* pfac_tune -- measure the tiled scan on a sample workload already in device memory (a
 * text when d_offsets is NULL, else a packet batch as in pfac_scan_batch) and keep the
 * fastest tuning: coordinate descent over span_log2, then root_depth, then filter_k, then
 * lane_bytes, then grid, each point timed with HIP events over `reps` scans (0 = 5) after
 * one warm-up, on `stream`. Every point must reproduce the match count and an
 * order-sensitive digest of the keys of the first scan, else PFAC_EINTERNAL. The tuner allocates its own key buffer (freed on return) and may grow
 * the stream's scratch. On success the automaton keeps the best point, *out receives it
 * (as pfac_get_tuning) and *out_ms (if not NULL) its mean milliseconds per scan; on error
 * the previous tuning is restored. No other host thread may scan with this automaton
 * while it runs. */
PFAC_API int pfac_tune(pfac_automaton *a, const uint8_t *d_bytes, uint64_t n_bytes, const uint64_t *d_offsets,
                       uint32_t n_pkts, uint32_t reps, void *stream, pfac_tuning *out, float *out_ms);

#ifdef __cplusplus
}
#endif

#endif /* PFAC_H */
